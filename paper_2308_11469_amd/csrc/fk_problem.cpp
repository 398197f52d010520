// fk_problem.cpp -- host-side problem setup (see fk_problem.hpp).
#include "fk_problem.hpp"

#include "fk_internal.hpp"

#include <cmath>
#include <algorithm>
#include <cstring>
#include <sstream>
#include <utility>

namespace fkh {

static thread_local std::string g_last_error;

void set_error(const std::string &msg) { g_last_error = msg; }
const char *last_error_cstr() { return g_last_error.c_str(); }

fk_status fail(fk_status st, const std::string &msg)
{
    set_error(msg);
    return st;
}

fk_status hip_fail(hipError_t e, const char *what)
{
    std::ostringstream os;
    os << what << ": " << hipGetErrorName(e) << " (" << hipGetErrorString(e) << ")";
    set_error(os.str());
    return e == hipErrorOutOfMemory ? FK_ENOMEM : FK_EDEVICE;
}

int path_kernel_blocks(int waves_per_cu)
{
    int dev = 0, n_cu = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&n_cu, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || n_cu <= 0)
        n_cu = 256;
    const int w = waves_per_cu > 0 ? waves_per_cu : 16;
    const int b = n_cu * w / 4;
    return b > 0 ? b : 1;
}

double lambda1_bounding_rect(const fk_domain &d)
{
    const double a = d.x1 - d.x0, b = d.y1 - d.y0;
    return M_PI * M_PI * (1.0 / (a * a) + 1.0 / (b * b));
}

int32_t auto_paths_per_item(int64_t n_interior, int64_t M)
{
    // Lanes stream across items, so items can be small; 256 paths (four per
    // lane) keep the queue fine-grained without many fetches.  Each item ends
    // with a flush of its node sums (device-scope 64-bit atomics, performed
    // beyond the per-XCD L2), so an instance with many paths takes items of up
    // to 1024 paths while it keeps at least 65536 items (16 per resident wave
    // of the default launch).  Fewer than 256 when an instance has too few
    // paths in total to fill a few thousand items.
    int64_t p = 256;
    while (p < 1024 && n_interior * ((M + 2 * p - 1) / (2 * p)) >= 65536) p *= 2;
    while (p > 64 && n_interior * ((M + p - 1) / p) < 4096) p /= 2;
    const int64_t mcap = ((M + 63) / 64) * 64;
    if (p > mcap) p = mcap;
    return (int32_t)p;
}

// Guided item sizes for the automatic choice: the first paths of every node
// go in large items (a whole number of small ones, at most three quarters of
// M), the rest in items of the automatic size.  The queue hands out all the
// large items first, so the end of the launch still balances at the small
// size while most of the work takes a fraction of the queue fetches and of
// the node-sum flushes (device-scope atomics, performed beyond the per-XCD
// L2).  The large items are as large as possible while every resident wave of
// the default launch (4096) still gets three.  Measured: the 129 x 129 source
// cavity writes 10.6 MB per launch instead of 34.6 (FP64), the 65 x 65 cavity
// 4.3 MB instead of 11.6 (FP32), at unchanged path-steps/s.
static constexpr int64_t kGuidedMinLargeItems = 3 * 4096;

static void guided_split(HostProblem &P, int64_t nint)
{
    P.ppi_a = P.items_a = 0;
    const int64_t M = P.par.M, b = P.ppi;
    const int64_t a_max = (3 * M / 4) / b * b;   // paths in large items, at most
    for (int64_t f = a_max / b; f >= 2; --f) {   // a large item = f small ones
        const int64_t per = a_max / (f * b);
        if (nint * per >= kGuidedMinLargeItems) {
            P.ppi_a = (int32_t)(f * b);
            P.items_a = (int32_t)per;
            break;
        }
    }
    const int64_t rest = M - (int64_t)P.items_a * P.ppi_a;
    P.items_per_node = (int32_t)((rest + P.ppi - 1) / P.ppi);
    P.n_items = nint * (P.items_a + P.items_per_node);
}

static bool finite_all(std::initializer_list<double> v)
{
    for (double x : v)
        if (!std::isfinite(x)) return false;
    return true;
}

static fk_status check_bc(const fk_bc &b, bool inner, bool reflecting_edge)
{
    if (b.kind < FK_BC_ZERO || b.kind > FK_BC_PLANE_WAVE_ROBIN) return fail(FK_EINVAL, "unknown boundary datum kind");
    if (b.kind == FK_BC_TABLE) {
        if (inner) return fail(FK_EINVAL, "TABLE datum is only allowed on the outer boundary");
        if (!b.table || b.table_len < 2) return fail(FK_EINVAL, "TABLE datum needs table_len >= 2 samples");
    }
    if (b.kind == FK_BC_PLANE_WAVE_ROBIN && (inner || !reflecting_edge))
        return fail(FK_EINVAL, "PLANE_WAVE_ROBIN is a Robin datum: only for a reflecting edge");
    for (double c : b.c)
        if (!std::isfinite(c)) return fail(FK_EINVAL, "boundary datum coefficients must be finite");
    return FK_OK;
}

// kappa = sqrt(k^2 + i p), the principal root (k when p = 0)
static void kappa_of(const fk_params &par, double &kr, double &ki)
{
    kr = par.k;
    ki = 0.0;
    if (par.damping != 0.0) {
        const double k2 = par.k * par.k;
        const double mod = std::sqrt(k2 * k2 + par.damping * par.damping);
        kr = std::sqrt(0.5 * (mod + k2));
        ki = par.damping / (2.0 * kr);
    }
}

// g at a boundary point on the host (FP64): the grid's boundary values.
static void host_bc(const HostProblem &P, const fk_bc &B, double x, double y, double &gr, double &gi)
{
    const fk_domain &d = P.dom;
    switch (B.kind) {
    case FK_BC_PLANE_WAVE: {
        // amp exp(i kappa s): the damped plane wave when p != 0
        double kr, ki;
        kappa_of(P.par, kr, ki);
        const double sd = x * std::cos(B.c[2]) + y * std::sin(B.c[2]);
        const double ph = kr * sd, decay = std::exp(-ki * sd);
        const double c = std::cos(ph) * decay, s = std::sin(ph) * decay;
        gr = B.c[0] * c - B.c[1] * s;
        gi = B.c[0] * s + B.c[1] * c;
        return;
    }
    case FK_BC_BILINEAR:
        gr = B.c[0] + B.c[2] * x + B.c[4] * y + B.c[6] * x * y;
        gi = B.c[1] + B.c[3] * x + B.c[5] * y + B.c[7] * x * y;
        return;
    case FK_BC_TABLE: {
        const double a = d.x1 - d.x0, b = d.y1 - d.y0;
        double s;
        if (y == d.y0) s = x - d.x0;
        else if (x == d.x1) s = a + (y - d.y0);
        else if (y == d.y1) s = a + b + (d.x1 - x);
        else s = 2.0 * a + b + (d.y1 - y);
        const int64_t L = (int64_t)P.table.size() / 2;
        const double u = s / (2.0 * (a + b)) * (double)L;
        const double fl = std::floor(u), w = u - fl;
        int64_t i0 = (int64_t)fl % L;
        if (i0 < 0) i0 += L;
        const int64_t i1 = (i0 + 1) % L;
        gr = (1.0 - w) * P.table[2 * i0] + w * P.table[2 * i1];
        gi = (1.0 - w) * P.table[2 * i0 + 1] + w * P.table[2 * i1 + 1];
        return;
    }
    default:
        gr = gi = 0.0;
    }
}

// Disc domains: each grid node outside the disc (class 3) is paired with its
// nearest unknown node (ties: the lowest node id), whose value it carries in
// the iterate.  Only unknown nodes with a 4-neighbour that is not unknown can
// be nearest: from any other unknown node u, the neighbour one grid step
// towards the exterior node is unknown and strictly nearer.  So each
// exterior node is compared with that frontier (a few times the grid's side
// in size), in increasing node order.  Distances are formed in separate
// statements, so no step is fused into a multiply-add.
static void exterior_pairs(HostProblem &P)
{
    const fk_domain &d = P.dom;
    const double sx = (d.x1 - d.x0) / (double)(d.nx - 1), sy = (d.y1 - d.y0) / (double)(d.ny - 1);
    auto coord = [](double o, double st, int32_t i) {
        const double t = (double)i * st;
        return o + t;
    };
    auto unknown = [&](int32_t i, int32_t j) { return P.cls[(size_t)i + (size_t)d.nx * j] == 0; };
    std::vector<int32_t> front;
    for (int32_t j = 0; j < d.ny; ++j)
        for (int32_t i = 0; i < d.nx; ++i) {
            if (!unknown(i, j)) continue;
            if ((i > 0 && !unknown(i - 1, j)) || (i + 1 < d.nx && !unknown(i + 1, j)) ||
                (j > 0 && !unknown(i, j - 1)) || (j + 1 < d.ny && !unknown(i, j + 1)))
                front.push_back(i + d.nx * j);
        }
    std::vector<double> fx(front.size()), fy(front.size());
    for (size_t k = 0; k < front.size(); ++k) {
        fx[k] = coord(d.x0, sx, front[k] % d.nx);
        fy[k] = coord(d.y0, sy, front[k] / d.nx);
    }
    P.ext.clear();
    for (int32_t je = 0; je < d.ny; ++je)
        for (int32_t ie = 0; ie < d.nx; ++ie) {
            const int32_t e = ie + d.nx * je;
            if (P.cls[(size_t)e] != 3) continue;
            const double xe = coord(d.x0, sx, ie), ye = coord(d.y0, sy, je);
            double best = INFINITY;
            int32_t arg = -1;
            for (size_t k = 0; k < front.size(); ++k) {
                const double ex = fx[k] - xe;
                const double ey = fy[k] - ye;
                const double ex2 = ex * ex;
                const double ey2 = ey * ey;
                const double d2 = ex2 + ey2;
                if (d2 < best) {   // the frontier is in increasing id order: ties keep the lowest
                    best = d2;
                    arg = front[k];
                }
            }
            P.ext.push_back(e);
            P.ext.push_back(arg);
        }
}

fk_status setup_problem(const fk_domain *domain, const fk_source *f, const fk_bc *g_outer, const fk_bc *g_inner,
                        const fk_params *params, HostProblem &P, bool single_instance)
{
    if (!domain || !params) return fail(FK_EINVAL, "domain and params are required");
    P.dom = *domain;
    P.par = *params;
    if (f) P.src = *f;
    else std::memset(&P.src, 0, sizeof(P.src));
    if (g_outer) P.outer = *g_outer;
    else std::memset(&P.outer, 0, sizeof(P.outer));
    if (g_inner) P.inner = *g_inner;
    else std::memset(&P.inner, 0, sizeof(P.inner));
    const fk_domain &d = P.dom;
    if (d.kind < FK_DOMAIN_RECT || d.kind > FK_DOMAIN_DISC_MINUS_DISC) return fail(FK_EINVAL, "unknown domain kind");
    const bool disc_dom = P.disc_domain();
    if (d.edge != FK_EDGE_ABSORBING && d.edge != FK_EDGE_REFLECTING)
        return fail(FK_EINVAL, "edge must be FK_EDGE_ABSORBING or FK_EDGE_REFLECTING");
    if (!finite_all({d.x0, d.x1, d.y0, d.y1}) || !(d.x1 > d.x0) || !(d.y1 > d.y0))
        return fail(FK_EINVAL, "rectangle needs finite x0 < x1 and y0 < y1");
    if (d.nx < 3 || d.ny < 3) return fail(FK_EINVAL, "nx and ny must be at least 3");
    if ((int64_t)d.nx * d.ny > (int64_t)1 << 26) return fail(FK_EINVAL, "grid too large (nx*ny > 2^26)");
    // cell offsets are formed with 24-bit integer products
    if (d.nx > (1 << 19) || d.ny >= (1 << 24)) return fail(FK_EINVAL, "nx must be <= 2^19 and ny < 2^24");
    if (d.kind == FK_DOMAIN_RECT_MINUS_DISC) {
        if (!finite_all({d.cx, d.cy, d.r}) || !(d.r > 0.0))
            return fail(FK_EINVAL, "disc needs a finite centre and r > 0");
        if (!(d.cx - d.r > d.x0 && d.cx + d.r < d.x1 && d.cy - d.r > d.y0 && d.cy + d.r < d.y1))
            return fail(FK_EINVAL, "disc must lie strictly inside the rectangle");
    }
    if (d.kind == FK_DOMAIN_RECT_MINUS_BOX) {
        if (!finite_all({d.cx, d.cy, d.r, d.ry}) || !(d.r > 0.0) || !(d.ry > 0.0))
            return fail(FK_EINVAL, "box hole needs a finite centre and half-sides r, ry > 0");
        if (!(d.cx - d.r > d.x0 && d.cx + d.r < d.x1 && d.cy - d.ry > d.y0 && d.cy + d.ry < d.y1))
            return fail(FK_EINVAL, "box must lie strictly inside the rectangle");
    }
    if (disc_dom) {
        const double side = d.x1 - d.x0;
        if (!(std::fabs(side - (d.y1 - d.y0)) <= 1e-12 * side))
            return fail(FK_EINVAL, "a disc domain needs a square box (the disc is inscribed in it)");
        if (d.edge != FK_EDGE_REFLECTING) return fail(FK_EINVAL, "a disc domain's edge must reflect");
        const double ocx = 0.5 * (d.x0 + d.x1), ocy = 0.5 * (d.y0 + d.y1), R = 0.5 * side;
        const bool rh = d.kind == FK_DOMAIN_DISC_MINUS_RHOMBUS;
        if (!finite_all({d.cx, d.cy, d.r}) || !(d.r > 0.0) || (rh && !(d.ry > 0.0 && std::isfinite(d.ry))))
            return fail(FK_EINVAL, "the hole needs a finite centre and r > 0 (and ry > 0 for the rhombus)");
        // the hole strictly inside the disc: its farthest point nearer than R
        const double far = rh ? std::fmax(std::hypot(std::fabs(d.cx - ocx) + d.r, d.cy - ocy),
                                          std::hypot(d.cx - ocx, std::fabs(d.cy - ocy) + d.ry))
                              : std::hypot(d.cx - ocx, d.cy - ocy) + d.r;
        if (!(far < R)) return fail(FK_EINVAL, "the hole must lie strictly inside the disc");
        // a step is shorter than 8.2 sqrt(2 h): one radial mirror lands inside
        if (!(side > 12.0 * std::sqrt(2.0 * params->h)))
            return fail(FK_EINVAL, "a disc domain needs a diameter longer than 12 sqrt(2 h)");
    }
    const bool reflecting = d.edge == FK_EDGE_REFLECTING;
    if (reflecting) {
        if (d.kind == FK_DOMAIN_RECT)
            return fail(FK_EINVAL, "a reflecting edge needs a hole (the paths are absorbed only there)");
        if (params->max_steps <= 0) return fail(FK_EINVAL, "a reflecting edge needs an explicit max_steps");
        if (params->g_unprojected) return fail(FK_EINVAL, "g_unprojected is not defined with a reflecting edge");
        // the largest normal step is sqrt(-2 ln 2^-24) sqrt(2h) < 5.8 sqrt(2h):
        // one mirror per coordinate brings any step back into the rectangle
        const double smax = 6.0 * std::sqrt(2.0 * params->h);
        if (!(d.x1 - d.x0 > smax && d.y1 - d.y0 > smax))
            return fail(FK_EINVAL, "a reflecting edge needs sides longer than 6 sqrt(2 h)");
    }
    if (P.src.kind < FK_SRC_ZERO || P.src.kind > FK_SRC_GAUSSIAN) return fail(FK_EINVAL, "unknown source kind");
    if (!finite_all({P.src.amp_re, P.src.amp_im, P.src.cx, P.src.cy}))
        return fail(FK_EINVAL, "source parameters must be finite");
    if (P.src.kind == FK_SRC_GAUSSIAN && !(P.src.sigma > 0.0 && std::isfinite(P.src.sigma)))
        return fail(FK_EINVAL, "Gaussian source needs sigma > 0");
    fk_status st;
    if ((st = check_bc(P.outer, false, reflecting)) != FK_OK) return st;
    if ((st = check_bc(P.inner, true, reflecting)) != FK_OK) return st;
    const fk_params &p = P.par;
    if (!std::isfinite(p.k) || p.k < 0.0) return fail(FK_EINVAL, "k must be finite and >= 0");
    if (!std::isfinite(p.h) || !(p.h > 0.0)) return fail(FK_EINVAL, "h must be > 0");
    if (p.M < 2 || p.M > (1ll << 20)) return fail(FK_EINVAL, "M must be in [2, 2^20]");
    if (p.precision != 32 && p.precision != 64) return fail(FK_EINVAL, "precision must be 32 or 64");
    if (p.max_steps < 0) return fail(FK_EINVAL, "max_steps must be >= 0");
    if (p.waves_per_cu < 0 || p.waves_per_cu > 32 || p.waves_per_cu % 4 != 0)
        return fail(FK_EINVAL, "waves_per_cu must be 0 or a multiple of 4 in [4, 32]");
    if (p.reserved != 0) return fail(FK_EINVAL, "fk_params.reserved must be 0");
    if (!std::isfinite(p.alpha) || (p.alpha != 0.0 && p.alpha < p.k * p.k))
        return fail(FK_EINVAL, "alpha must be 0 (meaning k^2) or >= k^2");
    if (!std::isfinite(p.damping) || p.damping < 0.0) return fail(FK_EINVAL, "damping must be finite and >= 0");
    if (p.gather_layout < FK_GATHER_AUTO || p.gather_layout > FK_GATHER_CELLS)
        return fail(FK_EINVAL, "gather_layout must be FK_GATHER_AUTO, _NODES or _CELLS");
    if (p.paths_per_item < 0 || p.paths_per_item % 64 != 0)
        return fail(FK_EINVAL, "paths_per_item must be 0 or a positive multiple of 64");
    if (p.max_iters < 0) return fail(FK_EINVAL, "max_iters must be >= 0");

    P.jmax = p.max_steps > 0 ? p.max_steps : (int64_t)std::ceil(40.0 / (lambda1_bounding_rect(d) * p.h));
    if (P.jmax < 1 || P.jmax > ((int64_t)1 << 31) - 4) return fail(FK_EINVAL, "step cap out of range (h too small)");

    if (P.outer.kind == FK_BC_TABLE) P.table.assign(P.outer.table, P.outer.table + 2 * P.outer.table_len);

    // node classes and the boundary values of the grid
    const double dx = (d.x1 - d.x0) / (double)(d.nx - 1), dy = (d.y1 - d.y0) / (double)(d.ny - 1);
    const size_t nn = P.n_nodes();
    P.cls.assign(nn, 0);
    P.grid0.assign(2 * nn, 0.0);
    P.interior.clear();
    // a node within 1e-9 grid steps of the box counts as in it
    const double tx = 1e-9 * dx, ty = 1e-9 * dy;
    for (int32_t j = 0; j < d.ny; ++j) {
        for (int32_t i = 0; i < d.nx; ++i) {
            const size_t id = (size_t)i + (size_t)d.nx * j;
            const double x = d.x0 + (double)i * dx, y = d.y0 + (double)j * dy;
            uint8_t c = 0;
            if (d.kind == FK_DOMAIN_RECT_MINUS_DISC || d.kind == FK_DOMAIN_DISC_MINUS_DISC) {
                const double ex = x - d.cx, ey = y - d.cy;
                if (ex * ex + ey * ey <= d.r * d.r) c = 2;
            } else if (d.kind == FK_DOMAIN_DISC_MINUS_RHOMBUS) {
                if (std::fabs(x - d.cx) / d.r + std::fabs(y - d.cy) / d.ry <= 1.0 + 1e-9) c = 2;
            } else if (d.kind == FK_DOMAIN_RECT_MINUS_BOX) {
                if (x >= d.cx - d.r - tx && x <= d.cx + d.r + tx && y >= d.cy - d.ry - ty && y <= d.cy + d.ry + ty)
                    c = 2;
            }
            if (c == 0 && !reflecting && (i == 0 || j == 0 || i == d.nx - 1 || j == d.ny - 1)) c = 1;
            if (c == 0 && disc_dom) {
                // outside the closed disc: exterior, no unknown, value 0
                const double R = 0.5 * (d.x1 - d.x0);
                const double ex = x - 0.5 * (d.x0 + d.x1), ey = y - 0.5 * (d.y0 + d.y1);
                if (ex * ex + ey * ey > R * R * (1.0 + 1e-12)) c = 3;
            }
            P.cls[id] = c;
            if (c == 0) P.interior.push_back((int32_t)id);
            else if (c != 3) host_bc(P, c == 2 ? P.inner : P.outer, x, y, P.grid0[2 * id], P.grid0[2 * id + 1]);
        }
    }
    if (disc_dom) {
        if (P.interior.empty()) return fail(FK_EINVAL, "the disc domain has no unknown grid node");
        exterior_pairs(P);
    }
    // Work order: nodes with the longest expected paths first, so that the
    // last items of a launch have short paths and the lanes drain quickly at
    // the end.  The proxy is the harmonic combination of the 1-D exit times
    // (x - x0)(x1 - x)/2, (y - y0)(y1 - y)/2 and, with a hole, d_c L/2 for the
    // distance d_c to the hole; with a reflecting edge (no exit there) the
    // distance to the hole alone.  The order does not change any result: node
    // sums are exact and independent of which path ran when.
    {
        std::vector<std::pair<double, int32_t>> key;
        key.reserve(P.interior.size());
        const double L = 0.5 * ((d.x1 - d.x0) + (d.y1 - d.y0));
        for (int32_t id : P.interior) {
            const double x = d.x0 + (double)(id % d.nx) * dx, y = d.y0 + (double)(id / d.nx) * dy;
            double dc = 0.0;
            if (d.kind == FK_DOMAIN_DISC_MINUS_RHOMBUS) {
                dc = std::fmax(std::fabs(x - d.cx) / d.r + std::fabs(y - d.cy) / d.ry - 1.0, 0.0) * std::fmin(d.r, d.ry);
            } else if (d.kind == FK_DOMAIN_RECT_MINUS_DISC || d.kind == FK_DOMAIN_DISC_MINUS_DISC) {
                dc = std::sqrt((x - d.cx) * (x - d.cx) + (y - d.cy) * (y - d.cy)) - d.r;
            } else if (d.kind == FK_DOMAIN_RECT_MINUS_BOX) {
                const double ox = std::fmax(std::fabs(x - d.cx) - d.r, 0.0);
                const double oy = std::fmax(std::fabs(y - d.cy) - d.ry, 0.0);
                dc = std::hypot(ox, oy);
            }
            double k;
            if (reflecting) {
                k = dc;
            } else {
                double inv = 2.0 / ((x - d.x0) * (d.x1 - x)) + 2.0 / ((y - d.y0) * (d.y1 - y));
                if (d.kind != FK_DOMAIN_RECT) inv += 2.0 / (dc * L);
                k = 1.0 / inv;
            }
            key.emplace_back(k, id);
        }
        std::stable_sort(key.begin(), key.end(),
                         [](const std::pair<double, int32_t> &a, const std::pair<double, int32_t> &b) {
                             return a.first > b.first;
                         });
        for (size_t i = 0; i < key.size(); ++i) P.interior[i] = key[i].second;
    }
    // The row-major FP32 copy is read as two 16-byte pieces of two rows per
    // step: cheap while the whole grid stays in the 32 KiB vector L1 cache.
    // Above that nearly every read misses to L2, and the cell-major copy
    // halves the L2 requests per step.
    const size_t node_bytes = p.precision == 32 ? 8 : 16;
    // a single FP32 instance whose row-major copy fits LDS reads it from
    // there (no L2 requests for the gather at all)
    const bool lds_fit = single_instance && p.precision == 32 && !reflecting &&
                         P.n_nodes() * node_bytes <= kLdsGridBytes;
    if (p.gather_layout == FK_GATHER_CELLS) P.cells = 1;
    else if (p.gather_layout == FK_GATHER_NODES) P.cells = 0;
    else P.cells = (P.n_nodes() * node_bytes > kL1GatherBytes && !lds_fit) ? 1 : 0;
    P.lds_grid = (lds_fit && !P.cells) ? 1 : 0;
    if (P.cells && P.n_cells() * 4 * node_bytes >= ((size_t)1 << 31))
        return fail(FK_EINVAL, "grid too large for the cell-major copy (2 GiB); use FK_GATHER_NODES");
    const int64_t nint = (int64_t)P.interior.size();
    if (p.paths_per_item > 0) {
        // the caller's item size, uniform
        P.ppi = p.paths_per_item;
        P.ppi_a = P.items_a = 0;
        P.items_per_node = (int32_t)((p.M + P.ppi - 1) / P.ppi);
        P.n_items = nint * P.items_per_node;
    } else {
        P.ppi = auto_paths_per_item(nint, p.M);
        guided_split(P, nint);
        if (reflecting) {
            // reflected paths are long (about 1400 steps on the annulus) and
            // the tail phase is off: uniform items kept the end of the launch
            // 1% shorter there
            P.ppi_a = P.items_a = 0;
            P.items_per_node = (int32_t)((p.M + P.ppi - 1) / P.ppi);
            P.n_items = nint * P.items_per_node;
        }
    }
    return FK_OK;
}

static size_t align256(size_t b) { return (b + 255) & ~(size_t)255; }

size_t instance_bytes(const HostProblem &P)
{
    const size_t nn = P.n_nodes();
    size_t b = 0;
    b += align256(nn * sizeof(double2));                 // u64
    b += align256(P.gather_bytes());                     // gather copy
    b += align256(P.interior.size() * sizeof(int32_t));  // nodes
    b += align256(P.interior.size() * sizeof(fkd::Slot));
    b += align256(nn * sizeof(double2));                 // se
    b += 2 * align256(nn * sizeof(int64_t));             // sum_j, capped
    b += align256(P.table.size() * sizeof(double));      // table
    b += align256(sizeof(fkd::DevState));
    b += align256(P.ext.size() * sizeof(int32_t));       // exterior pairs
    return b;
}

InstanceBuffers carve(const HostProblem &P, char *base)
{
    const size_t nn = P.n_nodes();
    InstanceBuffers B{};
    size_t o = 0;
    auto take = [&](size_t bytes) {
        char *p = base + o;
        o += align256(bytes);
        return p;
    };
    B.u64 = (double2 *)take(nn * sizeof(double2));
    B.gather = take(P.gather_bytes());
    B.nodes = (int32_t *)take(P.interior.size() * sizeof(int32_t));
    B.slots = (fkd::Slot *)take(P.interior.size() * sizeof(fkd::Slot));
    B.se = (double2 *)take(nn * sizeof(double2));
    B.sum_j = (int64_t *)take(nn * sizeof(int64_t));
    B.capped = (int64_t *)take(nn * sizeof(int64_t));
    B.table = (double2 *)take(P.table.size() * sizeof(double));
    B.state = (fkd::DevState *)take(sizeof(fkd::DevState));
    B.ext = (int32_t *)take(P.ext.size() * sizeof(int32_t));
    return B;
}

static void fill_bc(fkd::BCDev &dst, const fk_bc &src, const double2 *table, int64_t len, const fk_params &par)
{
    std::memset(&dst, 0, sizeof(dst));
    dst.kind = src.kind;
    if (src.kind == FK_BC_PLANE_WAVE || src.kind == FK_BC_PLANE_WAVE_ROBIN) {
        dst.c[0] = src.c[0];
        dst.c[1] = src.c[1];
        dst.c[2] = std::cos(src.c[2]);
        dst.c[3] = std::sin(src.c[2]);
        // wavenumber kappa = sqrt(k^2 + i p) (principal root; k when p = 0)
        double kr, ki;
        kappa_of(par, kr, ki);
        dst.c[4] = kr;
        dst.c[5] = ki;
    } else if (src.kind == FK_BC_BILINEAR) {
        for (int i = 0; i < 8; ++i) dst.c[i] = src.c[i];
    } else if (src.kind == FK_BC_TABLE) {
        dst.table = table;
        dst.len = len;
    }
}

fkd::Inst make_inst(const HostProblem &P, const InstanceBuffers &B)
{
    fkd::Inst D;
    std::memset(&D, 0, sizeof(D));
    const fk_domain &d = P.dom;
    D.x0 = d.x0; D.x1 = d.x1; D.y0 = d.y0; D.y1 = d.y1;
    D.dx = (d.x1 - d.x0) / (double)(d.nx - 1);
    D.dy = (d.y1 - d.y0) / (double)(d.ny - 1);
    D.idx = 1.0 / D.dx;
    D.idy = 1.0 / D.dy;
    D.cx = d.cx; D.cy = d.cy; D.r = d.r; D.r2 = d.r * d.r;
    D.bx0 = d.cx - d.r; D.bx1 = d.cx + d.r; D.by0 = d.cy - d.ry; D.by1 = d.cy + d.ry;
    // binary32 edges rounded outward: largest float <= x0, smallest float >= x1
    auto rd = [](double v) { float f = (float)v; return (double)f > v ? std::nextafter(f, -INFINITY) : f; };
    auto ru = [](double v) { float f = (float)v; return (double)f < v ? std::nextafter(f, INFINITY) : f; };
    D.x0_rd = rd(d.x0); D.x1_ru = ru(d.x1); D.y0_rd = rd(d.y0); D.y1_ru = ru(d.y1);
    // box: x >= bx0 exactly iff x >= RU(bx0) for a binary32 x, x <= bx1 iff x <= RD(bx1)
    D.bx0_ru = ru(D.bx0); D.bx1_rd = rd(D.bx1); D.by0_ru = ru(D.by0); D.by1_rd = rd(D.by1);
    // reflection: x < x0 exactly iff x < RU(x0), x > x1 iff x > RD(x1)
    D.x0_ri = ru(d.x0); D.x1_ri = rd(d.x1); D.y0_ri = ru(d.y0); D.y1_ri = rd(d.y1);
    D.nx = d.nx; D.ny = d.ny;
    D.hole = (d.kind == FK_DOMAIN_RECT_MINUS_DISC || d.kind == FK_DOMAIN_DISC_MINUS_DISC) ? fkd::HOLE_DISC
           : d.kind == FK_DOMAIN_RECT_MINUS_BOX ? fkd::HOLE_BOX
           : d.kind == FK_DOMAIN_DISC_MINUS_RHOMBUS ? fkd::HOLE_RHOMBUS : fkd::HOLE_NONE;
    D.reflect = P.reflect() ? 1 : 0;
    D.curved = P.disc_domain() ? 1 : 0;
    D.ry = d.ry;
    D.ocx = 0.5 * (d.x0 + d.x1);
    D.ocy = 0.5 * (d.y0 + d.y1);
    D.orad = 0.5 * (d.x1 - d.x0);
    D.orad2 = D.orad * D.orad;
    D.n_interior = (int32_t)P.interior.size();
    D.src_kind = P.src.kind;
    D.g_unproj = P.par.g_unprojected ? 1 : 0;
    D.src_re = P.src.amp_re; D.src_im = P.src.amp_im;
    D.src_cx = P.src.cx; D.src_cy = P.src.cy;
    D.src_c = P.src.kind == FK_SRC_GAUSSIAN ? 1.0 / (2.0 * P.src.sigma * P.src.sigma) : 0.0;
    fill_bc(D.outer, P.outer, B.table, (int64_t)P.table.size() / 2, P.par);
    fill_bc(D.inner, P.inner, nullptr, 0, P.par);
    D.k = P.par.k;
    D.k2 = P.par.k * P.par.k;
    D.alpha = P.alpha();
    D.damp = P.par.damping;
    D.q = std::exp(-(D.alpha - D.k2) * P.par.h);
    D.h = P.par.h;
    D.ih = 1.0 / P.par.h;
    D.sigma = std::sqrt(2.0 * P.par.h);
    D.M = P.par.M;
    D.jmax = P.jmax;
    D.key0 = (uint32_t)(P.par.seed & 0xFFFFFFFFull);
    D.key1 = (uint32_t)(P.par.seed >> 32);
    D.crn = P.par.crn ? 1 : 0;
    D.ppi = P.ppi;
    D.items_per_node = P.items_per_node;
    D.ppi_a = P.ppi_a;
    D.items_a = P.items_a;
    D.n_items_a = (int64_t)P.interior.size() * P.items_a;
    D.cells = P.cells;
    D.n_items = P.n_items;
    D.nodes = B.nodes;
    D.u64 = B.u64;
    D.gather = B.gather;
    D.prec = P.par.precision;
    D.slots = B.slots;
    D.se = B.se;
    D.node_sum_j = B.sum_j;
    D.node_capped = B.capped;
    D.state = B.state;
    D.ext = B.ext;
    D.n_ext = (int32_t)(P.ext.size() / 2);
    return D;
}

void gather_copy(const HostProblem &P, const double *grid, std::vector<uint8_t> &out)
{
    out.assign(P.gather_bytes(), 0);
    if (out.empty()) return;
    const size_t nx = (size_t)P.dom.nx, ny = (size_t)P.dom.ny;
    const bool f32 = P.par.precision == 32;
    auto put = [&](size_t at, size_t node) {   // at: complex slot index in out
        if (f32) {
            float *f = (float *)out.data();
            f[2 * at] = (float)grid[2 * node];
            f[2 * at + 1] = (float)grid[2 * node + 1];
        } else {
            double *d = (double *)out.data();
            d[2 * at] = grid[2 * node];
            d[2 * at + 1] = grid[2 * node + 1];
        }
    };
    if (!P.cells) {
        for (size_t i = 0; i < nx * ny; ++i) put(i, i);
        return;
    }
    // cell (p, q): corners u(p,q), u(p+1,q), u(p,q+1), u(p+1,q+1)
    size_t at = 0;
    for (size_t q = 0; q + 1 < ny; ++q)
        for (size_t p = 0; p + 1 < nx; ++p) {
            put(at++, p + nx * q);
            put(at++, p + 1 + nx * q);
            put(at++, p + nx * (q + 1));
            put(at++, p + 1 + nx * (q + 1));
        }
}

fk_status upload_instance(const HostProblem &P, const InstanceBuffers &B, hipStream_t s)
{
    const size_t nn = P.n_nodes();
    std::vector<uint8_t> g;
    gather_copy(P, P.grid0.data(), g);
    FK_HIP(hipMemcpyAsync(B.u64, P.grid0.data(), nn * sizeof(double2), hipMemcpyHostToDevice, s));
    if (!g.empty()) FK_HIP(hipMemcpyAsync(B.gather, g.data(), g.size(), hipMemcpyHostToDevice, s));
    FK_HIP(hipMemcpyAsync(B.nodes, P.interior.data(), P.interior.size() * sizeof(int32_t), hipMemcpyHostToDevice, s));
    if (!P.table.empty())
        FK_HIP(hipMemcpyAsync(B.table, P.table.data(), P.table.size() * sizeof(double), hipMemcpyHostToDevice, s));
    if (!P.ext.empty())
        FK_HIP(hipMemcpyAsync(B.ext, P.ext.data(), P.ext.size() * sizeof(int32_t), hipMemcpyHostToDevice, s));
    std::vector<double> zeros(2 * nn, 0.0);
    std::vector<int64_t> zi(nn, 0);
    std::vector<fkd::Slot> zs(P.interior.size());
    std::memset(zs.data(), 0, zs.size() * sizeof(fkd::Slot));
    if (!zs.empty())
        FK_HIP(hipMemcpyAsync(B.slots, zs.data(), zs.size() * sizeof(fkd::Slot), hipMemcpyHostToDevice, s));
    FK_HIP(hipMemcpyAsync(B.se, zeros.data(), nn * sizeof(double2), hipMemcpyHostToDevice, s));
    FK_HIP(hipMemcpyAsync(B.sum_j, zi.data(), nn * sizeof(int64_t), hipMemcpyHostToDevice, s));
    FK_HIP(hipMemcpyAsync(B.capped, zi.data(), nn * sizeof(int64_t), hipMemcpyHostToDevice, s));
    fkd::DevState st;
    std::memset(&st, 0, sizeof(st));
    FK_HIP(hipMemcpyAsync(B.state, &st, sizeof(st), hipMemcpyHostToDevice, s));
    // the staging vectors go out of scope: wait for the copies
    FK_HIP(hipStreamSynchronize(s));
    return FK_OK;
}

fk_status plan_pdd(const HostProblem &P, const int32_t *cuts_x, int32_t n_cuts_x, const int32_t *cuts_y,
                   int32_t n_cuts_y, PddPlan &out)
{
    const fk_domain &d = P.dom;
    if (P.reflect()) return fail(FK_EINVAL, "PDD needs an absorbing edge");
    if (n_cuts_x < 0 || n_cuts_y < 0 || n_cuts_x + n_cuts_y == 0 || (n_cuts_x > 0 && !cuts_x) ||
        (n_cuts_y > 0 && !cuts_y))
        return fail(FK_EINVAL, "at least one cut line");
    std::vector<int32_t> xs{0}, ys{0};
    for (int32_t i = 0; i < n_cuts_x; ++i) xs.push_back(cuts_x[i]);
    for (int32_t i = 0; i < n_cuts_y; ++i) ys.push_back(cuts_y[i]);
    xs.push_back(d.nx - 1);
    ys.push_back(d.ny - 1);
    for (auto *v : {&xs, &ys})
        for (size_t i = 1; i < v->size(); ++i)
            if ((*v)[i] <= (*v)[i - 1]) return fail(FK_EINVAL, "cuts must increase strictly within [1, n - 2]");
    PddPlan plan;
    std::vector<int32_t> offset(fkd::kPddMaxSide + 1, -1);
    auto table_of = [&](int m) {
        if (offset[m] < 0) {
            offset[m] = (int32_t)plan.tables.size();
            const double sc = std::sqrt(2.0 / (double)(m + 1));
            for (int t = 0; t < 2 * (m + 1); ++t)
                plan.tables.push_back(sc * std::sin(M_PI * (double)t / (double)(m + 1)));
            for (int q = 0; q < m; ++q) {
                const double sn = std::sin(M_PI * (double)(q + 1) / (2.0 * (double)(m + 1)));
                plan.tables.push_back(4.0 * sn * sn);
            }
        }
        return offset[m];
    };
    // a block with a hole node in it or on its frame holds part of the
    // hole's boundary: not a rectangle's Dirichlet problem, so its unknown
    // nodes keep the Feynman-Kac estimator (they join the interface)
    std::vector<uint8_t> to_mc(P.n_nodes(), 0);
    for (size_t b = 0; b + 1 < ys.size(); ++b)
        for (size_t a = 0; a + 1 < xs.size(); ++a) {
            PddPlan::Block B;
            B.i0 = xs[a] + 1;
            B.i1 = xs[a + 1];
            B.j0 = ys[b] + 1;
            B.j1 = ys[b + 1];
            if (B.i1 <= B.i0 || B.j1 <= B.j0) continue;   // adjacent cut lines: no block between
            bool clear = true;
            for (int32_t j = B.j0 - 1; j <= B.j1 && clear; ++j)
                for (int32_t i = B.i0 - 1; i <= B.i1; ++i)
                    if (P.cls[(size_t)j * d.nx + i] == 2) {
                        clear = false;
                        break;
                    }
            if (!clear) {
                for (int32_t j = B.j0; j < B.j1; ++j)
                    for (int32_t i = B.i0; i < B.i1; ++i) to_mc[(size_t)j * d.nx + i] = 1;
                continue;
            }
            const int mx = B.i1 - B.i0, my = B.j1 - B.j0;
            if (mx > fkd::kPddMaxSide || my > fkd::kPddMaxSide)
                return fail(FK_EINVAL, "a block between cut lines is wider than 64 nodes; cut finer");
            B.tx = table_of(mx);
            B.ty = table_of(my);
            plan.max_nodes = std::max(plan.max_nodes, mx * my);
            plan.blocks.push_back(B);
        }
    // the node list becomes the interface and the nodes of blocks touching
    // the hole (in the same longest-first order)
    std::vector<uint8_t> on_x(d.nx, 0), on_y(d.ny, 0);
    for (int32_t i = 0; i < n_cuts_x; ++i) on_x[cuts_x[i]] = 1;
    for (int32_t i = 0; i < n_cuts_y; ++i) on_y[cuts_y[i]] = 1;
    for (int32_t id : P.interior)
        if (on_x[id % d.nx] || on_y[id / d.nx] || to_mc[id]) plan.iface.push_back(id);
    out = std::move(plan);
    return FK_OK;
}

void apply_pdd(HostProblem &P, const PddPlan &plan, int64_t target_items)
{
    P.interior = plan.iface;
    if (P.par.paths_per_item == 0) {
        // far fewer nodes than the grid: smaller items, so that the launch's
        // waves still find work
        int64_t ppi = 64;
        while (ppi * 2 <= P.ppi) ppi *= 2;
        while (ppi > 64 && (int64_t)plan.iface.size() * ((P.par.M + ppi - 1) / ppi) < target_items) ppi /= 2;
        P.ppi = (int32_t)ppi;
        P.items_per_node = (int32_t)((P.par.M + ppi - 1) / ppi);
    }
    // uniform items over the interface nodes
    P.ppi_a = P.items_a = 0;
    P.n_items = (int64_t)plan.iface.size() * P.items_per_node;
}

fk_status load_iterate(const HostProblem &P, const InstanceBuffers &B, const double *u_reim, int32_t n,
                       bool on_device, hipStream_t s)
{
    const size_t nn = P.n_nodes();
    std::vector<double> full(2 * nn);
    if (on_device) {
        FK_HIP(hipMemcpyAsync(full.data(), u_reim, nn * sizeof(double2), hipMemcpyDeviceToHost, s));
        FK_HIP(hipStreamSynchronize(s));
    } else {
        std::memcpy(full.data(), u_reim, nn * sizeof(double2));
    }
    // boundary and hole nodes keep their data; exterior nodes carry their
    // nearest unknown node's value
    for (size_t i = 0; i < nn; ++i)
        if (P.cls[i] != 0) {
            full[2 * i] = P.grid0[2 * i];
            full[2 * i + 1] = P.grid0[2 * i + 1];
        }
    for (size_t e = 0; e < P.ext.size(); e += 2) {
        full[2 * (size_t)P.ext[e]] = full[2 * (size_t)P.ext[e + 1]];
        full[2 * (size_t)P.ext[e] + 1] = full[2 * (size_t)P.ext[e + 1] + 1];
    }
    std::vector<uint8_t> gc;
    gather_copy(P, full.data(), gc);
    fkd::DevState st;
    std::memset(&st, 0, sizeof(st));
    st.iter = n;
    st.use_u = 1;
    FK_HIP(hipMemcpyAsync(B.u64, full.data(), nn * sizeof(double2), hipMemcpyHostToDevice, s));
    if (!gc.empty()) FK_HIP(hipMemcpyAsync(B.gather, gc.data(), gc.size(), hipMemcpyHostToDevice, s));
    FK_HIP(hipMemcpyAsync(B.state, &st, sizeof(st), hipMemcpyHostToDevice, s));
    FK_HIP(hipStreamSynchronize(s));
    return FK_OK;
}

}  // namespace fkh
