// fk_device.hpp -- device-side pieces of the Feynman-Kac Helmholtz path for
// gfx950: counter-based normals, geometry, interpolation of the iterate and
// the per-wavefront work item (a chunk of paths from one grid node).
//
// Method: each Poisson step  Delta u_{n+1} = f - k^2 u_n  (Sec. 1 eq. (1.4)
// with alpha = k^2) is solved at a node y by the Feynman-Kac formula of
// Sec. 2.1 eq. (2.3) with c = 0 and a purely absorbing boundary:
//   u_{n+1}(y) = E[ g(Y_tau) - int_0^tau (f - k^2 u_n)(Y_t) dt ],
//   Y_t = y + sqrt(2) W_t,
// with a new Brownian motion for every n (Remark 2.1).
//
// Execution model: waves take work items (node, chunk of consecutive path
// indices m) from a queue; the 64 lanes of a wave run paths as one stream,
// each lane taking the next unused index when its path exits.  Every loop
// trip draws one Philox block (4 words) and takes two Euler steps.  Scores
// go into per-node slots as exact integers, so results do not depend on
// scheduling.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace fkd {

constexpr int kWave = 64;

// Optional parts of the path code.  The path kernel is compiled per set of
// features; an instance runs in any kernel whose set contains its own (the
// run-time checks stay), and a kernel without a feature carries neither its
// code nor its constants.
constexpr int kFeatDisc = 1;     // the domain has a hole (disc or box)
constexpr int kFeatSource = 2;   // f is not zero
constexpr int kFeatGeneral = 4;  // a shift alpha != k^2 or a damping p (discount, complex coefficient,
                                 // damped plane-wave data)
constexpr int kFeatReflect = 8;  // the rectangle's edge reflects (Robin condition, local time); always
                                 // with a hole
constexpr int kFeatAll = kFeatDisc | kFeatSource | kFeatGeneral | kFeatReflect;
// Not a feature: a build of the plain kernel for instances whose gather copy
// is row-major (held in the vector L1), with its own instruction order.
constexpr int kRowMajor = 16;
// Not a feature: FP32 kernels of one instance whose row-major copy is staged
// in LDS (a 1024-thread block per CU shares it).
constexpr int kLdsGrid = 32;
// The outer edge is the disc inscribed in the grid's square, reflecting
// (always with kFeatReflect and a hole); kernels of disc domains only (every
// path is mirrored radially), whose queued local-time moves carry both
// coordinates of their foot.
constexpr int kFeatCurved = 64;

enum : int32_t { BC_ZERO = 0, BC_PLANE_WAVE = 1, BC_BILINEAR = 2, BC_TABLE = 3, BC_PLANE_WAVE_ROBIN = 4 };
enum : int32_t { HOLE_NONE = 0, HOLE_DISC = 1, HOLE_BOX = 2, HOLE_RHOMBUS = 3 };
enum : int32_t { SRC_ZERO = 0, SRC_CONST = 1, SRC_GAUSSIAN = 2 };

struct BCDev {
    int32_t kind;
    int32_t pad;
    double c[8];            // PLANE_WAVE (and PLANE_WAVE_ROBIN): amp_re, amp_im, cos th, sin th,
                            // kappa_re, kappa_im; BILINEAR: c0..c3
    const double2 *table;   // TABLE samples (device)
    int64_t len;
};

// Sums of one interior node over one iteration, as exact integers (added
// with integer atomics, so their value does not depend on the order):
// s = sum over paths of the score, held as sum floor(s 2^16) (hi, two's
// complement) and sum frac(s 2^16) 2^40 (lo); s^2 likewise with scale 1.
struct Slot {
    unsigned long long s_re_hi, s_re_lo, s_im_hi, s_im_lo;
    unsigned long long q_re_hi, q_re_lo, q_im_hi, q_im_lo;
    unsigned long long sum_j;        // sum of exit-step indices
    unsigned long long capped;       // paths stopped by the step cap
    unsigned long long overflow;     // scores not representable (|s| >= 2^21 or not finite)
    unsigned long long pad;
};

// Per-instance device state written by the update kernel.
struct DevState {
    int32_t iter;          // index n of the iterate held in the grid
    int32_t use_u;         // 0 while u_n == 0 everywhere (n == 0)
    uint64_t max_du;       // bit pattern of a non-negative double (atomicMax)
    uint64_t sup;
    uint64_t max_se;
    unsigned long long path_steps;
    unsigned long long capped;
    unsigned long long nonfinite;
    // sum over nodes of min(|du|^2 / (2 |SE|^2), 4096) in units of 2^-20
    // (exact integers: independent of the order of addition), and the
    // number of nodes with a non-zero SE
    unsigned long long ratio_fx;
    unsigned long long ratio_n;
};

// Everything a work item needs about its instance (device memory, read
// through the scalar cache).
struct Inst {
    double x0, x1, y0, y1, dx, dy, idx, idy;
    double cx, cy, r, r2;
    double bx0, bx1, by0, by1;                       // box hole
    double ry;                                       // rhombus hole: |x - cx| / r + |y - cy| / ry <= 1
    double ocx, ocy, orad, orad2;                    // disc domains: the outer disc (centre, R, R^2)
    float x0_rd, x1_ru, y0_rd, y1_ru;                // edges rounded outward to binary32
    float bx0_ru, bx1_rd, by0_ru, by1_rd;            // box edges rounded inward to binary32
    float x0_ri, x1_ri, y0_ri, y1_ri;                // edges rounded inward (reflection tests)
    int32_t nx, ny, hole, n_interior;                // hole: HOLE_NONE / _DISC / _BOX
    int32_t reflect, curved;                         // 1: the outer edge reflects; 1: it is the disc
    int32_t src_kind, g_unproj;
    double src_re, src_im, src_cx, src_cy, src_c;   // src_c = 1 / (2 sigma^2)
    BCDev outer, inner;
    double k, k2, h, ih, sigma;                      // ih = 1 / h, sigma = sqrt(2 h)
    double alpha, damp, q;                           // shift, damping p, q = exp(-(alpha - k^2) h)
    int64_t M, jmax;
    uint32_t key0, key1;
    int32_t crn, ppi;                                // ppi: paths per small item
    int32_t items_per_node, cells;                   // small items per node; cells: the gather copy is cell-major
    int32_t prec, n_ext;                             // 32 or 64: the instance's stepping precision; ext pairs
    int64_t n_items;                                 // all items (large, then small)
    int64_t n_items_a;                               // large items (items_a per node, first in the queue)
    int32_t ppi_a, items_a;                          // paths per large item, large items per node
    const int32_t *nodes;                            // interior node ids
    double2 *u64;                                    // iterate, FP64 master
    void *gather;                                    // copy of u_n the paths read: FP32 row-major nodes
                                                     // or cells (FP32 path), FP64 cells (FP64 path with
                                                     // cells); unused by the FP64 row-major path
    Slot *slots;                                     // one per interior node
    double2 *se;                                     // per grid node
    int64_t *node_sum_j, *node_capped;               // per grid node
    DevState *state;
    const int32_t *ext;                              // disc domains: n_ext pairs (exterior node, the unknown
                                                     // node whose value it carries)
};

// ------------------------------------------------------------ Philox4x32-10
// Counter-based generator of Salmon, Moraes, Dror and Shaw (SC'11): ten
// rounds of two 32x32->64 products whose high halves are xor-ed into the
// other words with the round key; the key is bumped by two Weyl constants.
// a ^ b ^ k in one VALU op (gfx950 three-input bitwise op, truth table 0x96);
// k is wave-uniform (a round key) and sits in a scalar register.
__device__ __forceinline__ uint32_t xor3_uniform(uint32_t a, uint32_t b, uint32_t k)
{
    uint32_t r;
    asm("v_bitop3_b32 %0, %1, %2, %3 bitop3:0x96" : "=v"(r) : "v"(a), "v"(b), "s"(k));
    return r;
}

// k0, k1 must be wave-uniform (the instance's key).
__device__ __forceinline__ uint4 philox4x32_10(uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3,
                                               uint32_t k0, uint32_t k1)
{
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        const uint64_t p0 = (uint64_t)0xD2511F53u * c0;
        const uint64_t p1 = (uint64_t)0xCD9E8D57u * c2;
        const uint32_t n0 = xor3_uniform((uint32_t)(p1 >> 32), c1, k0);
        const uint32_t n2 = xor3_uniform((uint32_t)(p0 >> 32), c3, k1);
        c1 = (uint32_t)p1;
        c3 = (uint32_t)p0;
        c0 = n0;
        c2 = n2;
        k0 += 0x9E3779B9u;
        k1 += 0xBB67AE85u;
    }
    return make_uint4(c0, c1, c2, c3);
}

// -------------------------------------------------------------- normals
// U(r) = (2 (r >> 9) + 1) 2^-24 in (0, 1), exact in binary32 and binary64.
// Box-Muller: z = sqrt(-2 ln U(ra)) (cos 2 pi U(rb), sin 2 pi U(rb)).

// FP64.  U = j 2^-24 with j = (r >> 8) | 1 odd, 1 <= j < 2^24, so ln U and
// sincos(2 pi U) only ever see 2^23 arguments; two tables of 1024 points in
// LDS (16 KB each, built once per block by init_f64_tables) and short
// polynomials give them in far fewer operations than the general library
// functions, to about 1 ulp.
struct F64Tables {
    double2 sc[1024];   // (sin, cos)(pi i / 512)
    double2 lg[1024];   // (ln c, 1 / c) for c = (i + 512) / 1024
    double ex[64];      // 2^(i / 64): the exponential of the source term
};

// Every thread of the block calls this; the caller synchronises the block.
__device__ __forceinline__ void init_f64_tables(F64Tables &T)
{
    for (int i = threadIdx.x; i < 1024; i += blockDim.x) {
        double sn, cs;
        sincospi((double)i * 0x1p-9, &sn, &cs);
        T.sc[i] = make_double2(sn, cs);
        const double c = (double)(i + 512) * 0x1p-10;
        T.lg[i] = make_double2(log(c), 1.0 / c);
        if (i < 64) T.ex[i] = exp2((double)i * 0x1p-6);
    }
}

// e^a for a <= 0 (the Gaussian source, a = -|x - c|^2 / (2 sigma^2)) by the
// table-driven reduction of Tang (ACM TOMS 15, 1989): a = (64 m + j) ln2/64
// + r with j in [0, 64) and |r| <= ln2/128 (ln2/64 in two parts, the first
// with 35 significant bits so that n times it is exact for |n| < 2^18), then
// e^a = 2^m 2^(j/64) e^r with e^r - 1 by its Taylor series to r^5 (the next
// term is below 4e-17 relative, about a third of an ulp).  Far below the
// underflow threshold the integer conversion saturates and the scaling
// still gives 0.  Replaces the library exponential, whose wider reduction
// needs a degree-11 polynomial.
__device__ __forceinline__ double exp_nonpos(double a, const F64Tables &T)
{
    const double n = rint(a * 92.332482616893656877);     // 64 / ln 2
    const int i = (int)n;
    const double r = fma(n, 2.0164562921995537e-13, fma(n, -0.010830424696450791, a));
    double q = fma(r, 1.0 / 120.0, 1.0 / 24.0);
    q = fma(r, q, 1.0 / 6.0);
    q = fma(r, q, 0.5);
    q = fma(r, q, 1.0);
    const double t = T.ex[i & 63];
    return ldexp(fma(t, r * q, t), i >> 6);
}

// ln(j 2^-24).  j = 2^e y with y in [0x3FE55555 00000000, 0x3FF55555 00000000)
// as binary64 bit patterns (about [2/3, 4/3)): the exponent e comes from the
// high word of (double) j, offset so that the split falls at 2/3, and y is
// j with e taken out of its exponent field (exact).  y = c (1 + r) with
// c = k/1024 the table point nearest y, so |r| < 2^-11 / c < 7.4e-4 and y - c
// is exact; ln(1 + r) by its Taylor series to r^5.  The next term is below
// 3e-20, and below 2.4e-21 where |ln U| is smallest without c = 1 (c = 1023/1024,
// |ln U| > 4.8e-4): under 0.02 ulp.  Near U = 1 the table point is c = 1
// (ln c = 0, n = e - 24 = 0) and ln U is ln(1 + r) alone, without
// cancellation.  n ln 2 in two parts (Cody-Waite
// split: the high part has trailing zero bits, so n * ln2_hi is exact).
__device__ __forceinline__ double ln_uniform(uint32_t j, const F64Tables &T)
{
    const double dj = (double)j;
    const int hi = __double2hiint(dj);
    const int e = (hi - 0x3FE55555) >> 20;
    const double y = __hiloint2double(hi - (e << 20), __double2loint(dj));
    const int k = (int)(y * 1024.0 + 0.5);
    const double2 t = T.lg[k - 512];
    const double r = (y - (double)k * 0x1p-10) * t.y;
    double q = 1.0 / 5.0;
    q = fma(r, q, -0.25);
    q = fma(r, q, 1.0 / 3.0);
    q = fma(r, q, -0.5);
    const double l1p = fma(r, r * q, r);
    const double n = (double)(e - 24);
    const double ln2_hi = 6.93147180369123816490e-01, ln2_lo = 1.90821492927058770002e-10;
    return fma(n, ln2_hi, fma(n, ln2_lo, t.x + l1p));
}

// (sin, cos)(pi j 2^-23) = (sin, cos)(pi (jh 2^-9 + x/pi)) with jh = j >> 14
// from the table and x = pi (j mod 2^14) 2^-23 in [0, 0.0062): sin x to x^5
// and cos x - 1 to x^6 (next terms below 7e-20 and 6e-23), then the addition
// formulas.
__device__ __forceinline__ void sincospi_uniform(uint32_t j, const F64Tables &T, double &sn, double &cs)
{
    const double2 t = T.sc[j >> 14];
    const double x = (double)(j & 0x3FFFu) * 3.7450702829239286e-07;   // pi 2^-23
    const double x2 = x * x;
    const double s1 = fma(x * x2, fma(x2, 1.0 / 120.0, -1.0 / 6.0), x);
    const double c1 = x2 * fma(x2, fma(x2, -1.0 / 720.0, 1.0 / 24.0), -0.5);
    sn = fma(t.y, s1, fma(t.x, c1, t.x));
    cs = fma(-t.x, s1, fma(t.y, c1, t.y));
}

// sqrt(a) for a positive normal a (here a = -2 ln U in [2^-23, 33.3]):
// the hardware reciprocal square root y0, one coupled Newton step on
// g ~ sqrt(a) and h ~ 1/(2 sqrt(a)), then two residual corrections
// g += (a - g^2) h (Markstein's scheme), correctly rounded in practice.  The
// general sqrt adds range scaling for denormals and checks for 0, inf and
// NaN, which cannot occur here.
__device__ __forceinline__ double sqrt_pos(double a)
{
    const double y = __builtin_amdgcn_rsq(a);
    double g = a * y, h = 0.5 * y;
    const double r = fma(-h, g, 0.5);
    g = fma(g, r, g);
    h = fma(h, r, h);
    double d = fma(-g, g, a);
    g = fma(d, h, g);
    d = fma(-g, g, a);
    return fma(d, h, g);
}

__device__ __forceinline__ void normals(uint32_t ra, uint32_t rb, const F64Tables &T, double &zx, double &zy)
{
    const double rho = sqrt_pos(-2.0 * ln_uniform((ra >> 8) | 1u, T));
    double sn, cs;
    sincospi_uniform((rb >> 8) | 1u, T, sn, cs);
    zx = rho * cs;
    zy = rho * sn;
}

// FP32: 1 + (r >> 9) 2^-23 built from the bits, minus (1 - 2^-24), is the
// same uniform exactly.  Hardware log2, sqrt, sin and cos; the sin/cos
// instructions take their argument in revolutions, so 2 pi U needs no multiply.
// The bit pattern 0x3f800000 | (r >> 9) is the funnel shift of 127 : r right
// by 9 (one v_alignbit_b32).
__device__ __forceinline__ float unit_interval_bits(uint32_t r)
{
    return __uint_as_float(__builtin_amdgcn_alignbit(127u, r, 9u));
}

struct NoTables {};

__device__ __forceinline__ void normals(uint32_t ra, uint32_t rb, const NoTables &, float &zx, float &zy)
{
    const float ua = unit_interval_bits(ra) - 0x1.fffffep-1f;
    const float ub = unit_interval_bits(rb) - 0x1.fffffep-1f;
    const float rho = __builtin_amdgcn_sqrtf(-1.38629436111989061f * __builtin_amdgcn_logf(ua));
    zx = rho * __builtin_amdgcn_cosf(ub);
    zy = rho * __builtin_amdgcn_sinf(ub);
}

// ------------------------------------------------------------- geometry

// The closed rhombus |x - cx| / r + |y - cy| / ry <= 1, multiplied through
// by r ry > 0 (no division).  Separate statements: no product is fused into
// the sum, so every build rounds it the same way.
__device__ __forceinline__ bool in_rhombus(const Inst &D, double x, double y)
{
    const double a = fabs(x - D.cx) * D.ry;
    const double b = fabs(y - D.cy) * D.r;
    const double lim = D.r * D.ry;
    return a + b <= lim;
}

// The closed hole (FP64, the problem's own comparisons).  The rhombus only
// occurs in disc domains (kernels with kFeatCurved).
template <int F>
__device__ __forceinline__ bool in_hole(const Inst &D, double x, double y)
{
    if (D.hole == HOLE_DISC) {
        const double ex = x - D.cx, ey = y - D.cy;
        return ex * ex + ey * ey <= D.r2;
    }
    if (D.hole == HOLE_BOX) return x >= D.bx0 && x <= D.bx1 && y >= D.by0 && y <= D.by1;
    if ((F & kFeatCurved) && D.hole == HOLE_RHOMBUS) return in_rhombus(D, x, y);
    return false;
}

// Nearest point of the segment a-b to (x, y); returns the squared distance.
__device__ __forceinline__ double segment_project(double ax, double ay, double bx, double by, double x, double y,
                                                  double &px, double &py)
{
    const double vx = bx - ax, vy = by - ay;
    double t = ((x - ax) * vx + (y - ay) * vy) / (vx * vx + vy * vy);
    t = fmin(fmax(t, 0.0), 1.0);
    px = ax + t * vx;
    py = ay + t * vy;
    return (x - px) * (x - px) + (y - py) * (y - py);
}

// Nearest point of the hole's boundary and its distance.  Disc: radial
// projection.  Box: from inside, the nearest face; from outside, the clamp.
// Rhombus: the nearest of its four sides (the first one on a tie).
template <int F>
__device__ __forceinline__ double hole_project(const Inst &D, double x, double y, double &px, double &py)
{
    if ((F & kFeatCurved) && D.hole == HOLE_RHOMBUS) {
        const double vx[5] = {D.cx + D.r, D.cx, D.cx - D.r, D.cx, D.cx + D.r};
        const double vy[5] = {D.cy, D.cy + D.ry, D.cy, D.cy - D.ry, D.cy};
        double best = -1.0;
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            double qx, qy;
            const double d2 = segment_project(vx[e], vy[e], vx[e + 1], vy[e + 1], x, y, qx, qy);
            if (best < 0.0 || d2 < best) {
                best = d2;
                px = qx;
                py = qy;
            }
        }
        return sqrt(best);
    }
    if (D.hole == HOLE_DISC) {
        const double ex = x - D.cx, ey = y - D.cy;
        const double d = sqrt(ex * ex + ey * ey);
        if (d > 0.0) {
            px = D.cx + D.r * ex / d;
            py = D.cy + D.r * ey / d;
        } else {
            px = D.cx + D.r;
            py = D.cy;
        }
        return fabs(d - D.r);
    }
    if (in_hole<F>(D, x, y)) {
        double dd[4] = {x - D.bx0, D.bx1 - x, y - D.by0, D.by1 - y};
        int e = 0;
        for (int c = 1; c < 4; ++c)
            if (dd[c] < dd[e]) e = c;
        px = e == 0 ? D.bx0 : (e == 1 ? D.bx1 : x);
        py = e == 2 ? D.by0 : (e == 3 ? D.by1 : y);
        return dd[e];
    }
    px = fmin(fmax(x, D.bx0), D.bx1);
    py = fmin(fmax(y, D.by0), D.by1);
    return hypot(x - px, y - py);
}

// Nearest point of the Dirichlet boundary to X (FP64).  With a reflecting
// edge that is the hole's boundary alone.  Otherwise: outside the rectangle,
// the clamp (outer part); in the closed hole, its projection; inside the
// domain (a path stopped by the cap), the nearest of the four edges and the
// hole.  Returns 1 for the outer boundary, 2 for the hole.
template <int F>
__device__ __forceinline__ int project(const Inst &D, double x, double y, double &px, double &py)
{
    if (D.reflect) {
        hole_project<F>(D, x, y, px, py);
        return 2;
    }
    if (x <= D.x0 || x >= D.x1 || y <= D.y0 || y >= D.y1) {
        px = fmin(fmax(x, D.x0), D.x1);
        py = fmin(fmax(y, D.y0), D.y1);
        return 1;
    }
    if (!(D.hole && in_hole<F>(D, x, y))) {
        double dd[4] = {x - D.x0, D.x1 - x, y - D.y0, D.y1 - y};
        int e = 0;
        for (int c = 1; c < 4; ++c)
            if (dd[c] < dd[e]) e = c;
        double hx, hy;
        if (!D.hole || dd[e] <= hole_project<F>(D, x, y, hx, hy)) {
            px = e == 0 ? D.x0 : (e == 1 ? D.x1 : x);
            py = e == 2 ? D.y0 : (e == 3 ? D.y1 : y);
            return 1;
        }
    }
    hole_project<F>(D, x, y, px, py);
    return 2;
}

// The plane wave amp exp(i kappa s), s = x cos th + y sin th, kappa = kr + i ki.
template <int F>
__device__ __forceinline__ double2 plane_wave(const BCDev &B, double x, double y)
{
    // phase in half-turns: sincospi reduces its argument exactly
    const double sd = x * B.c[2] + y * B.c[3];
    const double ph = B.c[4] * sd;
    double s, c;
    sincospi(ph * 0.318309886183790671537767526745, &s, &c);
    if ((F & kFeatGeneral) && B.c[5] != 0.0) {
        const double decay = exp(-B.c[5] * sd);
        s *= decay;
        c *= decay;
    }
    return make_double2(B.c[0] * c - B.c[1] * s, B.c[0] * s + B.c[1] * c);
}

// Boundary datum at a point (FP64, once per path).
template <int F>
__device__ __forceinline__ double2 bc_eval(const Inst &D, const BCDev &B, double x, double y)
{
    switch (B.kind) {
    case BC_PLANE_WAVE:
        return plane_wave<F>(B, x, y);
    case BC_BILINEAR:
        return make_double2(B.c[0] + B.c[2] * x + B.c[4] * y + B.c[6] * x * y,
                            B.c[1] + B.c[3] * x + B.c[5] * y + B.c[7] * x * y);
    case BC_TABLE: {
        const double a = D.x1 - D.x0, b = D.y1 - D.y0;
        double s;
        if (y == D.y0) s = x - D.x0;
        else if (x == D.x1) s = a + (y - D.y0);
        else if (y == D.y1) s = a + b + (D.x1 - x);
        else s = 2.0 * a + b + (D.y1 - y);
        const double u = s / (2.0 * (a + b)) * (double)B.len;
        const double fl = floor(u);
        const double w = u - fl;
        int64_t i0 = (int64_t)fl % B.len;
        if (i0 < 0) i0 += B.len;
        const int64_t i1 = i0 + 1 == B.len ? 0 : i0 + 1;
        const double2 t0 = B.table[i0], t1 = B.table[i1];
        return make_double2((1.0 - w) * t0.x + w * t1.x, (1.0 - w) * t0.y + w * t1.y);
    }
    default:
        return make_double2(0.0, 0.0);
    }
}

// Robin datum g2 of a reflecting edge at a point of face `face` (0: x = x0,
// 1: x = x1, 2: y = y0, 3: y = y1).  PLANE_WAVE_ROBIN: for the plane wave w
// of direction d, d_n w = i kappa (d . n) w on a face with outward normal n,
// so g2 = d_n w - i k w = i (kappa (d . n) - k) w.  Any other kind is g2
// itself.
template <int F>
__device__ __forceinline__ double2 robin_datum(const Inst &D, int face, double x, double y)
{
    const BCDev &B = D.outer;
    if (B.kind != BC_PLANE_WAVE_ROBIN) return bc_eval<F>(D, B, x, y);
    // face 4 (kernels with kFeatCurved): the disc's edge, outward normal
    // (x - c) / R at the foot
    const double dn = ((F & kFeatCurved) && face == 4) ? ((x - D.ocx) * B.c[2] + (y - D.ocy) * B.c[3]) / D.orad
                    : (face == 0 ? -B.c[2] : (face == 1 ? B.c[2] : (face == 2 ? -B.c[3] : B.c[3])));
    const double2 w = plane_wave<F>(B, x, y);
    // i (kappa dn - k) = -ki dn + i (kr dn - k)
    const double ar = -B.c[5] * dn, ai = B.c[4] * dn - D.k;
    return make_double2(ar * w.x - ai * w.y, ar * w.y + ai * w.x);
}

// Score datum g at the end of a path whose last point is (x, y).
template <int F>
__device__ __forceinline__ double2 exit_datum(const Inst &D, double x, double y, bool exited)
{
    if (D.g_unproj && !D.reflect) {
        const bool outer = x <= D.x0 || x >= D.x1 || y <= D.y0 || y >= D.y1;
        return bc_eval<F>(D, (outer || !exited) ? D.outer : D.inner, x, y);
    }
    double px, py;
    const int which = project<F>(D, x, y, px, py);
    const BCDev *B = which == 2 ? &D.inner : &D.outer;
    return bc_eval<F>(D, *B, px, py);
}

// ------------------------------------------ iterate grid per precision

template <class R> struct Grid;
template <> struct Grid<double> {
    using C2 = double2;
    static __device__ __forceinline__ const double2 *ptr(const Inst &D)
    {
        return D.cells ? (const double2 *)D.gather : D.u64;
    }
};
template <> struct Grid<float> {
    using C2 = float2;
    static __device__ __forceinline__ const float2 *ptr(const Inst &D) { return (const float2 *)D.gather; }
};

}  // namespace fkd
