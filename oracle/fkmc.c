/*
 * fkmc.c -- FP64 CPU oracle for the Monte Carlo Feynman-Kac estimator of the
 * fixed-point Helmholtz iteration.
 *
 * TEST INFRASTRUCTURE ONLY.  This is the slow, plainly written reference the
 * HIP library is checked against.  Only the test suite, the smoke entry point
 * and the benchmark's CPU-baseline leg may load it; the product path never
 * does.  It shares no source, header, table or helper with the HIP library.
 *
 * Method (Bernal, Chen, dos Reis, "An iterative method for Helmholtz boundary
 * value problems arising in wave propagation"):
 *   - Problem: Delta u + k^2 u = f in Omega, u = g on dOmega, k real, f and g
 *     complex (Sec. 1, eq. (1.1); Sec. 2.2, eq. (2.4) with damping p = 0 and
 *     no reflecting boundary part).
 *   - With the shift alpha = k^2 (Sec. 1, eq. (1.4)) the problem becomes the
 *     fixed-point sequence  Delta u_{n+1} = f - k^2 u_n,  u_{n+1} = g on the
 *     boundary, u_0 = 0.  These are the partial sums sum_{j<=n} (v_j + i w_j)
 *     of the iteration (2.6)-(2.8), as written out in the proof of Theorem 2.2.
 *   - Each Poisson step is solved pointwise with the Feynman-Kac formula of
 *     Sec. 2.1, eq. (2.3), specialised to c = 0 and a purely absorbing
 *     boundary:  u_{n+1}(y) = E[g(Y_tau)] - E[int_0^tau (f - k^2 u_n)(Y_t) dt],
 *     with Y_t = y + sqrt(2) W_t (eq. (2.2)).
 *   - Every iterate n uses a new, independent Brownian motion (Remark 2.1);
 *     the counter of the random-number generator therefore contains n.
 *   - General shift alpha >= k^2 and damping p (Sec. 2.2, eq. (2.4) with
 *     the iteration (2.6)-(2.8) written for the partial sums U_n): the
 *     equation Delta u + (k^2 + i p) u = f becomes
 *       Delta U_{n+1} - (alpha - k^2) U_{n+1} = f - (alpha + i p) U_n,
 *     and the Feynman-Kac formula of eq. (2.3) with c = alpha - k^2 gives
 *       U_{n+1}(y) = E[e^{-c tau} g(Y_tau)]
 *                    - E[int_0^tau e^{-c s} (f - (alpha + i p) U_n)(Y_s) ds].
 *     alpha = k^2, p = 0 is the iteration above.
 *   - Reflecting outer boundary (Sec. 2.1 eqs. (2.1)-(2.3) with a Neumann
 *     part; the annular iteration of Sec. 2.3): the hole is absorbing
 *     (u = phi there), the rectangle's edge carries the Robin condition
 *     d_n u - i k u = g2.  The partial sums of the iteration of Sec. 2.3
 *     satisfy d_n U_{n+1} = i k U_n + g2 on the edge (for g2 = 0 the
 *     conditions on v_n and w_n written there), and the Feynman-Kac formula
 *     with the reflected diffusion dY = sqrt(2) dW - n dxi and its local time
 *     xi adds  + E[int_0^tau e^{-c s} (i k U_n + g2)(Y_s) dxi_s]  to U_{n+1}.
 *
 * Discretisation (the readings where the paper is silent):
 *   - Euler-Maruyama: X_0 = y, X_{t+1} = X_t + sqrt(2h) (z_x, z_y).
 *   - Normals from Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11) with
 *     key = (seed mod 2^32, seed div 2^32) and counter
 *     (floor(t/2), m, node_id, n)  (n replaced by 0 in common-random-number
 *     mode).  Increment t uses words (r0, r1) when t is even, (r2, r3) when
 *     odd.  Uniform U(r) = (2 (r >> 9) + 1) 2^-24, exactly representable in
 *     binary32 and binary64.  Box-Muller: rho = sqrt(-2 ln U(ra)),
 *     phi = 2 pi U(rb), z = rho (cos phi, sin phi).
 *   - Exit: J = first t >= 1 with X_t outside the open domain (a point on the
 *     boundary counts as outside), capped at jmax.  The boundary datum is taken
 *     at the nearest boundary point of X_J.
 *   - Integral: left-point rule over the J increments,
 *     s = e^{-c J h} g(Pi X_J) - h sum_{t<J} e^{-c t h} (f - (alpha + i p) I_h[u_n])(X_t),
 *     where I_h is bilinear interpolation of the grid of u_n.
 *   - Plane-wave data: amp exp(i kappa (x cos theta + y sin theta)) with
 *     kappa = sqrt(k^2 + i p) (principal root), the plane wave that solves
 *     the damped equation; kappa = k when p = 0.
 *   - Reflection (a reading: the paper gives no discretisation of the
 *     reflected diffusion): after each Euler step a coordinate that left the
 *     rectangle is mirrored back across the face it crossed, and the local
 *     time grows by the length of the mirror move, 2 x (overshoot); the
 *     local-time integrand (i k I_h[u_n] + g2) is taken at the foot of the
 *     move on the face (the mirrored point with that coordinate set to the
 *     face) and discounted to the end of the step.  Then the step is
 *     absorbed when the point lies in the closed hole.  Every edge node of
 *     the grid is an unknown.
 *   - Curved reflecting edge (the annular domains of Sec. 2.5 with a disc as
 *     the outer boundary; a reading, as above): the disc is the one inscribed
 *     in the square [x0, x1] x [y0, y1]; a point that left it is mirrored
 *     radially, X' = c + (R - o) (X - c) / |X - c| with the overshoot
 *     o = |X - c| - R, the local time grows by 2 o and the integrand is taken
 *     at the foot c + R (X - c) / |X - c| (outward normal (X - c) / |X - c|).
 *     The hole is a disc or a rhombus |x - cx| / r + |y - cy| / ry <= 1.
 *     Grid nodes outside the closed disc are exterior: no unknowns; the
 *     bilinear interpolant reads each of them as its nearest unknown node
 *     (the remap table, built by the caller).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

/* ---------------------------------------------------------------- types -- */

enum { ORC_RECT = 0, ORC_RECT_MINUS_DISC = 1, ORC_RECT_MINUS_BOX = 2, ORC_DISC_MINUS_RHOMBUS = 3,
       ORC_DISC_MINUS_DISC = 4 };
enum { ORC_SRC_ZERO = 0, ORC_SRC_CONST = 1, ORC_SRC_GAUSSIAN = 2 };
enum { ORC_BC_ZERO = 0, ORC_BC_PLANE_WAVE = 1, ORC_BC_BILINEAR = 2, ORC_BC_TABLE = 3,
       ORC_BC_PLANE_WAVE_ROBIN = 4 };

/* Boundary datum.  PLANE_WAVE: c = (amp_re, amp_im, theta) and
 * g = amp exp(i k (x cos theta + y sin theta)).  BILINEAR: c holds the complex
 * coefficients (c0, c1, c2, c3), g = c0 + c1 x + c2 y + c3 x y.  TABLE: samples
 * (re, im interleaved) at equal arclength steps round the rectangle,
 * counter-clockwise from (x0, y0), linearly interpolated and periodic.
 * PLANE_WAVE_ROBIN (reflecting edge only): the Robin datum
 * g2 = d_n w - i k w of the plane wave w of PLANE_WAVE, so that w itself
 * solves the Robin problem; on a reflecting edge every other kind gives g2
 * directly. */
typedef struct {
    int32_t kind;
    int32_t pad;
    double c[8];
    const double *table;
    int64_t table_len;
} orc_bc;

typedef struct {
    int32_t domain_kind;
    int32_t nx, ny;
    int32_t src_kind;
    double x0, x1, y0, y1;
    double cx, cy, r;
    double src_re, src_im, src_cx, src_cy, src_sigma;
    orc_bc outer, inner;
    double k, h;
    int64_t M;
    uint64_t seed;
    int64_t jmax;
    int32_t crn;
    int32_t g_unprojected; /* test variant: g taken at X_J itself */
    double alpha;          /* shift, >= k^2 */
    double p;              /* damping */
    double ry;             /* RECT_MINUS_BOX: the hole is [cx-r, cx+r] x [cy-ry, cy+ry] */
    int32_t reflect;       /* 1: the outer edge reflects (Robin datum outer) */
    int32_t pad2;
    const int32_t *remap;  /* disc domains: node id -> node read by the interpolant
                              (an exterior node's nearest unknown node; itself
                              otherwise); NULL: identity */
} orc_problem;

/* --------------------------------------------------------------- Philox -- */

/* One Philox4x32 round and the key schedule as defined by Salmon et al.,
 * SC'11, Sec. on the Philox family: two 32x32->64 products, the high halves
 * xor-ed with the other counter words and the key. */
void orc_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4])
{
    uint32_t c0 = ctr[0], c1 = ctr[1], c2 = ctr[2], c3 = ctr[3];
    uint32_t k0 = key[0], k1 = key[1];
    for (int round = 0; round < 10; ++round) {
        uint64_t p0 = (uint64_t)0xD2511F53u * (uint64_t)c0;
        uint64_t p1 = (uint64_t)0xCD9E8D57u * (uint64_t)c2;
        uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
        uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
        uint32_t n0 = hi1 ^ c1 ^ k0;
        uint32_t n1 = lo1;
        uint32_t n2 = hi0 ^ c3 ^ k1;
        uint32_t n3 = lo0;
        c0 = n0; c1 = n1; c2 = n2; c3 = n3;
        k0 += 0x9E3779B9u;
        k1 += 0xBB67AE85u;
    }
    out[0] = c0; out[1] = c1; out[2] = c2; out[3] = c3;
}

void orc_philox_batch(const uint32_t *ctrs, const uint32_t key[2], int64_t n, uint32_t *out)
{
    for (int64_t i = 0; i < n; ++i) orc_philox4x32_10(ctrs + 4 * i, key, out + 4 * i);
}

double orc_uniform(uint32_t r)
{
    return (2.0 * (double)(r >> 9) + 1.0) * ldexp(1.0, -24);
}

void orc_box_muller(uint32_t ra, uint32_t rb, double z[2])
{
    const double two_pi = 6.283185307179586476925286766559;
    double rho = sqrt(-2.0 * log(orc_uniform(ra)));
    double phi = two_pi * orc_uniform(rb);
    z[0] = rho * cos(phi);
    z[1] = rho * sin(phi);
}

/* ------------------------------------------------------ grid and domain -- */

static double grid_dx(const orc_problem *P) { return (P->x1 - P->x0) / (double)(P->nx - 1); }
static double grid_dy(const orc_problem *P) { return (P->y1 - P->y0) / (double)(P->ny - 1); }

void orc_node_xy(const orc_problem *P, int32_t node_id, double xy[2])
{
    int32_t i = node_id % P->nx, j = node_id / P->nx;
    xy[0] = P->x0 + (double)i * grid_dx(P);
    xy[1] = P->y0 + (double)j * grid_dy(P);
}

static int disc_domain(const orc_problem *P)
{
    return P->domain_kind == ORC_DISC_MINUS_RHOMBUS || P->domain_kind == ORC_DISC_MINUS_DISC;
}

/* The outer disc of a disc domain: inscribed in the (square) grid box. */
static void outer_disc(const orc_problem *P, double *ox, double *oy, double *R)
{
    *ox = 0.5 * (P->x0 + P->x1);
    *oy = 0.5 * (P->y0 + P->y1);
    *R = 0.5 * (P->x1 - P->x0);
}

/* The closed hole: the disc of radius r at (cx, cy), the box
 * [cx - r, cx + r] x [cy - ry, cy + ry], or the rhombus
 * |x - cx| / r + |y - cy| / ry <= 1. */
static int in_hole(const orc_problem *P, double x, double y)
{
    if (P->domain_kind == ORC_RECT_MINUS_DISC || P->domain_kind == ORC_DISC_MINUS_DISC) {
        double ex = x - P->cx, ey = y - P->cy;
        return ex * ex + ey * ey <= P->r * P->r;
    }
    if (P->domain_kind == ORC_RECT_MINUS_BOX)
        return x >= P->cx - P->r && x <= P->cx + P->r && y >= P->cy - P->ry && y <= P->cy + P->ry;
    if (P->domain_kind == ORC_DISC_MINUS_RHOMBUS) {
        /* |x - cx| / r + |y - cy| / ry <= 1, multiplied through by r ry > 0 */
        const double a = fabs(x - P->cx) * P->ry, b = fabs(y - P->cy) * P->r;
        return a + b <= P->r * P->ry;
    }
    return 0;
}

/* A point outside the domain: for an absorbing edge, outside the open
 * rectangle or in the closed hole; for a reflecting edge (whose points
 * belong to the domain), in the closed hole. */
int orc_outside(const orc_problem *P, double x, double y)
{
    if (!P->reflect && (x <= P->x0 || x >= P->x1 || y <= P->y0 || y >= P->y1)) return 1;
    return in_hole(P, x, y);
}

/* A grid node in the closed hole.  For the box, nodes within 1e-9 of a
 * grid step of its edges count as on them, so that a box whose edges are
 * meant to lie on grid lines keeps its edge nodes whatever the rounding of
 * x0 + i dx. */
static int node_in_hole(const orc_problem *P, double x, double y)
{
    if (P->domain_kind == ORC_DISC_MINUS_RHOMBUS)
        return fabs(x - P->cx) / P->r + fabs(y - P->cy) / P->ry <= 1.0 + 1e-9;
    if (P->domain_kind != ORC_RECT_MINUS_BOX) return in_hole(P, x, y);
    const double ex = 1e-9 * grid_dx(P), ey = 1e-9 * grid_dy(P);
    return x >= P->cx - P->r - ex && x <= P->cx + P->r + ex && y >= P->cy - P->ry - ey
        && y <= P->cy + P->ry + ey;
}

/* 0 unknown (interior, or on a reflecting edge), 1 on an absorbing edge,
 * 2 in the closed hole, 3 outside the closed disc of a disc domain. */
int orc_node_class(const orc_problem *P, int32_t node_id)
{
    int32_t i = node_id % P->nx, j = node_id / P->nx;
    double xy[2];
    orc_node_xy(P, node_id, xy);
    if (node_in_hole(P, xy[0], xy[1])) return 2;
    if (disc_domain(P)) {
        double ox, oy, R;
        outer_disc(P, &ox, &oy, &R);
        const double ex = xy[0] - ox, ey = xy[1] - oy;
        return ex * ex + ey * ey > R * R * (1.0 + 1e-12) ? 3 : 0;
    }
    if (!P->reflect && (i == 0 || j == 0 || i == P->nx - 1 || j == P->ny - 1)) return 1;
    return 0;
}

/* Nearest point of the segment a-b to (x, y), and its squared distance. */
static double segment_project(double ax, double ay, double bx, double by, double x, double y, double p[2])
{
    const double vx = bx - ax, vy = by - ay;
    double t = ((x - ax) * vx + (y - ay) * vy) / (vx * vx + vy * vy);
    t = t < 0.0 ? 0.0 : (t > 1.0 ? 1.0 : t);
    p[0] = ax + t * vx;
    p[1] = ay + t * vy;
    return (x - p[0]) * (x - p[0]) + (y - p[1]) * (y - p[1]);
}

/* Nearest point of the hole's boundary to (x, y), and its distance. */
static double hole_project(const orc_problem *P, double x, double y, double p[2])
{
    if (P->domain_kind == ORC_DISC_MINUS_RHOMBUS) {
        /* the four sides between the vertices (cx + r, cy), (cx, cy + ry),
           (cx - r, cy), (cx, cy - ry); the first nearest wins */
        const double vx[5] = {P->cx + P->r, P->cx, P->cx - P->r, P->cx, P->cx + P->r};
        const double vy[5] = {P->cy, P->cy + P->ry, P->cy, P->cy - P->ry, P->cy};
        double best = -1.0, q[2];
        for (int e = 0; e < 4; ++e) {
            const double d2 = segment_project(vx[e], vy[e], vx[e + 1], vy[e + 1], x, y, q);
            if (best < 0.0 || d2 < best) {
                best = d2;
                p[0] = q[0];
                p[1] = q[1];
            }
        }
        return sqrt(best);
    }
    if (P->domain_kind == ORC_RECT_MINUS_DISC || P->domain_kind == ORC_DISC_MINUS_DISC) {
        double ex = x - P->cx, ey = y - P->cy;
        double d = sqrt(ex * ex + ey * ey);
        if (d > 0.0) {
            p[0] = P->cx + P->r * ex / d;
            p[1] = P->cy + P->r * ey / d;
        } else {
            p[0] = P->cx + P->r;
            p[1] = P->cy;
        }
        return fabs(d - P->r);
    }
    double bx0 = P->cx - P->r, bx1 = P->cx + P->r, by0 = P->cy - P->ry, by1 = P->cy + P->ry;
    if (in_hole(P, x, y)) {
        /* inside the box: the nearest face */
        double dd[4] = {x - bx0, bx1 - x, y - by0, by1 - y};
        int e = 0;
        for (int c = 1; c < 4; ++c)
            if (dd[c] < dd[e]) e = c;
        p[0] = e == 0 ? bx0 : (e == 1 ? bx1 : x);
        p[1] = e == 2 ? by0 : (e == 3 ? by1 : y);
        return dd[e];
    }
    p[0] = x < bx0 ? bx0 : (x > bx1 ? bx1 : x);
    p[1] = y < by0 ? by0 : (y > by1 ? by1 : y);
    return hypot(x - p[0], y - p[1]);
}

/* Nearest boundary point of X.  Outside the rectangle: clamp into it (outer
 * boundary).  In the closed disc: radial projection onto the circle.  Inside
 * the domain (only for a path stopped by the step cap): the nearest of the four
 * edges and the circle.  Returns 1 for the outer boundary, 2 for the circle. */
int orc_project(const orc_problem *P, double x, double y, double p[2])
{
    const int hole = P->domain_kind != ORC_RECT;
    if (P->reflect) {
        /* the Dirichlet part is the hole's boundary alone */
        hole_project(P, x, y, p);
        return 2;
    }
    if (x <= P->x0 || x >= P->x1 || y <= P->y0 || y >= P->y1) {
        p[0] = x < P->x0 ? P->x0 : (x > P->x1 ? P->x1 : x);
        p[1] = y < P->y0 ? P->y0 : (y > P->y1 ? P->y1 : y);
        return 1;
    }
    if (!(hole && in_hole(P, x, y))) {
        double dd[4] = {x - P->x0, P->x1 - x, y - P->y0, P->y1 - y};
        int e = 0;
        for (int c = 1; c < 4; ++c)
            if (dd[c] < dd[e]) e = c;
        double hp[2];
        if (!hole || dd[e] <= hole_project(P, x, y, hp)) {
            p[0] = e == 0 ? P->x0 : (e == 1 ? P->x1 : x);
            p[1] = e == 2 ? P->y0 : (e == 3 ? P->y1 : y);
            return 1;
        }
    }
    hole_project(P, x, y, p);
    return 2;
}

/* Arclength of a point on the rectangle edge, counter-clockwise from (x0,y0). */
static double perimeter_s(const orc_problem *P, double x, double y)
{
    double a = P->x1 - P->x0, b = P->y1 - P->y0;
    if (y == P->y0) return x - P->x0;
    if (x == P->x1) return a + (y - P->y0);
    if (y == P->y1) return a + b + (P->x1 - x);
    return 2.0 * a + b + (P->y1 - y);
}

/* kappa = sqrt(k^2 + i p): kr = sqrt((|k^2 + i p| + k^2) / 2),
 * ki = p / (2 kr); kappa = k when p = 0 */
static void kappa_of(const orc_problem *P, double *kr, double *ki)
{
    *kr = P->k;
    *ki = 0.0;
    if (P->p != 0.0) {
        const double k2 = P->k * P->k;
        const double mod = sqrt(k2 * k2 + P->p * P->p);
        *kr = sqrt(0.5 * (mod + k2));
        *ki = P->p / (2.0 * *kr);
    }
}

static void plane_wave_eval(const orc_problem *P, const orc_bc *B, double x, double y, double g[2])
{
    double kr, ki;
    kappa_of(P, &kr, &ki);
    const double sx = x * cos(B->c[2]) + y * sin(B->c[2]);
    const double ph = kr * sx, decay = exp(-ki * sx);
    double cr = cos(ph) * decay, si = sin(ph) * decay;
    g[0] = B->c[0] * cr - B->c[1] * si;
    g[1] = B->c[0] * si + B->c[1] * cr;
}

static void bc_eval(const orc_problem *P, const orc_bc *B, double x, double y, double g[2])
{
    switch (B->kind) {
    case ORC_BC_PLANE_WAVE:
        plane_wave_eval(P, B, x, y, g);
        return;
    case ORC_BC_BILINEAR:
        g[0] = B->c[0] + B->c[2] * x + B->c[4] * y + B->c[6] * x * y;
        g[1] = B->c[1] + B->c[3] * x + B->c[5] * y + B->c[7] * x * y;
        return;
    case ORC_BC_TABLE: {
        double a = P->x1 - P->x0, b = P->y1 - P->y0;
        double per = 2.0 * (a + b);
        int64_t L = B->table_len;
        double u = perimeter_s(P, x, y) / per * (double)L;
        double fl = floor(u);
        double w = u - fl;
        int64_t i0 = ((int64_t)fl % L + L) % L;
        int64_t i1 = (i0 + 1) % L;
        g[0] = (1.0 - w) * B->table[2 * i0] + w * B->table[2 * i1];
        g[1] = (1.0 - w) * B->table[2 * i0 + 1] + w * B->table[2 * i1 + 1];
        return;
    }
    default:
        g[0] = 0.0;
        g[1] = 0.0;
    }
}

/* g at a boundary point; which = 1 outer rectangle, 2 hole. */
void orc_g(const orc_problem *P, int which, double x, double y, double g[2])
{
    bc_eval(P, which == 2 ? &P->inner : &P->outer, x, y, g);
}

/* Robin datum g2 of a reflecting edge at a point of face `face` (0: x = x0,
 * 1: x = x1, 2: y = y0, 3: y = y1).  For PLANE_WAVE_ROBIN, with the plane
 * wave w = amp exp(i kappa d.x), d = (cos theta, sin theta) and the outward
 * normal n of the face: d_n w = i kappa (d.n) w, so
 * g2 = d_n w - i k w = i (kappa (d.n) - k) w. */
void orc_robin(const orc_problem *P, int face, double x, double y, double g[2])
{
    if (P->outer.kind != ORC_BC_PLANE_WAVE_ROBIN) {
        bc_eval(P, &P->outer, x, y, g);
        return;
    }
    double dn;
    if (face == 4) {
        /* the disc's edge: outward normal (x - c) / R at the foot */
        double ox, oy, R;
        outer_disc(P, &ox, &oy, &R);
        dn = ((x - ox) * cos(P->outer.c[2]) + (y - oy) * sin(P->outer.c[2])) / R;
    } else {
        dn = face == 0 ? -cos(P->outer.c[2])
           : face == 1 ? cos(P->outer.c[2])
           : face == 2 ? -sin(P->outer.c[2]) : sin(P->outer.c[2]);
    }
    double kr, ki, w[2];
    kappa_of(P, &kr, &ki);
    plane_wave_eval(P, &P->outer, x, y, w);
    /* i (kappa dn - k) = -ki dn + i (kr dn - k) */
    const double ar = -ki * dn, ai = kr * dn - P->k;
    g[0] = ar * w[0] - ai * w[1];
    g[1] = ar * w[1] + ai * w[0];
}

/* Grid values that the iterate carries on non-interior nodes for n >= 1:
 * g on an absorbing rectangle edge, the inner datum's own formula on hole
 * nodes (a reflecting edge's nodes are unknowns). */
void orc_fill_boundary(const orc_problem *P, double *u)
{
    int64_t nn = (int64_t)P->nx * P->ny;
    for (int64_t id = 0; id < nn; ++id) {
        int cls = orc_node_class(P, (int32_t)id);
        if (cls == 0 || cls == 3) continue;   /* exterior nodes are read through the remap */
        double xy[2], g[2];
        orc_node_xy(P, (int32_t)id, xy);
        orc_g(P, cls, xy[0], xy[1], g);
        u[2 * id] = g[0];
        u[2 * id + 1] = g[1];
    }
}

/* Bilinear interpolation I_h of a complex grid (re, im interleaved, node
 * (i, j) at index i + nx j) on the cell that contains (x, y). */
void orc_interp(const orc_problem *P, const double *u, double x, double y, double out[2])
{
    double fx = (x - P->x0) / grid_dx(P);
    double fy = (y - P->y0) / grid_dy(P);
    int64_t p = (int64_t)floor(fx), q = (int64_t)floor(fy);
    if (p < 0) p = 0;
    if (p > P->nx - 2) p = P->nx - 2;
    if (q < 0) q = 0;
    if (q > P->ny - 2) q = P->ny - 2;
    double a = fx - (double)p, b = fy - (double)q;
    int64_t i00 = p + (int64_t)P->nx * q, i10 = i00 + 1, i01 = i00 + P->nx, i11 = i01 + 1;
    if (P->remap) {
        i00 = P->remap[i00];
        i10 = P->remap[i10];
        i01 = P->remap[i01];
        i11 = P->remap[i11];
    }
    for (int c = 0; c < 2; ++c)
        out[c] = (1.0 - a) * (1.0 - b) * u[2 * i00 + c] + a * (1.0 - b) * u[2 * i10 + c]
               + (1.0 - a) * b * u[2 * i01 + c] + a * b * u[2 * i11 + c];
}

static void source_eval(const orc_problem *P, double x, double y, double f[2])
{
    switch (P->src_kind) {
    case ORC_SRC_CONST:
        f[0] = P->src_re;
        f[1] = P->src_im;
        return;
    case ORC_SRC_GAUSSIAN: {
        double ex = x - P->src_cx, ey = y - P->src_cy;
        double e = exp(-(ex * ex + ey * ey) / (2.0 * P->src_sigma * P->src_sigma));
        f[0] = P->src_re * e;
        f[1] = P->src_im * e;
        return;
    }
    default:
        f[0] = 0.0;
        f[1] = 0.0;
    }
}

/* ----------------------------------------------------------- one path -- */

/* Local-time integrand (i k I_h[u_n] + g2) at a foot point on face `face`
 * (u == NULL: u_n = 0). */
static void local_time_integrand(const orc_problem *P, const double *u, int face, double x, double y,
                                 double out[2])
{
    double un[2] = {0.0, 0.0}, g2[2];
    if (u) orc_interp(P, u, x, y, un);
    orc_robin(P, face, x, y, g2);
    out[0] = -P->k * un[1] + g2[0];
    out[1] = P->k * un[0] + g2[1];
}

/* Mirrors X (the point after step t) back into the rectangle across the
 * faces it crossed and adds, per crossed face, the local-time increment
 * dxi = 2 x overshoot times the discounted integrand at the foot of the
 * move to lt.  One mirror per coordinate suffices: the rectangle is wider
 * than any single step (checked at set-up). */
static void reflect_disc(const orc_problem *P, const double *u, int64_t t, double X[2], double lt[2])
{
    double ox, oy, R;
    outer_disc(P, &ox, &oy, &R);
    const double ex = X[0] - ox, ey = X[1] - oy;
    const double d2 = ex * ex + ey * ey;
    if (d2 <= R * R) return;
    const double d = sqrt(d2);
    const double o = d - R;                   /* overshoot */
    const double inv = 1.0 / d;               /* one reciprocal for both scale factors */
    const double s = (R - o) * inv, f = R * inv;
    const double footx = ox + f * ex, footy = oy + f * ey;
    X[0] = ox + s * ex;
    X[1] = oy + s * ey;
    const double w = exp(-(P->alpha - P->k * P->k) * (double)t * P->h);
    double v[2];
    local_time_integrand(P, u, 4, footx, footy, v);
    lt[0] += w * (2.0 * o) * v[0];
    lt[1] += w * (2.0 * o) * v[1];
}

static void reflect_step(const orc_problem *P, const double *u, int64_t t, double X[2], double lt[2])
{
    if (disc_domain(P)) {
        reflect_disc(P, u, t, X, lt);
        return;
    }
    double dxi_x = 0.0, dxi_y = 0.0;
    int fx = -1, fy = -1;
    if (X[0] < P->x0) {
        dxi_x = 2.0 * (P->x0 - X[0]);
        X[0] = 2.0 * P->x0 - X[0];
        fx = 0;
    } else if (X[0] > P->x1) {
        dxi_x = 2.0 * (X[0] - P->x1);
        X[0] = 2.0 * P->x1 - X[0];
        fx = 1;
    }
    if (X[1] < P->y0) {
        dxi_y = 2.0 * (P->y0 - X[1]);
        X[1] = 2.0 * P->y0 - X[1];
        fy = 2;
    } else if (X[1] > P->y1) {
        dxi_y = 2.0 * (X[1] - P->y1);
        X[1] = 2.0 * P->y1 - X[1];
        fy = 3;
    }
    if (fx < 0 && fy < 0) return;
    const double w = exp(-(P->alpha - P->k * P->k) * (double)t * P->h);
    double v[2];
    if (fx >= 0) {
        local_time_integrand(P, u, fx, fx == 0 ? P->x0 : P->x1, X[1], v);
        lt[0] += w * dxi_x * v[0];
        lt[1] += w * dxi_x * v[1];
    }
    if (fy >= 0) {
        local_time_integrand(P, u, fy, X[0], fy == 2 ? P->y0 : P->y1, v);
        lt[0] += w * dxi_y * v[0];
        lt[1] += w * dxi_y * v[1];
    }
}

/* Simulates path m from node node_id for the Poisson step that produces
 * u_{n+1} from u_n (u == NULL means u_n = 0 everywhere, the start u_0).
 * Writes the score s (re, im), the exit-step index J, whether the cap was
 * hit, and the exit point X_J. */
void orc_path(const orc_problem *P, const double *u, int32_t n, int32_t node_id, int64_t m,
              double s[2], int64_t *J_out, int32_t *capped, double xJ[2])
{
    const double sigma = sqrt(2.0 * P->h);
    const double c = P->alpha - P->k * P->k;     /* killing rate, >= 0 */
    uint32_t key[2] = {(uint32_t)(P->seed & 0xFFFFFFFFu), (uint32_t)(P->seed >> 32)};
    uint32_t ctr[4], r[4];
    double X[2];
    orc_node_xy(P, node_id, X);
    double acc[2] = {0.0, 0.0};
    double lt[2] = {0.0, 0.0};   /* local-time integral (reflecting edge) */
    int64_t t = 0;
    int exited = 0;
    for (;;) {
        if (t % 2 == 0) {
            ctr[0] = (uint32_t)(t / 2);
            ctr[1] = (uint32_t)m;
            ctr[2] = (uint32_t)node_id;
            ctr[3] = P->crn ? 0u : (uint32_t)n;
            orc_philox4x32_10(ctr, key, r);
        }
        double z[2];
        if (t % 2 == 0)
            orc_box_muller(r[0], r[1], z);
        else
            orc_box_muller(r[2], r[3], z);
        /* left-point value of e^{-c s} (f - (alpha + i p) u_n) at X_t, s = t h */
        double f[2], un[2] = {0.0, 0.0};
        source_eval(P, X[0], X[1], f);
        if (u) orc_interp(P, u, X[0], X[1], un);
        const double w = exp(-c * (double)t * P->h);
        acc[0] += w * (f[0] - (P->alpha * un[0] - P->p * un[1]));
        acc[1] += w * (f[1] - (P->alpha * un[1] + P->p * un[0]));
        X[0] = X[0] + sigma * z[0];
        X[1] = X[1] + sigma * z[1];
        t += 1;
        if (P->reflect) reflect_step(P, u, t, X, lt);
        if (orc_outside(P, X[0], X[1])) { exited = 1; break; }
        if (t >= P->jmax) break;
    }
    double g[2];
    if (P->g_unprojected) {
        /* test variant: the datum's own formula at X_J (needs a global g) */
        int outer = X[0] <= P->x0 || X[0] >= P->x1 || X[1] <= P->y0 || X[1] >= P->y1;
        orc_g(P, (outer || !exited) ? 1 : 2, X[0], X[1], g);
    } else {
        double pr[2];
        int which = orc_project(P, X[0], X[1], pr);
        orc_g(P, which, pr[0], pr[1], g);
    }
    const double wJ = exp(-c * (double)t * P->h);
    s[0] = wJ * g[0] - P->h * acc[0] + lt[0];
    s[1] = wJ * g[1] - P->h * acc[1] + lt[1];
    *J_out = t;
    *capped = exited ? 0 : 1;
    xJ[0] = X[0];
    xJ[1] = X[1];
}

/* ------------------------------------------------- node estimates -- */

/* Node statistics of one Poisson step at the listed nodes: mean score
 * (re, im), unbiased sample variance (re, im; denominator M - 1), the sum of
 * exit-step indices and the number of capped paths.  Scores are kept and
 * reduced in path order m = 0 .. M-1 (two-pass variance). */
int orc_fk_nodes(const orc_problem *P, const double *u, int32_t n, const int32_t *node_ids,
                 int64_t count, double *mean, double *var, int64_t *sumJ, int64_t *capped,
                 int32_t nthreads)
{
    const int64_t M = P->M;
    int bad = 0;
#ifdef _OPENMP
    if (nthreads > 0) omp_set_num_threads(nthreads);
#else
    (void)nthreads;
#endif
#pragma omp parallel for schedule(dynamic, 1) reduction(| : bad)
    for (int64_t c = 0; c < count; ++c) {
        double *sc = (double *)malloc((size_t)M * 2 * sizeof(double));
        if (!sc) { bad = 1; continue; }
        int64_t sj = 0, nc = 0;
        for (int64_t m = 0; m < M; ++m) {
            double s[2], xj[2];
            int64_t J;
            int32_t cap;
            orc_path(P, u, n, node_ids[c], m, s, &J, &cap, xj);
            sc[2 * m] = s[0];
            sc[2 * m + 1] = s[1];
            sj += J;
            nc += cap;
        }
        for (int comp = 0; comp < 2; ++comp) {
            double sum = 0.0;
            for (int64_t m = 0; m < M; ++m) sum += sc[2 * m + comp];
            double mu = sum / (double)M;
            double ss = 0.0;
            for (int64_t m = 0; m < M; ++m) {
                double d = sc[2 * m + comp] - mu;
                ss += d * d;
            }
            mean[2 * c + comp] = mu;
            var[2 * c + comp] = M > 1 ? ss / (double)(M - 1) : 0.0;
        }
        sumJ[c] = sj;
        capped[c] = nc;
        free(sc);
    }
    return bad;
}

int orc_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}
