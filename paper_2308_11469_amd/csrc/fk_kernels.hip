// fk_kernels.hip -- HIP kernels of the Feynman-Kac Helmholtz path (gfx950).
//
//   fk_stream_f32 / _f64<F>   the paths: waves pull (instance, node, chunk)
//                             items from a device queue until it is empty and
//                             run their paths as one stream of lanes
//   fk_update_kernel          node mean / variance from the node slots, the
//                             fixed-point update of the iterate and the
//                             per-iteration status (max |du|, sup, max SE,
//                             path steps, capped and non-finite counts)
//   debug kernels             Philox words, normals, single paths
//
// No MFMA: nothing on this path is a dense contraction.  The stepping loop is
// bound by VALU issue (Philox integer products, transcendentals, the bilinear
// gather of u_n and the FP arithmetic of the step).
#include <type_traits>

#include "fk_device.hpp"
#include "fk_internal.hpp"

namespace fkd {

// bytes in LDS (address space 3): reads through it are ds_read instructions
typedef __attribute__((address_space(3))) const unsigned char lds_u8;

// Per-precision constants of an instance, hoisted out of the stepping loop.
// The normals' lookup tables per precision (FP64 only; they live in LDS).
template <class R> struct TablesOf { using type = F64Tables; };
template <> struct TablesOf<float> { using type = NoTables; };

// Builds the block's tables; every thread of the block must call it.
template <class R> __device__ __forceinline__ void setup_tables(typename TablesOf<R>::type &T)
{
    if constexpr (sizeof(R) == 8) init_f64_tables(T);
    __syncthreads();
}

// Everything the stepping loop reads is copied here once per instance, so the
// loop touches no instance memory.
template <class R> struct Consts {
    R x0, y0, idx, idy, sigma, k2;
    R ox, oy;               // -x0 / dx, -y0 / dy: grid coordinates as x / dx + ox
    R ex0, ex1, ey0, ey1;   // rectangle edges for the exit test (FP32: rounded outward)
    R cxf, cyf, r2f, band;
    R hx0, hx1, hy0, hy1;   // box hole for the exit test (FP32: rounded inward)
    R rx0, rx1, ry0, ry1;   // reflection thresholds (FP32: faces rounded inward)
    R lx0, lx1, ly0, ly1;   // faces as R (mirrors and the feet of mirror moves)
    R lx0l, lx1l, ly0l, ly1l;   // FP32: the faces minus their binary32 values (FP64: 0)
    R kk;                   // k (the Robin coupling i k u_n on a reflecting edge)
    double ih;              // 1 / h
    R src_re, src_im, src_cx, src_cy, src_c;
    R pmax, qmax;       // largest cell index as R (nx - 2, ny - 2): FP32 cell location
    int pmaxi, qmaxi;   // the same as integers: FP64 cell location
    int jmax;
    int hole, src_kind;
    int reflect;        // the rectangle's edge reflects
    int robin_g2;       // the Robin datum g2 is not zero
    int cells;          // the gather copy of u_n is cell-major
    double q;           // discount per step, e^{-(alpha - k^2) h}
    R alpha, damp;      // coefficient alpha + i p of the iterate
    int general;        // this instance has a shift or damping (else it
                        // takes the plain arithmetic, bit for bit)
    uint32_t key0, key1;
    const typename TablesOf<R>::type *tab;   // the block's normals tables
    // Byte offset of cell (p, q)'s first 16-byte read is p * sx + q * sy; the
    // second read is at + second.  Row-major nodes: the two reads are the
    // cell's bottom and top rows (u00 u10 | u01 u11).  Cell-major (FP32 copy
    // only): one 32-byte block per cell holding the same four corners in the
    // same order, so both layouts fill the registers identically.
    uint32_t sx, sy, second;
    __amdgpu_buffer_rsrc_t grid;   // buffer resource of the iterate grid
    const lds_u8 *lgrid;           // the row-major FP32 copy staged in LDS (kLdsGrid kernels)
    __device__ Consts(const Inst &D, const typename TablesOf<R>::type *T, const lds_u8 *L = nullptr)
        : x0((R)D.x0), y0((R)D.y0), idx((R)D.idx), idy((R)D.idy), sigma((R)D.sigma), k2((R)D.k2),
          ox((R)(-D.x0 * D.idx)), oy((R)(-D.y0 * D.idy)),
          cxf((R)D.cx), cyf((R)D.cy), r2f((R)D.r2), band((R)(1e-5 * (D.r + 1.0))),
          lx0((R)D.x0), lx1((R)D.x1), ly0((R)D.y0), ly1((R)D.y1), kk((R)D.k), ih(D.ih),
          src_re((R)D.src_re), src_im((R)D.src_im), src_cx((R)D.src_cx), src_cy((R)D.src_cy),
          src_c((R)D.src_c), pmax((R)(D.nx - 2)), qmax((R)(D.ny - 2)), pmaxi(D.nx - 2), qmaxi(D.ny - 2), jmax((int)D.jmax),
          hole(D.hole), src_kind(D.src_kind), reflect(D.reflect), robin_g2(D.outer.kind != BC_ZERO),
          cells(D.cells), q(D.q), alpha((R)D.alpha), damp((R)D.damp),
          general(D.alpha != D.k2 || D.damp != 0.0),
          key0(D.key0), key1(D.key1),
          tab(T), lgrid(L)
    {
        lx0l = (R)(D.x0 - (double)lx0);
        lx1l = (R)(D.x1 - (double)lx1);
        ly0l = (R)(D.y0 - (double)ly0);
        ly1l = (R)(D.y1 - (double)ly1);
        if (sizeof(R) == 4) {
            ex0 = (R)D.x0_rd; ex1 = (R)D.x1_ru; ey0 = (R)D.y0_rd; ey1 = (R)D.y1_ru;
            hx0 = (R)D.bx0_ru; hx1 = (R)D.bx1_rd; hy0 = (R)D.by0_ru; hy1 = (R)D.by1_rd;
            // x < x0 exactly iff x < RU(x0) for a binary32 x; x > x1 iff x > RD(x1)
            rx0 = (R)D.x0_ri; rx1 = (R)D.x1_ri; ry0 = (R)D.y0_ri; ry1 = (R)D.y1_ri;
        } else {
            ex0 = (R)D.x0; ex1 = (R)D.x1; ey0 = (R)D.y0; ey1 = (R)D.y1;
            hx0 = (R)D.bx0; hx1 = (R)D.bx1; hy0 = (R)D.by0; hy1 = (R)D.by1;
            rx0 = (R)D.x0; rx1 = (R)D.x1; ry0 = (R)D.y0; ry1 = (R)D.y1;
        }
        const uint32_t node_bytes = (uint32_t)(2 * sizeof(R));
        uint32_t bytes;
        if (cells) {
            sx = 4u * node_bytes;                 // one cell: four corners
            sy = sx * (uint32_t)(D.nx - 1);
            second = 2u * node_bytes;             // the top two corners
            bytes = sy * (uint32_t)(D.ny - 1);
        } else {
            sx = node_bytes;
            sy = node_bytes * (uint32_t)D.nx;
            second = sy;
            bytes = sy * (uint32_t)D.ny;
        }
        // raw buffer over the grid; dword 3 = 0x00020000 for gfx9-family
        grid = __builtin_amdgcn_make_buffer_rsrc((void *)Grid<R>::ptr(D), (short)0, (int)bytes, 0x00020000);
    }
};

// Path state.  The integral is held in FP64 in both precisions: the FP32 path
// adds the FP32 sum of each loop trip's (at most two) integrand values to it,
// so its rounding error does not grow with the path length.
template <class R> struct PathState {
    R x, y;       // position
    R xl, yl;     // FP32: the rounding error of the position, carried by a
                  // compensated addition at every step (x + xl is the position
                  // to far below an ulp of x); FP64: unused, 0
    double ar, ai;  // sum of the integrand over the left points
    double lr, li;  // reflecting edge: sum of the deferred local-time terms (batched
                    // evaluation), kept apart so that its value depends on the path alone
    double w;     // discount e^{-(alpha - k^2) t h} at the current point (1 without a shift)
    int t;        // steps taken
};

// exponential of the source term (argument <= 0): FP64 by the table-driven
// reduction, FP32 by the hardware base-2 exponential
__device__ __forceinline__ double exp_src(double a, const F64Tables &T) { return exp_nonpos(a, T); }
__device__ __forceinline__ float exp_src(float a, const NoTables &)
{
    return __builtin_amdgcn_exp2f(a * 1.44269504088896341f);
}

// Exit test: outside the open rectangle (unless its edge reflects), or in
// the closed hole.  FP64: the same comparisons as the problem statement.
// FP32: for a binary32 x, x <= x0 exactly iff x <= RD(x0) (x0 rounded down
// to binary32) and x >= x1 iff x >= RU(x1), so comparing with the
// outward-rounded edges equals the exact test against the FP64 edges (the
// box's edges likewise rounded inward); the disc test runs in FP32 and falls
// back to FP64 only within a thin band around the circle.
template <int F>
__device__ __forceinline__ bool is_out(const Inst &D, const Consts<double> &K, double x, double y)
{
    if (!((F & kFeatReflect) && K.reflect) && (x <= K.ex0 || x >= K.ex1 || y <= K.ey0 || y >= K.ey1))
        return true;
    if ((F & kFeatDisc) && K.hole == HOLE_DISC) {
        const double ex = x - K.cxf, ey = y - K.cyf;
        return ex * ex + ey * ey <= K.r2f;
    }
    if ((F & kFeatDisc) && K.hole == HOLE_BOX) return x >= K.hx0 && x <= K.hx1 && y >= K.hy0 && y <= K.hy1;
    if ((F & kFeatCurved) && K.hole == HOLE_RHOMBUS) return in_rhombus(D, x, y);
    return false;
}
template <int F>
__device__ __forceinline__ bool is_out(const Inst &D, const Consts<float> &K, float x, float y)
{
    if (!((F & kFeatReflect) && K.reflect) && (x <= K.ex0 || x >= K.ex1 || y <= K.ey0 || y >= K.ey1))
        return true;
    if ((F & kFeatDisc) && K.hole == HOLE_DISC) {
        const float ex = x - K.cxf, ey = y - K.cyf;
        const float d = ex * ex + ey * ey - K.r2f;
        if (d > K.band) return false;
        if (d < -K.band) return true;
        const double exd = (double)x - D.cx, eyd = (double)y - D.cy;
        return exd * exd + eyd * eyd <= D.r2;
    }
    if ((F & kFeatDisc) && K.hole == HOLE_BOX) return x >= K.hx0 && x <= K.hx1 && y >= K.hy0 && y <= K.hy1;
    // the rhombus (disc domains) in FP64, as the FP64 kernels test it
    if ((F & kFeatCurved) && K.hole == HOLE_RHOMBUS) return in_rhombus(D, (double)x, (double)y);
    return false;
}

// Reflection at the rectangle's faces (edge that reflects): a coordinate
// past a face is mirrored back across it, and the local time grows by the
// length of the mirror move, twice the overshoot.  The rectangle is wider
// than any single step (checked at set-up), so one mirror per coordinate
// lands inside.  face: 0 x = x0, 1 x = x1, 2 y = y0, 3 y = y1, -1 none.
// FP64 tests and mirrors against the faces themselves.  FP32 tests against
// the inward-rounded faces (the exact test for a binary32 point) and mirrors
// across the nearest binary32 face: forming the mirror in FP64 instead was
// measured 13% slower on the annulus (a lane-divergent branch whenever any
// lane mirrors) and changed no node by a measurable amount.
template <class R> struct Mirror {
    R lx, ly;     // local-time increments of the x and y faces
    int fx, fy;   // the faces crossed
};

template <class R>
__device__ __forceinline__ Mirror<R> reflect(const Consts<R> &K, R &x, R &y)
{
    Mirror<R> m{(R)0, (R)0, -1, -1};
    if (x < K.rx0) {
        m.lx = (R)2 * (K.lx0 - x);
        x = (R)2 * K.lx0 - x;
        m.fx = 0;
    } else if (x > K.rx1) {
        m.lx = (R)2 * (x - K.lx1);
        x = (R)2 * K.lx1 - x;
        m.fx = 1;
    }
    if (y < K.ry0) {
        m.ly = (R)2 * (K.ly0 - y);
        y = (R)2 * K.ly0 - y;
        m.fy = 2;
    } else if (y > K.ry1) {
        m.ly = (R)2 * (y - K.ly1);
        y = (R)2 * K.ly1 - y;
        m.fy = 3;
    }
    return m;
}

// The Euler step x + sigma z.  FP64: one multiply-add.  FP32, compensated:
// d = sigma z + xl (the step and the carried rounding error, one multiply-add)
// is added to x, and the exact rounding error of that sum (Fast2Sum: exact
// for |x| >= |d|; within one step of the origin its error stays below an ulp
// of d) becomes the new xl.  The position's drift over a path is then set by
// the rounding of d (an ulp of the step, not of the position): on the
// reflected paths of about 2000 steps, ~1e-8 against ~1e-6 uncompensated.
__device__ __forceinline__ void move(const Consts<double> &K, double x, double, double z, double &nx, double &nl)
{
    nx = x + K.sigma * z;
    nl = 0.0;
}
__device__ __forceinline__ void move(const Consts<float> &K, float x, float xl, float z, float &nx, float &nl)
{
    const float d = fmaf(K.sigma, z, xl);
    nx = x + d;
    nl = d - (nx - x);
}

// FP32 reflection with the compensated position: the overshoot past the
// face (x0 = lx0 + lx0l, its binary32 value and the rest) is
// o = (lx0 - x) + (lx0l - xl), exact in its leading part; the mirrored point
// is the face plus o, again as a compensated pair, and the local time grows
// by 2 o.  Same tests against the inward-rounded faces as the FP64 reflect.
__device__ __forceinline__ void mirror_lo(float face, float face_l, float o, float &x, float &xl)
{
    x = face + o;
    xl = face_l + (o - (x - face));
}
__device__ __forceinline__ Mirror<float> reflect_c(const Consts<float> &K, float &x, float &y, float &xl, float &yl)
{
    Mirror<float> m{0.0f, 0.0f, -1, -1};
    if (x < K.rx0) {
        const float o = (K.lx0 - x) + (K.lx0l - xl);
        m.lx = 2.0f * o;
        mirror_lo(K.lx0, K.lx0l, o, x, xl);
        m.fx = 0;
    } else if (x > K.rx1) {
        const float o = (x - K.lx1) + (xl - K.lx1l);
        m.lx = 2.0f * o;
        mirror_lo(K.lx1, K.lx1l, -o, x, xl);
        m.fx = 1;
    }
    if (y < K.ry0) {
        const float o = (K.ly0 - y) + (K.ly0l - yl);
        m.ly = 2.0f * o;
        mirror_lo(K.ly0, K.ly0l, o, y, yl);
        m.fy = 2;
    } else if (y > K.ry1) {
        const float o = (y - K.ly1) + (yl - K.ly1l);
        m.ly = 2.0f * o;
        mirror_lo(K.ly1, K.ly1l, -o, y, yl);
        m.fy = 3;
    }
    return m;
}
// FP64 keeps its reflect (no compensation term)
__device__ __forceinline__ Mirror<double> reflect_c(const Consts<double> &K, double &x, double &y, double &, double &)
{
    return reflect(K, x, y);
}

// Reflection at the disc's edge (disc domains, FP64): a point past the
// circle is mirrored radially, X' = c + (R - o) (X - c) / |X - c| with the
// overshoot o = |X - c| - R; the local time grows by 2 o, and the move's foot
// c + R (X - c) / |X - c| is returned in (fx, fy).  face 4, or -1 for none.
__device__ __forceinline__ Mirror<double> reflect_disc(const Inst &D, double &x, double &y, double &fx, double &fy)
{
    Mirror<double> m{0.0, 0.0, -1, -1};
    const double ex = x - D.ocx, ey = y - D.ocy;
    const double d2 = ex * ex + ey * ey;
    if (d2 > D.orad2) {
        const double d = sqrt(d2);
        const double o = d - D.orad;
        const double inv = 1.0 / d;
        const double s = (D.orad - o) * inv, f = D.orad * inv;
        fx = D.ocx + f * ex;
        fy = D.ocy + f * ey;
        x = D.ocx + s * ex;
        y = D.ocy + s * ey;
        m.lx = 2.0 * o;
        m.fx = 4;
    }
    return m;
}
// With the compensated FP32 position: the point x + xl is tested and
// mirrored in FP64 (the same arithmetic as above), and the mirrored point is
// split back into its binary32 value and the rest.  Every lane forms the
// test: with one lane in ten mirroring per trip, a wave almost never skips
// the mirror branch, so a binary32 pre-test would save nothing.
__device__ __forceinline__ Mirror<float> reflect_disc_c(const Inst &D, float &x, float &y, float &xl, float &yl,
                                                        float &fx, float &fy)
{
    Mirror<float> m{0.0f, 0.0f, -1, -1};
    double X = (double)x + (double)xl, Y = (double)y + (double)yl, FX = 0.0, FY = 0.0;
    const Mirror<double> md = reflect_disc(D, X, Y, FX, FY);
    if (md.fx >= 0) {
        x = (float)X;
        xl = (float)(X - (double)x);
        y = (float)Y;
        yl = (float)(Y - (double)y);
        fx = (float)FX;
        fy = (float)FY;
        m.lx = (float)md.lx;
        m.fx = 4;
    }
    return m;
}
__device__ __forceinline__ Mirror<double> reflect_disc_c(const Inst &D, double &x, double &y, double &, double &,
                                                         double &fx, double &fy)
{
    return reflect_disc(D, x, y, fx, fy);
}

// Bilinear interpolation of u_n at (x, y): cell p = floor((x - x0)/dx)
// clamped to [0, nx-2] (likewise q), fractions a, b; lerp in x then in y.
// The grid is read with raw buffer loads: the base address stays in scalar
// registers, the offset is 32-bit, and an offset outside the grid returns
// zero instead of touching other memory.
__device__ __forceinline__ float clamp_cell(float v, float hi) { return __builtin_amdgcn_fmed3f(v, 0.0f, hi); }

template <class R> struct Cell {
    R a, b;          // fractions within the cell
    uint32_t off;    // byte offset of the cell's first read
};

template <class R>
__device__ __forceinline__ Cell<R> locate(const Consts<R> &K, R x, R y)
{
    // one multiply-add per coordinate; just inside the lower edge the
    // rounding may give a fraction a few ulp below 0, which the clamp keeps
    // in the first cell (the interpolant is continuous there)
    const R fx = fma(x, K.idx, K.ox), fy = fma(y, K.idy, K.oy);
    if constexpr (sizeof(R) == 8) {
        // FP64: truncate, then clamp as integers (half the issue cost of
        // FP64 floor / max / min); for fx > -1 truncation is the floor, and
        // below it both clamp to cell 0, so cell and fraction are those of
        // the clamped floor.  Points lie within a few cells of the grid
        // (|z| < 6), well inside the int range.
        const int p = min(max((int)fx, 0), K.pmaxi);
        const int q = min(max((int)fy, 0), K.qmaxi);
        const uint32_t off = (uint32_t)__umul24((uint32_t)p, K.sx) + (uint32_t)__umul24((uint32_t)q, K.sy);
        return Cell<R>{fx - (R)p, fy - (R)q, off};
    } else {
        const R pf = clamp_cell(floor(fx), K.pmax);
        const R qf = clamp_cell(floor(fy), K.qmax);
        // p, q < 2^24 and the strides < 2^24 (checked at set-up): full-rate
        // 24-bit products
        const uint32_t off = (uint32_t)__umul24((uint32_t)pf, K.sx) + (uint32_t)__umul24((uint32_t)qf, K.sy);
        return Cell<R>{fx - pf, fy - qf, off};
    }
}

template <class R>
__device__ __forceinline__ void lerp(const Cell<R> &c, R u00r, R u00i, R u10r, R u10i, R u01r, R u01i, R u11r,
                                     R u11i, R &vr, R &vi)
{
    const R lr0 = u00r + c.a * (u10r - u00r), li0 = u00i + c.a * (u10i - u00i);
    const R lr1 = u01r + c.a * (u11r - u01r), li1 = u01i + c.a * (u11i - u01i);
    vr = lr0 + c.b * (lr1 - lr0);
    vi = li0 + c.b * (li1 - li0);
}

typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));
typedef unsigned int u32x2 __attribute__((ext_vector_type(2)));

__device__ __forceinline__ u32x4 grid_load(const __amdgpu_buffer_rsrc_t &g, uint32_t off)
{
    return __builtin_amdgcn_raw_buffer_load_b128(g, off, 0, 0);
}

// Reads of u_n at one point: its cell, and the 16-byte reads in flight.
// FP32: u00 u10 | u01 u11 (two reads); FP64: u00 | u10 | u01 | u11 (four).
// The top pair sits at + second: the next row, or the second half of the
// cell's block in the cell-major copy.
template <class R> struct CellReads;
template <> struct CellReads<float> {
    Cell<float> c;
    u32x4 a, b;
};
template <> struct CellReads<double> {
    Cell<double> c;
    u32x4 a0, a1, b0, b1;
};

// Large grids miss the vector L1 on nearly every read, and the stepping loop
// is then bound by the rate of L2 requests.  In the cell-major copy a cell's
// reads share one line: issued back to back, the later reads join the first
// one's miss, for one L2 request per step.  Any instruction or wait the
// scheduler puts between them was measured to cost extra requests (the line
// is not yet allocated, or already evicted), so the reads of a cell are
// fenced off from the scheduler.
// With the row-major FP32 copy staged in LDS (kLdsGrid), the same two
// pairs of corners come from LDS, in 8-byte reads (a row offset is only
// 8-byte aligned).
template <int F = 0>
__device__ __forceinline__ void issue_reads(const Consts<float> &K, uint32_t off, CellReads<float> &r)
{
    if constexpr ((F & kLdsGrid) != 0) {
        typedef __attribute__((address_space(3))) const u32x2 lds_u2;
        const lds_u2 *a = (const lds_u2 *)(K.lgrid + off);
        const lds_u2 *b = (const lds_u2 *)(K.lgrid + off + K.second);
        const u32x2 a0 = a[0], a1 = a[1], b0 = b[0], b1 = b[1];
        r.a = u32x4{a0.x, a0.y, a1.x, a1.y};
        r.b = u32x4{b0.x, b0.y, b1.x, b1.y};
    } else {
        __builtin_amdgcn_sched_barrier(0);
        r.a = grid_load(K.grid, off);
        r.b = grid_load(K.grid, off + K.second);
        __builtin_amdgcn_sched_barrier(0);
    }
}
template <int F = 0>
__device__ __forceinline__ void issue_reads(const Consts<double> &K, uint32_t off, CellReads<double> &r)
{
    r.a0 = grid_load(K.grid, off);
    r.a1 = grid_load(K.grid, off + 16u);
    r.b0 = grid_load(K.grid, off + K.second);
    r.b1 = grid_load(K.grid, off + K.second + 16u);
}

// In the cell-major copy the second point's reads are issued only once the
// first point's have returned, so that at most one cell per lane is in
// flight (two in flight were measured to cost more L2 requests).
__device__ __forceinline__ void after_reads(uint32_t &off, const CellReads<float> &r)
{
    asm volatile("" : "+v"(off) : "v"(r.b[0]));
}
__device__ __forceinline__ void after_reads(uint32_t &off, const CellReads<double> &r)
{
    asm volatile("" : "+v"(off) : "v"(r.b1[0]));
}

__device__ __forceinline__ void value(const CellReads<float> &r, float &vr, float &vi)
{
    auto f = [](uint32_t w) { return __uint_as_float(w); };
    lerp(r.c, f(r.a[0]), f(r.a[1]), f(r.a[2]), f(r.a[3]), f(r.b[0]), f(r.b[1]), f(r.b[2]), f(r.b[3]), vr, vi);
}
__device__ __forceinline__ void value(const CellReads<double> &r, double &vr, double &vi)
{
    auto d = [](uint32_t lo, uint32_t hi) {
        return __longlong_as_double((long long)(((uint64_t)hi << 32) | lo));
    };
    lerp(r.c, d(r.a0[0], r.a0[1]), d(r.a0[2], r.a0[3]), d(r.a1[0], r.a1[1]), d(r.a1[2], r.a1[3]),
         d(r.b0[0], r.b0[1]), d(r.b0[2], r.b0[3]), d(r.b1[0], r.b1[1]), d(r.b1[2], r.b1[3]), vr, vi);
}

// source f at a point (the caller branches on K.src_kind != SRC_ZERO)
template <class R>
__device__ __forceinline__ void source(const Consts<R> &K, R x, R y, R &fr, R &fi)
{
    if (K.src_kind == SRC_CONST) {
        fr = K.src_re;
        fi = K.src_im;
    } else {
        const R ex = x - K.src_cx, ey = y - K.src_cy;
        const R e = exp_src(-K.src_c * (ex * ex + ey * ey), *K.tab);
        fr = K.src_re * e;
        fi = K.src_im * e;
    }
}

// One Philox block = normals for two increments; takes up to two Euler steps.
// Both points of the trip are computed first, so the gathers of u_n at the
// two left points are in flight together and overlap the exit tests; the
// second step counts only if the first did not end the path.  Returns true
// when the path is finished (exited or capped).
// The integrand f - (alpha + i p) I_h[u_n] is formed as -(cu v) + f with the
// coefficient cu = alpha + i p (k^2 without a shift or damping), or 0 while
// u_n = 0 (n = 0): the gather then still runs but adds nothing, so no
// lane-dependent branch separates the two gathers.  With a shift the
// values at step t carry the discount e^{-(alpha - k^2) t h}, kept in FP64 and
// advanced by the factor q = e^{-(alpha - k^2) h} per step.
template <class R> struct Coef {
    R re, im;
    R ik;         // k while u_n != 0 (the Robin coupling i k u_n), else 0
};

// Local-time term of one mirror move (reflecting edge): the integrand
// i k I_h[u_n] + g2 at the foot of the move on face `face`, times the
// increment dxi and the discount w at the end of the step.  It enters the
// score with a plus sign; it is folded into the left-point sum, which the
// score multiplies by -h, as -w dxi (...) / h.
template <class R, int F>
__device__ __forceinline__ void local_time_term(const Inst &D, const Consts<R> &K, int face, R fx, R fy, R dxi,
                                                double w, R ik, PathState<R> &P)
{
    CellReads<R> g;
    g.c = locate(K, fx, fy);
    issue_reads<F>(K, g.c.off, g);
    R vr, vi;
    value(g, vr, vi);
    double gr = -(double)(ik * vi), gi = (double)(ik * vr);
    if (K.robin_g2) {
        const double xf = face == 0 ? D.x0 : (face == 1 ? D.x1 : (double)fx);
        const double yf = face == 2 ? D.y0 : (face == 3 ? D.y1 : (double)fy);
        const double2 g2 = robin_datum<F>(D, face, xf, yf);
        gr += g2.x;
        gi += g2.y;
    }
    const double c = w * (double)dxi * K.ih;
    P.ar -= c * gr;
    P.ai -= c * gi;
}

// The local-time moves of one trip, handed to the wave's batched evaluation
// instead of being evaluated at once (reflecting edge, path kernels): up to
// four per lane (bits of todo: step 1 x face, step 1 y face, step 2 x face,
// step 2 y face, the chronological order), each with w dxi, the foot's
// coordinate along its face and the face.  The disc's edge has at most one
// move per step (bits 0 and 2), its foot's x and y in coord[kk], coord[kk+1].
template <class R> struct LtEvents {
    uint32_t bits;     // todo (bits 0-3) | the four faces (2 bits each, from bit 4)
    R dxi[4];          // increments of the local time
    R coord[4];
    double w1, w2;     // end-of-step discounts (1 without a shift)
};

// Batched local-time terms (reflecting edge).  Evaluated one move at a time,
// the term runs for the whole wave whenever any lane mirrors (nearly every
// trip, with one lane in ten active).  Instead the wave appends its moves to
// a queue in LDS, in chronological order, and evaluates 64 of them at once,
// one per lane; each owner then adds the results of its own moves, in queue
// order, to its path's local-time sum.  That sum is kept apart from the
// left-point sum, so a path's score depends on its own moves only, not on
// when its wave happened to evaluate them.  A path's queued moves are
// evaluated before its score (the wave drains the queue whenever a finishing
// lane still owns a move).
constexpr int kLtCap = 2 * kWave;   // queued moves per wave

template <class R> struct LtStore {
    double cw[kLtCap];      // w dxi
    R coord[kLtCap];        // the foot's coordinate along its face (the disc: its x)
    int32_t fo[kLtCap];     // face | owner lane << 2
    double res_r[kWave], res_i[kWave];
};
// The disc's edge: a foot has two coordinates (face 4 throughout).
template <class R> struct LtStoreC : LtStore<R> {
    R coord2[kLtCap];       // the foot's y
};
struct LtNone {};

template <class R> struct LtQueue {
    LtStore<R> *s;
    int count;                  // moves held (wave-uniform)
    unsigned long long own0, own1;   // this lane's moves at queue positions 0..63 and 64..127
};

// Evaluates the first min(count, 64) queued moves, one per lane, and adds
// each owner's results in order to its local-time sum; moves the rest down.
// Every lane of the wave calls it.
template <class R, int F>
__device__ __forceinline__ void lt_eval(const Inst &D, const Consts<R> &K, LtQueue<R> &Q, R ik, PathState<R> &P)
{
    constexpr bool kC = (F & kFeatCurved) != 0;
    const int lane = threadIdx.x & (kWave - 1);
    const int n = Q.count < kWave ? Q.count : kWave;
    LtStore<R> &S = *Q.s;
    if (lane < n) {
        const int fo = S.fo[lane];
        const int face = kC ? 4 : fo & 3;
        const R c = S.coord[lane];
        R fx, fy;
        if constexpr (kC) {
            fx = c;
            fy = static_cast<LtStoreC<R> &>(S).coord2[lane];
        } else {
            fx = face == 0 ? K.lx0 : (face == 1 ? K.lx1 : c);
            fy = face == 2 ? K.ly0 : (face == 3 ? K.ly1 : c);
        }
        CellReads<R> g;
        g.c = locate(K, fx, fy);
        issue_reads<F>(K, g.c.off, g);
        R vr, vi;
        value(g, vr, vi);
        double gr = -(double)(ik * vi), gi = (double)(ik * vr);
        if (K.robin_g2) {
            const double xf = face == 0 ? D.x0 : (face == 1 ? D.x1 : (double)fx);
            const double yf = face == 2 ? D.y0 : (face == 3 ? D.y1 : (double)fy);
            const double2 g2 = robin_datum<F>(D, face, xf, yf);
            gr += g2.x;
            gi += g2.y;
        }
        const double cc = S.cw[lane] * K.ih;
        S.res_r[lane] = cc * gr;
        S.res_i[lane] = cc * gi;
    }
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    unsigned long long mine = Q.own0;
    while (mine) {
        const int q = __ffsll((long long)mine) - 1;
        mine &= mine - 1ull;
        P.lr -= S.res_r[q];
        P.li -= S.res_i[q];
    }
    const int rest = Q.count - n;
    if (rest > 0) {
        // positions 64.. move down to 0..
        double cw = 0.0;
        R co = (R)0, co2 = (R)0;
        int32_t fo = 0;
        if (lane < rest) {
            cw = S.cw[kWave + lane];
            co = S.coord[kWave + lane];
            fo = S.fo[kWave + lane];
            if constexpr (kC) co2 = static_cast<LtStoreC<R> &>(S).coord2[kWave + lane];
        }
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        if (lane < rest) {
            S.cw[lane] = cw;
            S.coord[lane] = co;
            S.fo[lane] = fo;
            if constexpr (kC) static_cast<LtStoreC<R> &>(S).coord2[lane] = co2;
        }
    }
    Q.own0 = rest > 0 ? Q.own1 : 0ull;
    Q.own1 = 0ull;
    Q.count = rest;
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Appends one kind of move of the trip (the lanes where `has`) to the queue,
// evaluating a batch first when 64 are waiting (the queue then has room for
// 64 more).  Every lane of the wave calls it.
template <class R, int F>
__device__ __forceinline__ void lt_push(const Inst &D, const Consts<R> &K, LtQueue<R> &Q, R ik, PathState<R> &P,
                                        bool has, double cw, R coord, R coord2, int face)
{
    const unsigned long long b = __ballot(has);
    if (b == 0ull) return;
    if (Q.count >= kWave) lt_eval<R, F>(D, K, Q, ik, P);
    const int lane = threadIdx.x & (kWave - 1);
    if (has) {
        const int q = Q.count + (int)__builtin_amdgcn_mbcnt_hi((uint32_t)(b >> 32),
                                                               __builtin_amdgcn_mbcnt_lo((uint32_t)b, 0u));
        Q.s->cw[q] = cw;
        Q.s->coord[q] = coord;
        Q.s->fo[q] = face | (lane << 2);
        if constexpr ((F & kFeatCurved) != 0) static_cast<LtStoreC<R> *>(Q.s)->coord2[q] = coord2;
        if (q < kWave) Q.own0 |= 1ull << q;
        else Q.own1 |= 1ull << (q - kWave);
    }
    Q.count += __popcll(b);
}

// The trip's moves (in the order of LtEvents) into the queue, then every
// queued move if a finishing path (fin) owns one.
template <class R, int F>
__device__ __forceinline__ void lt_trip(const Inst &D, const Consts<R> &K, LtQueue<R> &Q, R ik, PathState<R> &P,
                                        const LtEvents<R> &ev, bool fin)
{
    if constexpr ((F & kFeatCurved) != 0) {
        // the disc: at most one move per step (bits 0 and 2), its foot in
        // coord[kk], coord[kk + 1]
#pragma unroll
        for (int kk = 0; kk < 4; kk += 2)
            lt_push<R, F>(D, K, Q, ik, P, ((ev.bits >> kk) & 1u) != 0u,
                          (kk < 2 ? ev.w1 : ev.w2) * (double)ev.dxi[kk], ev.coord[kk], ev.coord[kk + 1], 4);
    } else {
#pragma unroll
        for (int kk = 0; kk < 4; ++kk)
            lt_push<R, F>(D, K, Q, ik, P, ((ev.bits >> kk) & 1u) != 0u,
                          (kk < 2 ? ev.w1 : ev.w2) * (double)ev.dxi[kk], ev.coord[kk], (R)0,
                          (int)((ev.bits >> (4 + 2 * kk)) & 3u));
    }
    if (__ballot(fin && (Q.own0 | Q.own1) != 0ull))
        while (Q.count > 0) lt_eval<R, F>(D, K, Q, ik, P);
}

template <class R, int F, bool kDefer = false>
__device__ __forceinline__ bool advance(const Inst &D, const Consts<R> &K, PathState<R> &P, uint32_t m,
                                        uint32_t node, uint32_t ctr3, Coef<R> cu, bool &exited,
                                        LtEvents<R> *ev = nullptr)
{
    // Both points' reads are issued after the normals, except in the build
    // for row-major copies.  (Issuing the current point's before the Philox
    // block was measured slower on large grids in FP32, where the loop is
    // bound by L2 requests.)
    CellReads<R> g0, g1;
    constexpr bool early = (F & kRowMajor) != 0;
    uint32_t ctr0 = (uint32_t)(P.t >> 1);
    if constexpr (early) {
        // Row-major copy (L1 hits): the current point's cell is read first,
        // its latency covered by the Philox block and both pairs of normals;
        // the empty asm statement keeps the reads ahead of the Philox block.
        // (Measured on the 65 x 65 and 33 x 33 cavities against the other
        // orders: +1-3% over both reads after the normals, +1% over the
        // second pair of normals run under both reads or under the second.)
        g0.c = locate(K, P.x, P.y);
        issue_reads<F>(K, g0.c.off, g0);
        asm volatile("" : "+v"(ctr0));
    }
    // The round keys k + r (Weyl constants) are loop-invariant; hoisted, all
    // twenty no longer fit the scalar registers and were spilled to vector
    // lanes and read back (two VALU reads per round).  An opaque scalar zero
    // per trip keeps the key schedule in scalar adds next to its use.
    uint32_t kz;
    asm volatile("s_mov_b32 %0, 0" : "=s"(kz));
    const uint4 w = philox4x32_10(ctr0, m, node, ctr3, K.key0 + kz, K.key1 + kz);
    R z0x, z0y, z1x, z1y;
    normals(w.x, w.y, *K.tab, z0x, z0y);
    normals(w.z, w.w, *K.tab, z1x, z1y);
    R x1, y1, x1l, y1l;
    move(K, P.x, P.xl, z0x, x1, x1l);
    move(K, P.y, P.yl, z0y, y1, y1l);
    if constexpr (early) {
        // the second pair stays ahead of the branch of the second step (the
        // compiler would move it there), and the second cell's reads follow
        asm volatile("" : : "v"(z1x), "v"(z1y));
        g1.c = locate(K, x1, y1);
        issue_reads<F>(K, g1.c.off, g1);
    }
    // a reflecting edge mirrors each step back into the rectangle
    const bool refl = (F & kFeatReflect) && K.reflect;
    Mirror<R> m1{(R)0, (R)0, -1, -1}, m2{(R)0, (R)0, -1, -1};
    R f1x = (R)0, f1y = (R)0, f2x = (R)0, f2y = (R)0;   // feet of the disc's mirror moves
    if (refl) {
        if constexpr ((F & kFeatCurved) != 0) m1 = reflect_disc_c(D, x1, y1, x1l, y1l, f1x, f1y);
        else m1 = reflect_c(K, x1, y1, x1l, y1l);
    }
    R x2, y2, x2l, y2l;
    move(K, x1, x1l, z1x, x2, x2l);
    move(K, y1, y1l, z1y, y2, y2l);
    if (refl) {
        if constexpr ((F & kFeatCurved) != 0) m2 = reflect_disc_c(D, x2, y2, x2l, y2l, f2x, f2y);
        else m2 = reflect_c(K, x2, y2, x2l, y2l);
    }
    const bool general = (F & kFeatGeneral) && K.general;
    bool out1, out2, second;
    if constexpr ((F & kFeatReflect) != 0) {
        // with a reflecting edge the exit tests and the local-time terms come
        // before the left-point gathers, so that the mirror state is dead
        // while those are in flight
        out1 = is_out<F>(D, K, x1, y1);
        out2 = is_out<F>(D, K, x2, y2);
        second = !out1 && P.t + 1 < K.jmax;
        // local time of the step(s) taken: up to one mirror move per face and
        // step (bits 0-3: step 1 x, step 1 y, step 2 x, step 2 y), each at
        // the end-of-step discount.  The path kernels hand the moves to the
        // wave's batched evaluation (a trip has a move in about one lane in
        // ten); evaluated at once (single paths), each lane works through its
        // own moves.
        uint32_t todo = (uint32_t)(m1.fx >= 0) | ((uint32_t)(m1.fy >= 0) << 1);
        if (second) todo |= ((uint32_t)(m2.fx >= 0) << 2) | ((uint32_t)(m2.fy >= 0) << 3);
        if constexpr (kDefer && (F & kFeatCurved) != 0) {
            // the disc: one radial move per step (bits 0 and 2), with its
            // foot's two coordinates
            ev->w1 = general ? P.w * K.q : 1.0;
            ev->w2 = general ? ev->w1 * K.q : 1.0;
            ev->bits = todo;
            ev->dxi[0] = m1.lx;
            ev->coord[0] = f1x;
            ev->coord[1] = f1y;
            ev->dxi[2] = m2.lx;
            ev->coord[2] = f2x;
            ev->coord[3] = f2y;
        } else if constexpr (kDefer) {
            // the moves in chronological order; the foot of an x-face move is
            // (face, y of the mirrored point), of a y-face move (x, face)
            ev->w1 = general ? P.w * K.q : 1.0;
            ev->w2 = general ? ev->w1 * K.q : 1.0;
            ev->bits = todo | ((uint32_t)(m1.fx & 3) << 4) | ((uint32_t)(m1.fy & 3) << 6) |
                       ((uint32_t)(m2.fx & 3) << 8) | ((uint32_t)(m2.fy & 3) << 10);
            ev->dxi[0] = m1.lx;
            ev->coord[0] = y1;
            ev->dxi[1] = m1.ly;
            ev->coord[1] = x1;
            ev->dxi[2] = m2.lx;
            ev->coord[2] = y2;
            ev->dxi[3] = m2.ly;
            ev->coord[3] = x2;
        } else if (todo) {
            const double w1 = general ? P.w * K.q : 1.0;
            const double w2 = general ? w1 * K.q : 1.0;
            do {
                const int c = __builtin_ctz(todo);
                todo &= todo - 1u;
                const bool s2 = c >= 2, ym = (c & 1) != 0;
                if constexpr ((F & kFeatCurved) != 0) {
                    // the disc's edge: one radial move per step, at its foot
                    local_time_term<R, F>(D, K, 4, s2 ? f2x : f1x, s2 ? f2y : f1y, s2 ? m2.lx : m1.lx,
                                          s2 ? w2 : w1, cu.ik, P);
                } else {
                    const int face = ym ? (s2 ? m2.fy : m1.fy) : (s2 ? m2.fx : m1.fx);
                    const R px = s2 ? x2 : x1, py = s2 ? y2 : y1;
                    const R fx = face == 0 ? K.lx0 : (face == 1 ? K.lx1 : px);
                    const R fy = face == 2 ? K.ly0 : (face == 3 ? K.ly1 : py);
                    const R dxi = ym ? (s2 ? m2.ly : m1.ly) : (s2 ? m2.lx : m1.lx);
                    local_time_term<R, F>(D, K, face, fx, fy, dxi, s2 ? w2 : w1, cu.ik, P);
                }
            } while (todo);
        }
    }
    if constexpr (!early) {
        g0.c = locate(K, P.x, P.y);
        g1.c = locate(K, x1, y1);
        issue_reads<F>(K, g0.c.off, g0);
        uint32_t o1 = g1.c.off;
        if (!early && K.cells) after_reads(o1, g0);
        issue_reads<F>(K, o1, g1);
    }
    R v0r, v0i, v1r, v1i;
    value(g0, v0r, v0i);
    value(g1, v1r, v1i);
    R fr, fi, gr, gi;
    if (general) {
        fr = -(cu.re * v0r - cu.im * v0i);
        fi = -(cu.re * v0i + cu.im * v0r);
        gr = -(cu.re * v1r - cu.im * v1i);
        gi = -(cu.re * v1i + cu.im * v1r);
    } else {
        fr = -(cu.re * v0r);
        fi = -(cu.re * v0i);
        gr = -(cu.re * v1r);
        gi = -(cu.re * v1i);
    }
    if ((F & kFeatSource) && K.src_kind != SRC_ZERO) {
        R sr, si;
        source<R>(K, P.x, P.y, sr, si);
        fr += sr;
        fi += si;
        source<R>(K, x1, y1, sr, si);
        gr += sr;
        gi += si;
    }
    if constexpr ((F & kFeatReflect) == 0) {
        out1 = is_out<F>(D, K, x1, y1);
        out2 = is_out<F>(D, K, x2, y2);
        second = !out1 && P.t + 1 < K.jmax;
    }
    if (general) {
        // each value with its own discount, summed in FP64
        const double w1 = P.w * K.q;
        P.ar += P.w * (double)fr;
        P.ai += P.w * (double)fi;
        if (second) {
            P.ar += w1 * (double)gr;
            P.ai += w1 * (double)gi;
        }
        P.w = second ? w1 * K.q : w1;
    } else {
        if (second) {
            fr += gr;
            fi += gi;
        }
        P.ar += (double)fr;
        P.ai += (double)fi;
    }
    P.x = second ? x2 : x1;
    P.y = second ? y2 : y1;
    if constexpr (sizeof(R) == 4) {
        P.xl = second ? x2l : x1l;
        P.yl = second ? y2l : y1l;
    }
    P.t += second ? 2 : 1;
    exited = second ? out2 : out1;
    return exited || P.t >= K.jmax;
}

// ------------------------------------------------------------ tail mode
// At the end of an iteration the last paths run on a nearly idle GPU, each at
// the latency of one lonely wave; the longest of ~10^7 paths takes ~20 mean
// path lengths, and this tail was a sixth of an iteration.  But a path's
// positions depend only on its normals (counter-based, one Philox block per
// trip), not on u_n, so its future can be computed in parallel in time: with
// all 64 lanes of the wave on one path, lane i draws the normals of trip i of
// the next 64, one serial chain of the same multiply-adds (in the same order,
// on uniform values) gives every trip's points, the exit tests and the
// gathers of all trips run at once, and a serial pass adds the trips'
// integrands in path order.  Every value is the one the step-by-step loop
// forms, so the results are identical.  Not used with a reflecting edge.
// A wave enters it once the queue has nothing left for it and at most
// FK_TAIL_LANES of its lanes still run a path; several paths share a pass in
// lane groups (measured on the 65 x 65 cavity: 16 best, 8 and 32 within 1%;
// with one path per pass 8 was best and 32 or more lost to no tail mode).

#ifndef FK_TAIL_LANES
#define FK_TAIL_LANES 16
#endif
constexpr int kTailLanes = FK_TAIL_LANES;   // a wave with no work left and at most this many active lanes

template <class R> struct TailPath {
    R x, y, xl, yl;
    double ar, ai, w;
    int t;
    uint32_t m, node;
};

__device__ __forceinline__ float lane_value(float v, int i) { return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), i)); }
__device__ __forceinline__ double lane_value(double v, int i)
{
    const long long b = __double_as_longlong(v);
    const uint32_t lo = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)b, i);
    const uint32_t hi = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)(b >> 32), i);
    return __longlong_as_double((long long)(((uint64_t)hi << 32) | lo));
}
__device__ __forceinline__ int lane_value(int v, int i) { return __builtin_amdgcn_readlane(v, i); }
__device__ __forceinline__ uint32_t lane_value(uint32_t v, int i) { return (uint32_t)__builtin_amdgcn_readlane((int)v, i); }

// Up to 64 trips (128 steps) of path S, by the whole wave (S uniform).
// Returns true when the path finished (exited or capped); S is advanced.
template <class R, int F>
__device__ __forceinline__ bool tail_pass(const Inst &D, const Consts<R> &K, TailPath<R> &S, uint32_t ctr3, Coef<R> cu,
                                       bool &exited)
{
    const int lane = threadIdx.x & (kWave - 1);
    uint32_t kz;
    asm volatile("s_mov_b32 %0, 0" : "=s"(kz));
    const uint4 wd = philox4x32_10((uint32_t)(S.t >> 1) + (uint32_t)lane, S.m, S.node, ctr3, K.key0 + kz,
                                   K.key1 + kz);
    R z0x, z0y, z1x, z1y;
    normals(wd.x, wd.y, *K.tab, z0x, z0y);
    normals(wd.z, wd.w, *K.tab, z1x, z1y);
    // the points of every trip, in the order and form of the step loop
    R px = S.x, py = S.y, x1 = S.x, y1 = S.y, x2 = S.x, y2 = S.y;
    R x1l = S.xl, y1l = S.yl, x2l = S.xl, y2l = S.yl;
    {
        R cx = S.x, cy = S.y, cxl = S.xl, cyl = S.yl;
#pragma unroll 1
        for (int i = 0; i < kWave; ++i) {
            const R a0 = lane_value(z0x, i), b0 = lane_value(z0y, i);
            const R a1 = lane_value(z1x, i), b1 = lane_value(z1y, i);
            R nx1, ny1, nx2, ny2, nx1l, ny1l, nx2l, ny2l;
            move(K, cx, cxl, a0, nx1, nx1l);
            move(K, cy, cyl, b0, ny1, ny1l);
            move(K, nx1, nx1l, a1, nx2, nx2l);
            move(K, ny1, ny1l, b1, ny2, ny2l);
            if (lane == i) {
                px = cx; py = cy; x1 = nx1; y1 = ny1; x2 = nx2; y2 = ny2;
                x1l = nx1l; y1l = ny1l; x2l = nx2l; y2l = ny2l;
            }
            cx = nx2;
            cy = ny2;
            cxl = nx2l;
            cyl = ny2l;
        }
    }
    const int ts = S.t + 2 * lane;                      // steps taken before this lane's trip
    const bool out1 = is_out<F>(D, K, x1, y1);
    const bool out2 = is_out<F>(D, K, x2, y2);
    const bool second = !out1 && ts + 1 < K.jmax;
    const bool ends = (second ? out2 : out1) || ts + (second ? 2 : 1) >= K.jmax;
    const unsigned long long em = __ballot(ends);
    const int n = em ? __ffsll((long long)em) : kWave;   // trips that count
    // integrands at the two left points of each counted trip (as in advance)
    R fr = (R)0, fi = (R)0, gr = (R)0, gi = (R)0;
    const bool general = (F & kFeatGeneral) && K.general;
    if (lane < n) {
        CellReads<R> g0, g1;
        g0.c = locate(K, px, py);
        g1.c = locate(K, x1, y1);
        issue_reads<F>(K, g0.c.off, g0);
        uint32_t o1 = g1.c.off;
        if (K.cells) after_reads(o1, g0);
        issue_reads<F>(K, o1, g1);
        R v0r, v0i, v1r, v1i;
        value(g0, v0r, v0i);
        value(g1, v1r, v1i);
        if (general) {
            fr = -(cu.re * v0r - cu.im * v0i);
            fi = -(cu.re * v0i + cu.im * v0r);
            gr = -(cu.re * v1r - cu.im * v1i);
            gi = -(cu.re * v1i + cu.im * v1r);
        } else {
            fr = -(cu.re * v0r);
            fi = -(cu.re * v0i);
            gr = -(cu.re * v1r);
            gi = -(cu.re * v1i);
        }
        if ((F & kFeatSource) && K.src_kind != SRC_ZERO) {
            R sr, si;
            source<R>(K, px, py, sr, si);
            fr += sr;
            fi += si;
            source<R>(K, x1, y1, sr, si);
            gr += sr;
            gi += si;
        }
        if (!general && second) {
            fr += gr;
            fi += gi;
        }
    }
    // the trips' sums in path order
    const unsigned long long sm = __ballot(second);
    double ar = S.ar, ai = S.ai, w = S.w;
#pragma unroll 1
    for (int i = 0; i < n; ++i) {
        const bool sec = (sm >> i) & 1ull;
        const R a = lane_value(fr, i), b = lane_value(fi, i);
        if (general) {
            const R c = lane_value(gr, i), d = lane_value(gi, i);
            const double w1 = w * K.q;
            ar += w * (double)a;
            ai += w * (double)b;
            if (sec) {
                ar += w1 * (double)c;
                ai += w1 * (double)d;
            }
            w = sec ? w1 * K.q : w1;
        } else {
            ar += (double)a;
            ai += (double)b;
        }
    }
    const int l = n - 1;                                  // the last counted trip
    const bool sec_l = (sm >> l) & 1ull;
    S.x = lane_value(sec_l ? x2 : x1, l);
    S.y = lane_value(sec_l ? y2 : y1, l);
    if constexpr (sizeof(R) == 4) {
        S.xl = lane_value(sec_l ? x2l : x1l, l);
        S.yl = lane_value(sec_l ? y2l : y1l, l);
    }
    S.ar = ar;
    S.ai = ai;
    S.w = w;
    S.t = S.t + 2 * l + (sec_l ? 2 : 1);
    exited = lane_value((int)(sec_l ? out2 : out1), l) != 0;
    return n < kWave || (em >> (kWave - 1)) != 0ull;
}

// The same for several paths at once: the wave is split into groups of G
// lanes (G = 64 / 2^ceil(log2 k) for k paths), group g takes the g-th path
// and G trips of it per pass; values move between lanes by shuffles.
// S holds the group's path on every lane of the group.
__device__ __forceinline__ float lane_from(float v, int src) { return __shfl(v, src, kWave); }
__device__ __forceinline__ double lane_from(double v, int src) { return __shfl(v, src, kWave); }
__device__ __forceinline__ int lane_from(int v, int src) { return __shfl(v, src, kWave); }

template <class R, int F>
__device__ __forceinline__ bool tail_pass_grouped(const Inst &D, const Consts<R> &K, TailPath<R> &S, int G,
                                                  uint32_t ctr3, Coef<R> cu, bool &exited)
{
    const int lane = threadIdx.x & (kWave - 1);
    const int base = lane & ~(G - 1), j = lane - base;
    uint32_t kz;
    asm volatile("s_mov_b32 %0, 0" : "=s"(kz));
    const uint4 wd = philox4x32_10((uint32_t)(S.t >> 1) + (uint32_t)j, S.m, S.node, ctr3, K.key0 + kz,
                                   K.key1 + kz);
    R z0x, z0y, z1x, z1y;
    normals(wd.x, wd.y, *K.tab, z0x, z0y);
    normals(wd.z, wd.w, *K.tab, z1x, z1y);
    R px = S.x, py = S.y, x1 = S.x, y1 = S.y, x2 = S.x, y2 = S.y;
    R x1l = S.xl, y1l = S.yl, x2l = S.xl, y2l = S.yl;
    {
        R cx = S.x, cy = S.y, cxl = S.xl, cyl = S.yl;
#pragma unroll 1
        for (int i = 0; i < G; ++i) {
            const R a0 = lane_from(z0x, base + i), b0 = lane_from(z0y, base + i);
            const R a1 = lane_from(z1x, base + i), b1 = lane_from(z1y, base + i);
            R nx1, ny1, nx2, ny2, nx1l, ny1l, nx2l, ny2l;
            move(K, cx, cxl, a0, nx1, nx1l);
            move(K, cy, cyl, b0, ny1, ny1l);
            move(K, nx1, nx1l, a1, nx2, nx2l);
            move(K, ny1, ny1l, b1, ny2, ny2l);
            if (j == i) {
                px = cx; py = cy; x1 = nx1; y1 = ny1; x2 = nx2; y2 = ny2;
                x1l = nx1l; y1l = ny1l; x2l = nx2l; y2l = ny2l;
            }
            cx = nx2;
            cy = ny2;
            cxl = nx2l;
            cyl = ny2l;
        }
    }
    const int ts = S.t + 2 * j;
    const bool out1 = is_out<F>(D, K, x1, y1);
    const bool out2 = is_out<F>(D, K, x2, y2);
    const bool second = !out1 && ts + 1 < K.jmax;
    const bool ends = (second ? out2 : out1) || ts + (second ? 2 : 1) >= K.jmax;
    const unsigned long long gmask = (G == kWave) ? ~0ull : ((1ull << G) - 1ull);
    const unsigned long long em = (__ballot(ends) >> base) & gmask;
    const unsigned long long sm = (__ballot(second) >> base) & gmask;
    const int n = em ? __ffsll((long long)em) : G;
    R fr = (R)0, fi = (R)0, gr = (R)0, gi = (R)0;
    const bool general = (F & kFeatGeneral) && K.general;
    if (j < n) {
        CellReads<R> g0, g1;
        g0.c = locate(K, px, py);
        g1.c = locate(K, x1, y1);
        issue_reads<F>(K, g0.c.off, g0);
        uint32_t o1 = g1.c.off;
        if (K.cells) after_reads(o1, g0);
        issue_reads<F>(K, o1, g1);
        R v0r, v0i, v1r, v1i;
        value(g0, v0r, v0i);
        value(g1, v1r, v1i);
        if (general) {
            fr = -(cu.re * v0r - cu.im * v0i);
            fi = -(cu.re * v0i + cu.im * v0r);
            gr = -(cu.re * v1r - cu.im * v1i);
            gi = -(cu.re * v1i + cu.im * v1r);
        } else {
            fr = -(cu.re * v0r);
            fi = -(cu.re * v0i);
            gr = -(cu.re * v1r);
            gi = -(cu.re * v1i);
        }
        if ((F & kFeatSource) && K.src_kind != SRC_ZERO) {
            R sr, si;
            source<R>(K, px, py, sr, si);
            fr += sr;
            fi += si;
            source<R>(K, x1, y1, sr, si);
            gr += sr;
            gi += si;
        }
        if (!general && second) {
            fr += gr;
            fi += gi;
        }
    }
    double ar = S.ar, ai = S.ai, w = S.w;
#pragma unroll 1
    for (int i = 0; i < G; ++i) {
        const R a = lane_from(fr, base + i), b = lane_from(fi, base + i);
        const R c = lane_from(gr, base + i), d = lane_from(gi, base + i);
        if (i < n) {
            const bool sec = (sm >> i) & 1ull;
            if (general) {
                const double w1 = w * K.q;
                ar += w * (double)a;
                ai += w * (double)b;
                if (sec) {
                    ar += w1 * (double)c;
                    ai += w1 * (double)d;
                }
                w = sec ? w1 * K.q : w1;
            } else {
                ar += (double)a;
                ai += (double)b;
            }
        }
    }
    const int l = base + n - 1;
    const bool sec_l = (sm >> (n - 1)) & 1ull;
    S.x = lane_from(sec_l ? x2 : x1, l);
    S.y = lane_from(sec_l ? y2 : y1, l);
    if constexpr (sizeof(R) == 4) {
        S.xl = lane_from(sec_l ? x2l : x1l, l);
        S.yl = lane_from(sec_l ? y2l : y1l, l);
    }
    S.ar = ar;
    S.ai = ai;
    S.w = w;
    S.t = S.t + 2 * (n - 1) + (sec_l ? 2 : 1);
    exited = lane_from((int)(sec_l ? out2 : out1), l) != 0;
    return em != 0ull;
}

// A finished path waiting for its score: the last point and the left-point
// sum (FP64), its exit-step index and the node it belongs to.
struct Pending {
    double x, y, ar, ai;
    double wj;            // discount at the exit step
    int32_t t, node_idx;
    bool exited, live;
};

template <class R, bool kLt = false>
__device__ __forceinline__ void park(Pending &Q, const PathState<R> &P, bool exited, int32_t node_idx)
{
    if constexpr (sizeof(R) == 4) {
        Q.x = (double)P.x + (double)P.xl;   // the compensated position
        Q.y = (double)P.y + (double)P.yl;
    } else {
        Q.x = (double)P.x;
        Q.y = (double)P.y;
    }
    // with batched local-time terms, their sum joins the left-point sum here
    Q.ar = kLt ? P.ar + P.lr : P.ar;
    Q.ai = kLt ? P.ai + P.li : P.ai;
    Q.wj = P.w;
    Q.t = P.t;
    Q.node_idx = node_idx;
    Q.exited = exited;
    Q.live = true;
}

// Score of a finished path: the discounted datum g at the nearest boundary
// point minus h times the (discounted) left-point sum (Sec. 2.1 eq. (2.3)
// with killing rate c = alpha - k^2: the f-term enters with a minus sign).
template <int F>
__device__ __forceinline__ double2 score(const Inst &D, const Pending &Q)
{
    const double2 g = exit_datum<F>(D, Q.x, Q.y, Q.exited);
    // an instance without shift or damping scores exactly as in the kernels
    // without the feature (no multiply by the unit discount)
    if ((F & kFeatGeneral) && (D.alpha != D.k2 || D.damp != 0.0))
        return make_double2(Q.wj * g.x - D.h * Q.ar, Q.wj * g.y - D.h * Q.ai);
    return make_double2(g.x - D.h * Q.ar, g.y - D.h * Q.ai);
}

// Exact fixed-point split of v * scale into floor (hi) and the fraction in
// units of 2^-40 (lo).  v * scale and its fraction are exact in binary64, so
// the same score always gives the same integers, and integer sums do not
// depend on the order in which paths are added.
__device__ __forceinline__ void fix_split(double v, double scale, unsigned long long &hi, unsigned long long &lo)
{
    const double t = v * scale;
    const double f = floor(t);
    hi = (unsigned long long)(long long)f;
    lo = (unsigned long long)((t - f) * 0x1p40);
}

// Component i of one path's contribution to its node slot, as an exact
// integer (the Slot fields in order): 0-3 the score's real and imaginary
// parts (hi, lo at scale 2^16), 4-7 their squares (hi, lo at scale 1), 8 the
// exit-step index, 9 capped, 10 overflow.  Scores of magnitude 2^21 or more
// (and non-finite ones) count as overflow instead: the iteration is then
// reported as non-finite.
constexpr int kSlotSums = 11;

__device__ __forceinline__ unsigned long long contribution(int i, double2 sc, bool ok, int32_t J, bool capped)
{
    if (i == 8) return (unsigned long long)J;
    if (i == 9) return capped ? 1ull : 0ull;
    if (i == 10) return ok ? 0ull : 1ull;
    if (!ok) return 0ull;
    const double v = i < 2 ? sc.x : (i < 4 ? sc.y : (i < 6 ? sc.x * sc.x : sc.y * sc.y));
    unsigned long long hi, lo;
    fix_split(v, i < 4 ? 0x1p16 : 1.0, hi, lo);
    return (i & 1) ? lo : hi;
}

// A wave's LDS node accumulators, a ring of kNodeAcc: the node it takes
// paths from now and the ones before, whose long paths may still be
// running.  A new node takes the oldest accumulator after moving its sums
// to that node's slot (device-scope atomics, performed beyond the per-XCD
// L2).  With two, about 0.5% of the paths on the 65 x 65 cavity outlived two
// node changes and went to global memory one by one (half of the launch's
// 84 MB of writes); four keep nearly all of them in LDS.
constexpr int kNodeAcc = 4;
struct NodeAcc {
    // most recent first: b0 holds the current node n0's sums (12 each); a new
    // node evicts (b3, n3) and takes b3 as its b0 (node -1: none)
    unsigned long long *b0, *b1, *b2, *b3;
    int32_t n0, n1, n2, n3;
};

// Scores the parked paths of the wave and adds them to their node sums:
// exact 64-bit LDS atomics (no return) into the accumulator of the path's
// node, or, for a path that outlived four node changes of its wave,
// straight to the node's slot in global memory.
template <int F>
__device__ __forceinline__ void deposit_parked(const Inst &D, Pending &Q, const NodeAcc &A)
{
    if (Q.live) {
        const double2 sc = score<F>(D, Q);
        const bool ok = fabs(sc.x) < 0x1p21 && fabs(sc.y) < 0x1p21;
        unsigned long long *dst = Q.node_idx == A.n0   ? A.b0
                                  : Q.node_idx == A.n1 ? A.b1
                                  : Q.node_idx == A.n2 ? A.b2
                                  : Q.node_idx == A.n3 ? A.b3
                                                       : (unsigned long long *)(D.slots + Q.node_idx);
#pragma unroll 1
        for (int i = 0; i < kSlotSums; ++i) {
            const unsigned long long v = contribution(i, sc, ok, Q.t, !Q.exited);
            if (v != 0ull) atomicAdd(dst + i, v);
        }
        Q.live = false;
    }
}

// Moves one LDS accumulator into its node's slot (lane i < 11 posts sum i)
// and clears it.
__device__ __forceinline__ void flush_acc(const Inst &D, unsigned long long *acc, int32_t acc_node)
{
    const int lane = threadIdx.x & (kWave - 1);
    __builtin_amdgcn_wave_barrier();
    if (acc_node >= 0 && lane < kSlotSums) {
        const unsigned long long v = __hip_atomic_load(acc + lane, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
        if (v != 0ull) atomicAdd((unsigned long long *)(D.slots + acc_node) + lane, v);
    }
    __builtin_amdgcn_wave_barrier();
    if (lane < 12) acc[lane] = 0ull;
    __builtin_amdgcn_wave_barrier();
}

// Pending scores gather until more than this many lanes hold one (or a lane
// finishes a second path first, or the stream drains); then the wave scores
// them together.  Lanes refill at once, and the costly exit datum (nearest
// point, plane wave or table) runs for many lanes per pass.
constexpr int kScoreBatch = 40;

template <class R>
__device__ __forceinline__ void start(PathState<R> &P, R sx, R sy, R sxl = (R)0, R syl = (R)0)
{
    P.x = sx;
    P.y = sy;
    P.xl = sxl;
    P.yl = syl;
    P.ar = P.ai = 0.0;
    P.lr = P.li = 0.0;
    P.w = 1.0;
    P.t = 0;
}

// Next item number from the queue head.  Only the first active lane adds 1;
// every lane takes part in the atomic and the first lane's old value is read
// into scalar registers, so the value is wave-uniform and no branch on the
// lane id surrounds the fetch (a lane-0 branch here once let the compiler
// build a divergent loop in which lanes read a stale broadcast forever).
__device__ __forceinline__ int64_t fetch_item(unsigned long long *head)
{
    const unsigned long long ex = __ballot(true);
    const int lane = threadIdx.x & (kWave - 1);
    const bool first = lane == __ffsll((long long)ex) - 1;
    const unsigned long long a = atomicAdd(head, first ? 1ull : 0ull);
    const uint32_t lo32 = __builtin_amdgcn_readfirstlane((uint32_t)a);
    const uint32_t hi32 = __builtin_amdgcn_readfirstlane((uint32_t)(a >> 32));
    return (int64_t)(((uint64_t)hi32 << 32) | lo32);
}

// Segment s of the queue holds the items of instance seg_inst[s]; seg_end is
// the inclusive prefix sum of item counts.  Binary search (wave-uniform).
__device__ __forceinline__ int32_t find_segment(const EngineQueue *Q, int32_t nseg, int64_t g)
{
    int32_t lo = 0, hi = nseg - 1;
    while (lo < hi) {
        const int32_t mid = (lo + hi) >> 1;
        if (Q->seg_end[mid] > g) hi = mid;
        else lo = mid + 1;
    }
    return lo;
}

// The path kernel.  Work items (instance, node, chunk of ppi consecutive path
// indices) are numbered consecutively over the queue's instances; waves take
// items from an atomic counter until all are taken.  Within a wave the lanes
// form one stream: a lane whose path ends takes the next unused path index of
// the wave's current item, and when that item has no index left the wave
// fetches the next item, so lanes never wait for the slow paths of an item.
// A wave only mixes items of one instance; at an instance boundary it drains
// first.  Each path's score goes into its node's slot as exact integers, so
// the node sums do not depend on which wave, lane or launch ran which path:
// an instance gives bit-identical results alone, in any batch and for any
// item size.
template <class R, int F>
__device__ __forceinline__ void stream_paths(const Inst *__restrict__ insts, const EngineQueue *__restrict__ Q,
                                             unsigned long long *head)
{
    __shared__ typename TablesOf<R>::type tables;
    setup_tables<R>(tables);
    // waves per block: 4, or 16 when the block shares the staged FP32 grid
    constexpr bool kLds = (F & kLdsGrid) != 0;
    constexpr int kWpb = kLds ? 16 : 4;
    __shared__ unsigned long long lds_acc[kWpb][kNodeAcc * 12];   // node accumulators per wave
    // the queue of local-time moves of each wave (reflecting edge; the
    // disc's moves carry both coordinates of their foot)
    constexpr bool kLt = (F & kFeatReflect) != 0;
    using LtQ = typename std::conditional<(F & kFeatCurved) != 0, LtStoreC<R>, LtStore<R>>::type;
    using LtS = typename std::conditional<kLt, LtQ, LtNone>::type;
    __shared__ LtS lt_store[kWpb];
    // the staged copy of the (only) instance's row-major FP32 iterate
    const lds_u8 *lgrid = nullptr;
    if constexpr (kLds) {
        extern __shared__ u32x2 lds_grid_words[];
        typedef __attribute__((address_space(3))) u32x2 lds_w;
        lds_w *L = (lds_w *)lds_grid_words;
        if (Q->n_seg > 0) {
            const Inst &D0 = insts[Q->seg_inst[0]];
            const int nn = D0.nx * D0.ny;
            const u32x2 *src = (const u32x2 *)D0.gather;
            for (int i = threadIdx.x; i < nn; i += blockDim.x) L[i] = src[i];
        }
        __syncthreads();
        lgrid = (const lds_u8 *)L;
    }
    LtQueue<R> ltq;
    if constexpr (kLt) ltq.s = (LtStore<R> *)&lt_store[threadIdx.x / kWave];
    ltq.count = 0;
    ltq.own0 = ltq.own1 = 0ull;
    NodeAcc A;
    {
        unsigned long long *w = lds_acc[threadIdx.x / kWave];
        A.b0 = w;
        A.b1 = w + 12;
        A.b2 = w + 24;
        A.b3 = w + 36;
        if ((threadIdx.x & (kWave - 1)) < kNodeAcc * 12) w[threadIdx.x & (kWave - 1)] = 0ull;
    }
    __builtin_amdgcn_wave_barrier();
    const int32_t nseg = Q->n_seg;
    const int64_t total = nseg > 0 ? Q->seg_end[nseg - 1] : 0;
    int64_t carry = -1;    // an item fetched for another instance, run next
    for (;;) {
        int64_t g = carry >= 0 ? carry : fetch_item(head);
        carry = -1;
        if (g >= total) break;
        int32_t seg = find_segment(Q, nseg, g);
        const int32_t inst = Q->seg_inst[seg];
        const Inst &D = insts[inst];
        const Consts<R> K(D, &tables, lgrid);
        const bool use_u = D.state->use_u != 0;
        Coef<R> cu;
        cu.re = use_u ? ((F & kFeatGeneral) ? K.alpha : K.k2) : (R)0;
        cu.im = use_u && (F & kFeatGeneral) ? K.damp : (R)0;
        cu.ik = use_u ? K.kk : (R)0;
        const uint32_t ctr3 = D.crn ? 0u : (uint32_t)D.state->iter;

        // wave-uniform pool: path indices [pool_m, pool_end) of one node
        int64_t pool_m = 0, pool_end = 0;
        int32_t pool_node_idx = 0, pool_node = 0;
        A.n0 = A.n1 = A.n2 = A.n3 = -1;
        R pool_sx = (R)0, pool_sy = (R)0, pool_sxl = (R)0, pool_syl = (R)0;
        bool more = true;       // the queue may hold further items of this instance
        auto open_item = [&](int64_t gg) {
            const int64_t item = gg - (seg > 0 ? Q->seg_end[seg - 1] : 0);
            if (item < D.n_items_a) {
                // a large item: paths [chunk ppi_a, (chunk + 1) ppi_a) of its node
                pool_node_idx = (int32_t)(item / D.items_a);
                const int64_t chunk = item % D.items_a;
                pool_m = chunk * D.ppi_a;
                pool_end = pool_m + D.ppi_a;
            } else {
                // a small item, after the node's large ones
                const int64_t it = item - D.n_items_a;
                pool_node_idx = (int32_t)(it / D.items_per_node);
                const int64_t chunk = it % D.items_per_node;
                pool_m = (int64_t)D.items_a * D.ppi_a + chunk * D.ppi;
                pool_end = pool_m + D.ppi < D.M ? pool_m + D.ppi : D.M;
            }
            pool_node = D.nodes[pool_node_idx];
            const int32_t gi = pool_node % D.nx, gj = pool_node / D.nx;
            // the start node, and in FP32 its rounding remainder (the
            // compensated position starts at the node itself)
            const double sx = D.x0 + (double)gi * D.dx, sy = D.y0 + (double)gj * D.dy;
            pool_sx = (R)sx;
            pool_sy = (R)sy;
            pool_sxl = (R)(sx - (double)pool_sx);
            pool_syl = (R)(sy - (double)pool_sy);
            // a new node takes the oldest accumulator (wave-uniform branch)
            if (pool_node_idx != A.n0) {
                flush_acc(D, A.b3, A.n3);
                unsigned long long *const b = A.b3;
                A.b3 = A.b2;
                A.n3 = A.n2;
                A.b2 = A.b1;
                A.n2 = A.n1;
                A.b1 = A.b0;
                A.n1 = A.n0;
                A.b0 = b;
                A.n0 = pool_node_idx;
            }
        };
        open_item(g);

        PathState<R> P;
        start(P, (R)0, (R)0);
        Pending Qp;
        Qp.live = false;
        bool active = false;
        int32_t node = 0, node_idx = 0;
        uint32_t m = 0;
        auto flush = [&]() { deposit_parked<F>(D, Qp, A); };
        // a lane whose path finished parks it; parked paths are scored first
        // when a finishing lane still holds one, or when enough have gathered
        auto on_done = [&](bool fin, bool exited) {
            const unsigned long long done = __ballot(fin);
            if (done) {
                const unsigned long long pend = __ballot(Qp.live);
                if ((done & pend) || __popcll(done | pend) > kScoreBatch) flush();
                if (fin) {
                    park<R, kLt>(Qp, P, exited, node_idx);
                    active = false;
                }
            }
        };

        for (;;) {
            // give every idle lane the next path index, opening items as needed
            for (;;) {
                const unsigned long long need = __ballot(!active);
                if (need == 0ull) break;
                if (pool_m >= pool_end) {
                    if (!more) break;
                    const int64_t g2 = fetch_item(head);
                    if (g2 >= total) {
                        more = false;
                        break;
                    }
                    if (Q->seg_inst[find_segment(Q, nseg, g2)] != inst) {
                        carry = g2;      // another instance: drain this one first
                        more = false;
                        break;
                    }
                    open_item(g2);
                    continue;
                }
                const int64_t avail = pool_end - pool_m;
                const uint32_t rank = __builtin_amdgcn_mbcnt_hi((uint32_t)(need >> 32),
                                                                __builtin_amdgcn_mbcnt_lo((uint32_t)need, 0u));
                if (!active && (int64_t)rank < avail) {
                    m = (uint32_t)(pool_m + rank);
                    node = pool_node;
                    node_idx = pool_node_idx;
                    start(P, pool_sx, pool_sy, pool_sxl, pool_syl);
                    active = true;
                }
                const int64_t taken = (int64_t)__popcll(need);
                pool_m += taken < avail ? taken : avail;
            }
            const unsigned long long act = __ballot(active);
            if (act == 0ull) break;
            // no work left for this wave and few paths running: tail phase
            if (!(F & kFeatReflect) && !more && pool_m >= pool_end && __popcll(act) <= kTailLanes) break;
            bool fin = false, exited = false;
            LtEvents<R> ev;
            ev.bits = 0u;
            if (active) fin = advance<R, F, kLt>(D, K, P, m, (uint32_t)node, ctr3, cu, exited, &ev);
            // the trip's local-time moves join the wave's queue, in order; a
            // finishing path's moves are evaluated before its score
            if constexpr (kLt) lt_trip<R, F>(D, K, ltq, cu.ik, P, ev, fin);
            on_done(fin, exited);
        }
        if constexpr (!(F & kFeatReflect)) {
            // tail mode: the whole wave takes the remaining paths one at a
            // time (the main loop leaves only when no refill is possible)
            const int lane = threadIdx.x & (kWave - 1);
            for (;;) {
                const unsigned long long act = __ballot(active);
                if (act == 0ull) break;
                bool fin = false, exited = false;
                const int k = __popcll(act);
                if (k >= 2) {
                    // k paths at once: group g (G lanes) takes the g-th
                    int P2 = 2;
                    while (P2 < k) P2 <<= 1;
                    const int G = kWave / P2, g = lane / G;
                    // the owner of path g: the g-th set bit of act
                    unsigned long long b = act;
                    for (int r = 0; r < g && b; ++r) b &= b - 1ull;
                    const int owner = b ? __ffsll((long long)b) - 1 : 0;
                    TailPath<R> S;
                    S.x = lane_from(P.x, owner);
                    S.y = lane_from(P.y, owner);
                    S.xl = (R)0;
                    S.yl = (R)0;
                    if constexpr (sizeof(R) == 4) {
                        S.xl = lane_from(P.xl, owner);
                        S.yl = lane_from(P.yl, owner);
                    }
                    S.ar = lane_from(P.ar, owner);
                    S.ai = lane_from(P.ai, owner);
                    S.w = lane_from(P.w, owner);
                    S.t = lane_from(P.t, owner);
                    S.m = (uint32_t)lane_from((int)m, owner);
                    S.node = (uint32_t)lane_from((int)node, owner);
                    bool ex = false;
                    const bool f = tail_pass_grouped<R, F>(D, K, S, G, ctr3, cu, ex) && g < k;
                    // every active lane takes its path's results from its group's first lane
                    const int mine = __builtin_amdgcn_mbcnt_hi((uint32_t)(act >> 32),
                                                               __builtin_amdgcn_mbcnt_lo((uint32_t)act, 0u)) * G;
                    const R nx = lane_from(S.x, mine), ny = lane_from(S.y, mine);
                    R nxl = (R)0, nyl = (R)0;
                    if constexpr (sizeof(R) == 4) {
                        nxl = lane_from(S.xl, mine);
                        nyl = lane_from(S.yl, mine);
                    }
                    const double nar = lane_from(S.ar, mine), nai = lane_from(S.ai, mine), nw = lane_from(S.w, mine);
                    const int nt = lane_from(S.t, mine), nf = lane_from((int)f, mine), ne = lane_from((int)ex, mine);
                    if (active) {
                        P.x = nx;
                        P.y = ny;
                        P.xl = nxl;
                        P.yl = nyl;
                        P.ar = nar;
                        P.ai = nai;
                        P.w = nw;
                        P.t = nt;
                        fin = nf != 0;
                        exited = ne != 0;
                    }
                    on_done(fin, exited);
                    continue;
                }
                unsigned long long todo = act;
                while (todo) {
                    const int L = __ffsll((long long)todo) - 1;
                    todo &= todo - 1ull;
                    TailPath<R> S;
                    S.x = lane_value(P.x, L);
                    S.y = lane_value(P.y, L);
                    S.xl = (R)0;
                    S.yl = (R)0;
                    if constexpr (sizeof(R) == 4) {
                        S.xl = lane_value(P.xl, L);
                        S.yl = lane_value(P.yl, L);
                    }
                    S.ar = lane_value(P.ar, L);
                    S.ai = lane_value(P.ai, L);
                    S.w = lane_value(P.w, L);
                    S.t = lane_value(P.t, L);
                    S.m = lane_value(m, L);
                    S.node = lane_value((uint32_t)node, L);
                    bool ex = false;
                    const bool f = tail_pass<R, F>(D, K, S, ctr3, cu, ex);
                    if (lane == L) {
                        P.x = S.x;
                        P.y = S.y;
                        P.xl = S.xl;
                        P.yl = S.yl;
                        P.ar = S.ar;
                        P.ai = S.ai;
                        P.w = S.w;
                        P.t = S.t;
                        fin = f;
                        exited = ex;
                    }
                }
                on_done(fin, exited);
            }
        }
        flush();
        flush_acc(D, A.b0, A.n0);
        flush_acc(D, A.b1, A.n1);
        flush_acc(D, A.b2, A.n2);
        flush_acc(D, A.b3, A.n3);
    }
}

// Occupancy targets (waves per SIMD) of the path kernels; they bound the
// registers the compiler may use.  FP32 runs four waves, also where that
// spills (the reflecting kernels): at three the FP32 disc kernel spilled
// nothing but ran 4% slower, the rectangle's 10%.  FP64 runs three waves.  A second build of
// the plain FP64 kernel runs four (128 VGPRs, a small spill): 2% faster on
// the 65 x 65 cavity, whose row-major copy sits in the vector L1, but 37%
// slower on 257 x 257 with the cell-major copy, where the loop is bound by
// L2 requests; the solver takes it for row-major instances only.
#ifndef FK_WAVES_F32
#define FK_WAVES_F32 4
#endif
#ifndef FK_WAVES_F64
#define FK_WAVES_F64 3
#endif
#ifndef FK_WAVES_F64_L1
#define FK_WAVES_F64_L1 4
#endif

template <int F>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(FK_WAVES_F32)))
fk_stream_f32(const Inst *__restrict__ insts, const EngineQueue *__restrict__ Q, unsigned long long *head)
{
    stream_paths<float, F>(insts, Q, head);
}

template <int F>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(FK_WAVES_F64)))
fk_stream_f64(const Inst *__restrict__ insts, const EngineQueue *__restrict__ Q, unsigned long long *head)
{
    stream_paths<double, F>(insts, Q, head);
}

// FP32 with the row-major copy of u_n staged in LDS: one 1024-thread block
// per CU shares it (up to about 141 x 141 nodes), single-instance launches only
template <int F>
__global__ void __launch_bounds__(1024) __attribute__((amdgpu_waves_per_eu(FK_WAVES_F32)))
fk_stream_f32_lds(const Inst *__restrict__ insts, const EngineQueue *__restrict__ Q, unsigned long long *head)
{
    stream_paths<float, F | kLdsGrid>(insts, Q, head);
}

// the plain FP64 kernel at four waves, for a row-major copy in the vector L1
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(FK_WAVES_F64_L1)))
fk_stream_f64_l1(const Inst *__restrict__ insts, const EngineQueue *__restrict__ Q, unsigned long long *head)
{
    stream_paths<double, kRowMajor>(insts, Q, head);
}

// Instance lists: `which` (device, optional) names the instances by index
// into `insts`; their count is *n_dev when given (graph replays read it from
// the device), else n.
__device__ __forceinline__ int32_t list_count(int32_t n, const int32_t *n_dev) { return n_dev ? *n_dev : n; }

__global__ void fk_reset_kernel(const Inst *__restrict__ insts, const int32_t *__restrict__ which, int32_t n,
                                const int32_t *__restrict__ n_dev, unsigned long long *head)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (head && i == 0) *head = 0ull;
    if (i >= list_count(n, n_dev)) return;
    DevState *st = insts[which ? which[i] : i].state;
    st->max_du = 0ull;
    st->sup = 0ull;
    st->max_se = 0ull;
    st->path_steps = 0ull;
    st->capped = 0ull;
    st->nonfinite = 0ull;
    st->ratio_fx = 0ull;
    st->ratio_n = 0ull;
}

__device__ __forceinline__ unsigned long long bits_of(double v)
{
    return (unsigned long long)__double_as_longlong(v);
}

// One thread per interior node of instance which[blockIdx.y] (or instance
// blockIdx.y when which is null): fixed-order sum over the node's item slots,
// mean and unbiased variance, the new iterate (FP64 master and FP32 copy),
// and the instance status by atomics that do not depend on order (max of
// non-negative doubles via their bit patterns, integer sums).
// Writes the value of a grid node into the FP64 master and the gather copy.
// In the cell-major copy a node is corner dp + 2 dq of cell (gi - dp, gj - dq)
// for each of the (up to four) cells around it that exist (corner index
// 0..3 = (p,q), (p+1,q), (p,q+1), (p+1,q+1)); a node on the rectangle's edge
// has two, a corner one.
__device__ __forceinline__ void store_node(const Inst &D, int32_t node, double mr, double mi)
{
    D.u64[node] = make_double2(mr, mi);
    const int gi = node % D.nx, gj = node / D.nx, cw = D.nx - 1;
    if (D.prec == 32 && !D.cells) {
        ((float2 *)D.gather)[node] = make_float2((float)mr, (float)mi);
    } else if (D.cells) {
#pragma unroll
        for (int cq = 1; cq >= 0; --cq)
#pragma unroll
            for (int cp = 1; cp >= 0; --cp) {
                const int p = gi - cp, q = gj - cq;
                if (p < 0 || p > D.nx - 2 || q < 0 || q > D.ny - 2) continue;
                const int at = 4 * (p + cw * q) + cp + 2 * cq;
                if (D.prec == 32) ((float2 *)D.gather)[at] = make_float2((float)mr, (float)mi);
                else ((double2 *)D.gather)[at] = make_double2(mr, mi);
            }
    }
}

__global__ void __launch_bounds__(256) fk_update_kernel(const Inst *__restrict__ insts,
                                                        const int32_t *__restrict__ which,
                                                        const int32_t *__restrict__ n_dev)
{
    if (n_dev && (int32_t)blockIdx.y >= *n_dev) return;
    const Inst &D = insts[which ? which[blockIdx.y] : blockIdx.y];
    if ((int64_t)blockIdx.x * blockDim.x >= D.n_interior) return;
    const int idx = blockIdx.x * blockDim.x + threadIdx.x;
    double du = 0.0, sup = 0.0, sem = 0.0;
    long long sj = 0, nc = 0, nf = 0, rq = 0, rn = 0;
    const bool use_u = D.state->use_u != 0;
    if (idx < D.n_interior) {
        const int32_t node = D.nodes[idx];
        Slot *sl = D.slots + idx;
        // exact integer sums of the iteration; the slot is cleared for the next
        const double s_re = (double)(long long)sl->s_re_hi * 0x1p-16 + (double)sl->s_re_lo * 0x1p-56;
        const double s_im = (double)(long long)sl->s_im_hi * 0x1p-16 + (double)sl->s_im_lo * 0x1p-56;
        const double q_re = (double)sl->q_re_hi + (double)sl->q_re_lo * 0x1p-40;
        const double q_im = (double)sl->q_im_hi + (double)sl->q_im_lo * 0x1p-40;
        sj = (long long)sl->sum_j;
        nc = (long long)sl->capped;
        const unsigned long long ovf = sl->overflow;
        *sl = Slot{};
        const double Mf = (double)D.M;
        const double mr = s_re / Mf, mi = s_im / Mf;
        const double vr = fmax((q_re - s_re * mr) / (Mf - 1.0), 0.0);
        const double vi = fmax((q_im - s_im * mi) / (Mf - 1.0), 0.0);
        const double ser = sqrt(vr / Mf), sei = sqrt(vi / Mf);
        const double2 old = use_u ? D.u64[node] : make_double2(0.0, 0.0);
        store_node(D, node, mr, mi);
        D.se[node] = make_double2(ser, sei);
        D.node_sum_j[node] = sj;
        D.node_capped[node] = nc;
        du = hypot(mr - old.x, mi - old.y);
        sup = hypot(mr, mi);
        sem = hypot(ser, sei);
        // change against its Monte Carlo noise: |du|^2 / (2 |SE|^2)
        const double s2 = ser * ser + sei * sei;
        const double d2 = (mr - old.x) * (mr - old.x) + (mi - old.y) * (mi - old.y);
        if (s2 > 0.0 && isfinite(d2)) {
            rq = (long long)(fmin(d2 / (2.0 * s2), 4096.0) * 0x1p20);
            rn = 1;
        }
        if (ovf != 0ull || !(isfinite(mr) && isfinite(mi))) {
            nf = 1;
            du = HUGE_VAL;
            sup = HUGE_VAL;
        }
    }
    // block reduction: waves by shuffles, then across the block's waves
    __shared__ double r_du[4], r_sup[4], r_se[4];
    __shared__ long long r_sj[4], r_nc[4], r_nf[4], r_rq[4], r_rn[4];
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) {
        du = fmax(du, __shfl_xor(du, o, kWave));
        sup = fmax(sup, __shfl_xor(sup, o, kWave));
        sem = fmax(sem, __shfl_xor(sem, o, kWave));
        sj += __shfl_xor(sj, o, kWave);
        nc += __shfl_xor(nc, o, kWave);
        nf += __shfl_xor(nf, o, kWave);
        rq += __shfl_xor(rq, o, kWave);
        rn += __shfl_xor(rn, o, kWave);
    }
    const int w = threadIdx.x / kWave;
    if ((threadIdx.x & (kWave - 1)) == 0) {
        r_du[w] = du; r_sup[w] = sup; r_se[w] = sem;
        r_sj[w] = sj; r_nc[w] = nc; r_nf[w] = nf; r_rq[w] = rq; r_rn[w] = rn;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        const int nw = blockDim.x / kWave;
        for (int i = 1; i < nw; ++i) {
            du = fmax(du, r_du[i]); sup = fmax(sup, r_sup[i]); sem = fmax(sem, r_se[i]);
            sj += r_sj[i]; nc += r_nc[i]; nf += r_nf[i]; rq += r_rq[i]; rn += r_rn[i];
        }
        DevState *st = D.state;
        atomicMax(&st->max_du, bits_of(du));
        atomicMax(&st->sup, bits_of(sup));
        atomicMax(&st->max_se, bits_of(sem));
        atomicAdd(&st->path_steps, (unsigned long long)sj);
        atomicAdd(&st->capped, (unsigned long long)nc);
        atomicAdd(&st->nonfinite, (unsigned long long)nf);
        atomicAdd(&st->ratio_fx, (unsigned long long)rq);
        atomicAdd(&st->ratio_n, (unsigned long long)rn);
    }
}

// Disc domains: after the update, each grid node outside the disc takes the
// new value of its nearest unknown node (the pairs of D.ext), so that the
// bilinear interpolant of the next iteration reads the iterate extended
// beyond the circle in the cells the circle cuts.  Runs after the update
// kernel has finished (a launch of its own on the same stream).
__global__ void __launch_bounds__(256) fk_extend_kernel(const Inst *__restrict__ inst)
{
    const Inst &D = *inst;
    for (int32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < D.n_ext; i += gridDim.x * blockDim.x) {
        const double2 v = D.u64[D.ext[2 * i + 1]];
        store_node(D, D.ext[2 * i], v.x, v.y);
    }
}

// Advances the iteration index of each listed instance after its update.
__global__ void fk_advance_kernel(const Inst *__restrict__ insts, const int32_t *__restrict__ which, int32_t n,
                                  const int32_t *__restrict__ n_dev)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= list_count(n, n_dev)) return;
    DevState *st = insts[which ? which[i] : i].state;
    st->iter += 1;
    st->use_u = 1;
}

// ------------------------------------------- probabilistic domain decomposition
// Sec. 3's two-stage procedure: the path kernel has estimated u_{n+1} at the
// interface nodes only (the instance's node list is the interface); the
// update kernel has written them.  Every block of unknown nodes between the
// interface lines is then the Dirichlet problem
//   (Delta_h - (alpha - k^2)) u_{n+1} = f - (alpha + i p) u_n
// with the 5-point Laplacian, the interface values and the edge data g as
// boundary values.  The 5-point Laplacian of an mx x my block is
// S_x L_x S_x (x) + S_y L_y S_y (y) with the orthonormal DST-I matrices
// S_m[a][b] = sqrt(2/(m+1)) sin(pi (a+1)(b+1)/(m+1)) (symmetric, S_m^2 = I)
// and L_m = -(4/h^2) sin^2(pi (p+1)/(2(m+1))), so
//   u = S_x ((S_x r S_y) / (L_x[p] + L_y[q] - (alpha - k^2))) S_y.
// Tables per block size m (host-built): 2(m+1) values sqrt(2/(m+1))
// sin(pi t/(m+1)) (entry S[a][b] is t = (a+1)(b+1) mod 2(m+1)), then m
// values 4 sin^2(pi (p+1)/(2(m+1))).

__device__ __forceinline__ double comp_of(double2 v, int c) { return c ? v.y : v.x; }

// Right-hand side of every block node (both components); workgroups loop
// over the tasks.  Kept apart from the solve, which overwrites u_n.
__global__ void __launch_bounds__(256) fk_pdd_rhs_kernel(const Inst *__restrict__ insts,
                                                         const PddTask *__restrict__ tasks, int32_t n_tasks,
                                                         const int32_t *__restrict__ n_dev)
{
    const int32_t count = list_count(n_tasks, n_dev);
    for (int32_t t = blockIdx.x; t < count; t += gridDim.x) {
        const PddTask B = tasks[t];
        const Inst &D = insts[B.inst];
        const int mx = B.i1 - B.i0, my = B.j1 - B.j0, n = mx * my;
        const double idx2 = D.idx * D.idx, idy2 = D.idy * D.idy;
        const bool use_u = D.state->use_u != 0;
        for (int e = threadIdx.x; e < n; e += blockDim.x) {
            const int a = e / my, b = e - (e / my) * my;
            const int gi = B.i0 + a, gj = B.j0 + b;
            const int node = gi + D.nx * gj;
            double rr = 0.0, ri = 0.0;
            if (D.src_kind == SRC_CONST) {
                rr = D.src_re;
                ri = D.src_im;
            } else if (D.src_kind == SRC_GAUSSIAN) {
                const double ex = D.x0 + (double)gi * D.dx - D.src_cx, ey = D.y0 + (double)gj * D.dy - D.src_cy;
                const double g = exp(-D.src_c * (ex * ex + ey * ey));
                rr = D.src_re * g;
                ri = D.src_im * g;
            }
            if (use_u) {
                const double2 u = D.u64[node];
                rr -= D.alpha * u.x - D.damp * u.y;
                ri -= D.alpha * u.y + D.damp * u.x;
            }
            // Dirichlet neighbours outside the block: interface values of
            // u_{n+1} (already written) or the edge data
            if (a == 0) { const double2 v = D.u64[node - 1]; rr -= idx2 * v.x; ri -= idx2 * v.y; }
            if (a == mx - 1) { const double2 v = D.u64[node + 1]; rr -= idx2 * v.x; ri -= idx2 * v.y; }
            if (b == 0) { const double2 v = D.u64[node - D.nx]; rr -= idy2 * v.x; ri -= idy2 * v.y; }
            if (b == my - 1) { const double2 v = D.u64[node + D.nx]; rr -= idy2 * v.x; ri -= idy2 * v.y; }
            B.rhs[node] = make_double2(rr, ri);
        }
    }
}

// One (task, component) at a time per workgroup (component blockIdx.y): r
// and a work array of mx * my doubles in LDS (at most 64 x 64: 64 KiB), four
// dense products with the DST tables.  Writes the component into the FP64
// iterate and the gather copy.
__global__ void __launch_bounds__(256) fk_pdd_solve_kernel(const Inst *__restrict__ insts,
                                                           const PddTask *__restrict__ tasks, int32_t n_tasks,
                                                           const int32_t *__restrict__ n_dev)
{
    extern __shared__ double lds_pdd[];
    const int comp = blockIdx.y;
    const int32_t count = list_count(n_tasks, n_dev);
    for (int32_t t = blockIdx.x; t < count; t += gridDim.x) {
        const PddTask B = tasks[t];
        const Inst &D = insts[B.inst];
        const int mx = B.i1 - B.i0, my = B.j1 - B.j0, n = mx * my;
        const int px = 2 * (mx + 1), py = 2 * (my + 1);
        const double *sx = B.tx, *sy = B.ty;                  // sines
        const double *ex = sx + px, *ey = sy + py;            // eigenvalue factors
        double *R = lds_pdd, *T = lds_pdd + n;
        __syncthreads();   // the previous task's last reads of T are done
        for (int e = threadIdx.x; e < n; e += blockDim.x) {
            const int a = e / my, b = e - (e / my) * my;
            R[e] = comp_of(B.rhs[(B.i0 + a) + D.nx * (B.j0 + b)], comp);
        }
        __syncthreads();
        // T = R S_y
        for (int e = threadIdx.x; e < n; e += blockDim.x) {
            const int a = e / my, q = e - (e / my) * my;
            double acc = 0.0;
            for (int b = 0; b < my; ++b) acc = fma(R[a * my + b], sy[((b + 1) * (q + 1)) % py], acc);
            T[e] = acc;
        }
        __syncthreads();
        // R = S_x T, divided by the eigenvalue of (Delta_h - c)
        const double idx2 = D.idx * D.idx, idy2 = D.idy * D.idy, c = D.alpha - D.k2;
        for (int e = threadIdx.x; e < n; e += blockDim.x) {
            const int p = e / my, q = e - (e / my) * my;
            double acc = 0.0;
            for (int a = 0; a < mx; ++a) acc = fma(sx[((p + 1) * (a + 1)) % px], T[a * my + q], acc);
            R[e] = acc / (-(idx2 * ex[p] + idy2 * ey[q]) - c);
        }
        __syncthreads();
        // T = S_x R
        for (int e = threadIdx.x; e < n; e += blockDim.x) {
            const int a = e / my, q = e - (e / my) * my;
            double acc = 0.0;
            for (int p = 0; p < mx; ++p) acc = fma(sx[((a + 1) * (p + 1)) % px], R[p * my + q], acc);
            T[e] = acc;
        }
        __syncthreads();
        // u = T S_y, into the iterate and its gather copy
        const int cw = D.nx - 1;
        for (int e = threadIdx.x; e < n; e += blockDim.x) {
            const int a = e / my, b = e - (e / my) * my;
            double v = 0.0;
            for (int q = 0; q < my; ++q) v = fma(T[a * my + q], sy[((q + 1) * (b + 1)) % py], v);
            const int gi = B.i0 + a, gj = B.j0 + b;
            const int node = gi + D.nx * gj;
            ((double *)D.u64)[2 * node + comp] = v;
            if (D.prec == 32 && !D.cells) {
                ((float *)D.gather)[2 * node + comp] = (float)v;
            } else if (D.cells) {
                for (int cq = 1; cq >= 0; --cq)
                    for (int cp = 1; cp >= 0; --cp) {
                        const int p = gi - cp, q = gj - cq;
                        if (p < 0 || p > D.nx - 2 || q < 0 || q > D.ny - 2) continue;
                        const int at = 4 * (p + cw * q) + cp + 2 * cq;
                        if (D.prec == 32) ((float *)D.gather)[2 * at + comp] = (float)v;
                        else ((double *)D.gather)[2 * at + comp] = v;
                    }
            }
        }
    }
}

// ------------------------------------------------------------------ debug

__global__ void fk_debug_philox_kernel(uint32_t k0, uint32_t k1, const uint4 *__restrict__ ctr, int64_t n,
                                       uint4 *__restrict__ out)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const uint4 c = ctr[i];
    out[i] = philox4x32_10(c.x, c.y, c.z, c.w, k0, k1);
}

template <class R>
__global__ void fk_debug_normals_kernel(const uint2 *__restrict__ words, int64_t n, double2 *__restrict__ z)
{
    __shared__ typename TablesOf<R>::type tables;
    setup_tables<R>(tables);
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    R zx, zy;
    normals(words[i].x, words[i].y, tables, zx, zy);
    z[i] = make_double2((double)zx, (double)zy);
}

// One lane per listed path, same step code as the item kernels.
template <class R>
__global__ void fk_debug_paths_kernel(const Inst *__restrict__ inst, const int32_t *__restrict__ nodes,
                                      const int64_t *__restrict__ ms, int64_t n, long long *__restrict__ J,
                                      double2 *__restrict__ score_out, double2 *__restrict__ xj)
{
    __shared__ typename TablesOf<R>::type tables;
    setup_tables<R>(tables);
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const Inst &D = *inst;
    const Consts<R> K(D, &tables);
    const bool use_u = D.state->use_u != 0;
    Coef<R> cu;
    cu.re = use_u ? K.alpha : (R)0;
    cu.im = use_u ? K.damp : (R)0;
    cu.ik = use_u ? K.kk : (R)0;
    const uint32_t ctr3 = D.crn ? 0u : (uint32_t)D.state->iter;
    if (i >= n) return;
    const int32_t node = nodes[i];
    const int32_t gi = node % D.nx, gj = node / D.nx;
    PathState<R> P;
    const double sx = D.x0 + (double)gi * D.dx, sy = D.y0 + (double)gj * D.dy;
    start(P, (R)sx, (R)sy, (R)(sx - (double)(R)sx), (R)(sy - (double)(R)sy));
    bool exited = false;
    if (D.curved) {
        while (!advance<R, kFeatAll | kFeatCurved>(D, K, P, (uint32_t)ms[i], (uint32_t)node, ctr3, cu, exited)) {
        }
    } else {
        while (!advance<R, kFeatAll>(D, K, P, (uint32_t)ms[i], (uint32_t)node, ctr3, cu, exited)) {
        }
    }
    J[i] = P.t;
    Pending Q;
    park<R>(Q, P, exited, 0);
    // the rhombus hole's projection is compiled only with the curved edge
    score_out[i] = D.curved ? score<kFeatAll | kFeatCurved>(D, Q) : score<kFeatAll>(D, Q);
    if constexpr (sizeof(R) == 4)
        xj[i] = make_double2((double)P.x + (double)P.xl, (double)P.y + (double)P.yl);
    else
        xj[i] = make_double2((double)P.x, (double)P.y);
}

}  // namespace fkd

// ------------------------------------------------------------ launchers

namespace fkk {
using namespace fkd;

static int blocks_for(int64_t n, int per) { return (int)((n + per - 1) / per); }

template <int F>
static void launch_stream_f(int precision, dim3 grid, dim3 block, const Inst *d_insts, const EngineQueue *Q,
                            unsigned long long *head, hipStream_t s)
{
    if (precision == 32)
        hipLaunchKernelGGL(fk_stream_f32<F>, grid, block, 0, s, d_insts, Q, head);
    else
        hipLaunchKernelGGL(fk_stream_f64<F>, grid, block, 0, s, d_insts, Q, head);
}

template <int F>
static hipError_t launch_lds(const Inst *d_insts, const EngineQueue *Q, unsigned long long *head, int n_blocks,
                             size_t lds_bytes, hipStream_t s)
{
    hipError_t e = hipFuncSetAttribute((const void *)fk_stream_f32_lds<F>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                       (int)lds_bytes);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(fk_stream_f32_lds<F>, dim3(n_blocks), dim3(1024), lds_bytes, s, d_insts, Q, head);
    return hipGetLastError();
}

hipError_t launch_stream(int precision, int features, const Inst *d_insts, const EngineQueue *Q,
                         unsigned long long *head, int n_blocks, hipStream_t s, bool l1_grid, size_t lds_bytes)
{
    if (precision == 32 && lds_bytes > 0 && (features & kFeatReflect) == 0) {
        // the same waves in 1024-thread blocks (four 256-thread blocks each)
        const int nb = n_blocks / 4 > 0 ? n_blocks / 4 : 1;
        switch (features & kFeatAll) {
        case 0: return launch_lds<0>(d_insts, Q, head, nb, lds_bytes, s);
        case 1: return launch_lds<1>(d_insts, Q, head, nb, lds_bytes, s);
        case 2: return launch_lds<2>(d_insts, Q, head, nb, lds_bytes, s);
        case 3: return launch_lds<3>(d_insts, Q, head, nb, lds_bytes, s);
        case 4: return launch_lds<4>(d_insts, Q, head, nb, lds_bytes, s);
        case 5: return launch_lds<5>(d_insts, Q, head, nb, lds_bytes, s);
        case 6: return launch_lds<6>(d_insts, Q, head, nb, lds_bytes, s);
        default: return launch_lds<7>(d_insts, Q, head, nb, lds_bytes, s);
        }
    }
    dim3 grid(n_blocks), block(256);
    if (features & kFeatCurved) {
        // disc domains: a hole and the reflecting edge always
        switch (features & kFeatAll) {
        case 9: launch_stream_f<9 | kFeatCurved>(precision, grid, block, d_insts, Q, head, s); break;
        case 11: launch_stream_f<11 | kFeatCurved>(precision, grid, block, d_insts, Q, head, s); break;
        case 13: launch_stream_f<13 | kFeatCurved>(precision, grid, block, d_insts, Q, head, s); break;
        default: launch_stream_f<15 | kFeatCurved>(precision, grid, block, d_insts, Q, head, s); break;
        }
        return hipGetLastError();
    }
    if (precision == 64 && (features & kFeatAll) == 0 && l1_grid) {
        hipLaunchKernelGGL(fk_stream_f64_l1, grid, block, 0, s, d_insts, Q, head);
        return hipGetLastError();
    }
    // a reflecting edge comes with a hole: the sets with bit 3 all have bit 0
    switch (features & kFeatAll) {
    case 0: launch_stream_f<0>(precision, grid, block, d_insts, Q, head, s); break;
    case 1: launch_stream_f<1>(precision, grid, block, d_insts, Q, head, s); break;
    case 2: launch_stream_f<2>(precision, grid, block, d_insts, Q, head, s); break;
    case 3: launch_stream_f<3>(precision, grid, block, d_insts, Q, head, s); break;
    case 4: launch_stream_f<4>(precision, grid, block, d_insts, Q, head, s); break;
    case 5: launch_stream_f<5>(precision, grid, block, d_insts, Q, head, s); break;
    case 6: launch_stream_f<6>(precision, grid, block, d_insts, Q, head, s); break;
    case 7: launch_stream_f<7>(precision, grid, block, d_insts, Q, head, s); break;
    case 9: launch_stream_f<9>(precision, grid, block, d_insts, Q, head, s); break;
    case 11: launch_stream_f<11>(precision, grid, block, d_insts, Q, head, s); break;
    case 13: launch_stream_f<13>(precision, grid, block, d_insts, Q, head, s); break;
    default: launch_stream_f<15>(precision, grid, block, d_insts, Q, head, s); break;
    }
    return hipGetLastError();
}

hipError_t launch_reset(const Inst *d_insts, const int32_t *which, int32_t n, const int32_t *n_dev,
                        unsigned long long *head, hipStream_t s)
{
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(fk_reset_kernel, dim3(blocks_for(n, 64)), dim3(64), 0, s, d_insts, which, n, n_dev, head);
    return hipGetLastError();
}

hipError_t launch_update(const Inst *d_insts, const int32_t *which, int32_t n_inst, const int32_t *n_dev,
                         int32_t max_interior, hipStream_t s)
{
    if (n_inst <= 0 || max_interior <= 0) return hipSuccess;
    hipLaunchKernelGGL(fk_update_kernel, dim3(blocks_for(max_interior, 256), n_inst), dim3(256), 0, s, d_insts,
                       which, n_dev);
    return hipGetLastError();
}

hipError_t launch_extend(const Inst *d_inst, int32_t n_ext, hipStream_t s)
{
    if (n_ext <= 0) return hipSuccess;
    const int nb = blocks_for(n_ext, 256) < 1024 ? blocks_for(n_ext, 256) : 1024;
    hipLaunchKernelGGL(fk_extend_kernel, dim3(nb), dim3(256), 0, s, d_inst);
    return hipGetLastError();
}

hipError_t launch_advance(const Inst *d_insts, const int32_t *which, int32_t n, const int32_t *n_dev, hipStream_t s)
{
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(fk_advance_kernel, dim3(blocks_for(n, 64)), dim3(64), 0, s, d_insts, which, n, n_dev);
    return hipGetLastError();
}

hipError_t launch_pdd(const Inst *d_insts, const PddTask *tasks, int32_t n, const int32_t *n_dev, int32_t grid,
                      int32_t max_nodes, hipStream_t s)
{
    if ((n <= 0 && !n_dev) || grid <= 0) return hipSuccess;
    hipLaunchKernelGGL(fk_pdd_rhs_kernel, dim3(grid), dim3(256), 0, s, d_insts, tasks, n, n_dev);
    hipLaunchKernelGGL(fk_pdd_solve_kernel, dim3(grid, 2), dim3(256), (size_t)2 * max_nodes * sizeof(double), s,
                       d_insts, tasks, n, n_dev);
    return hipGetLastError();
}

hipError_t launch_debug_philox(uint32_t k0, uint32_t k1, const uint4 *ctr, int64_t n, uint4 *out, hipStream_t s)
{
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(fk_debug_philox_kernel, dim3(blocks_for(n, 256)), dim3(256), 0, s, k0, k1, ctr, n, out);
    return hipGetLastError();
}

hipError_t launch_debug_normals(int precision, const uint2 *words, int64_t n, double2 *z, hipStream_t s)
{
    if (n <= 0) return hipSuccess;
    if (precision == 32)
        hipLaunchKernelGGL(fk_debug_normals_kernel<float>, dim3(blocks_for(n, 256)), dim3(256), 0, s, words, n, z);
    else
        hipLaunchKernelGGL(fk_debug_normals_kernel<double>, dim3(blocks_for(n, 256)), dim3(256), 0, s, words, n, z);
    return hipGetLastError();
}

hipError_t launch_debug_paths(int precision, const Inst *d_inst, const int32_t *nodes, const int64_t *ms, int64_t n,
                              long long *J, double2 *score, double2 *xj, hipStream_t s)
{
    if (n <= 0) return hipSuccess;
    if (precision == 32)
        hipLaunchKernelGGL(fk_debug_paths_kernel<float>, dim3(blocks_for(n, 64)), dim3(64), 0, s, d_inst, nodes, ms,
                           n, J, score, xj);
    else
        hipLaunchKernelGGL(fk_debug_paths_kernel<double>, dim3(blocks_for(n, 64)), dim3(64), 0, s, d_inst, nodes,
                           ms, n, J, score, xj);
    return hipGetLastError();
}

}  // namespace fkk
