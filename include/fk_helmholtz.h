/*
 * fk_helmholtz.h -- C ABI of the MI355X (gfx950) Monte Carlo Feynman-Kac
 * solver for the fixed-point Helmholtz iteration.
 *
 * The method (Bernal, Chen, dos Reis, "An iterative method for Helmholtz
 * boundary value problems arising in wave propagation"):
 *   Delta u + k^2 u = f in Omega, u = g on dOmega (Sec. 1 eq. (1.1); Sec. 2.2
 *   eq. (2.4) with damping p = 0 and no reflecting boundary part) is solved as
 *   the sequence of Poisson problems  Delta u_{n+1} = f - k^2 u_n,
 *   u_{n+1} = g on dOmega, u_0 = 0 (the shift alpha = k^2 of eq. (1.4); the
 *   partial sums in the proof of Theorem 2.2).  Each Poisson step is solved at
 *   every unknown grid node y by the Feynman-Kac formula of Sec. 2.1 eq. (2.3)
 *   with c = 0:  u_{n+1}(y) = E[g(Y_tau)] - E[int_0^tau (f - k^2 u_n)(Y_t) dt],
 *   Y = y + sqrt(2) W, averaged over M paths that are independent for every n
 *   (Remark 2.1).  The iteration converges when k^2 is below the first
 *   Dirichlet eigenvalue (Sec. 2.4, Remark 2.4); it is stopped by the
 *   sup-norm change (Sec. 3).
 *
 *   With a reflecting edge (the annular problem of Sec. 2.3) the rectangle's
 *   edge carries the Robin condition d_n u - i k u = g2 and only the hole is
 *   absorbing: Y is the diffusion reflected at the edge, dY = sqrt(2) dW -
 *   n dxi with local time xi (Sec. 2.1 eqs. (2.1)-(2.3)), and each step adds
 *   E[int_0^tau e^{-(alpha - k^2) t} (i k u_n + g2)(Y_t) dxi_t] (the partial
 *   sums of the iteration of Sec. 2.3 satisfy d_n u_{n+1} = i k u_n + g2).
 *   The sufficient condition for convergence is alpha E[tau] + k E[xi] < 1
 *   (Theorem 2.3).
 *
 * Discretisation: Euler-Maruyama with step h; normals by Box-Muller from
 * Philox4x32-10 words, key = seed, counter = (t/2, path m, node id, n) (n
 * replaced by 0 when crn != 0); uniform U(r) = (2 (r >> 9) + 1) 2^-24; exit at
 * the first step outside the open domain, boundary datum at the nearest
 * boundary point; left-point rule for the integral; u_n read by bilinear
 * interpolation of the grid.  Reflecting edge: after each step a coordinate
 * that left the rectangle is mirrored back across the face it crossed; the
 * local time grows by twice the overshoot, and the local-time integrand is
 * taken at the foot of the mirror move on the face, discounted to the end of
 * the step; the step is absorbed when the point lies in the closed hole.
 *
 * Conventions for every entry point:
 *   - Grids are row-major nx * ny, node (i, j) at index i + nx * j, x fastest;
 *     complex values are interleaved (re, im) doubles.
 *   - Host pointers unless the argument says "device".  The library copies
 *     what it needs from host inputs before returning.
 *   - Every call returns an fk_status; nothing is thrown across the ABI.  On
 *     failure fk_helmholtz_last_error() returns a message (thread-local,
 *     valid until the next call on that thread).
 *   - A solver handle is not thread-safe; distinct handles may be used from
 *     distinct threads on distinct streams.
 *   - hip_stream is a hipStream_t (NULL = the null stream).  All device work
 *     of a handle is ordered on that stream.
 */
#ifndef FK_HELMHOLTZ_H
#define FK_HELMHOLTZ_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    FK_OK = 0,
    FK_EINVAL = 1,         /* invalid argument: geometry, sizes, parameters   */
    FK_ENOMEM = 2,         /* arena too small / allocation failed             */
    FK_EDEVICE = 3,        /* a HIP runtime call failed                       */
    FK_EDIVERGED = 4,      /* divergence rule fired (result still readable)   */
    FK_ENOTCONVERGED = 5,  /* max_iters reached above tol (result readable)   */
    FK_EBUSY = 6,          /* engine: no free slot                            */
    FK_ECANCELLED = 7      /* fk_helmholtz_cancel stopped the call (result
                              readable: the last completed iterate)       */
} fk_status;

/* Omega: the open rectangle (x0,x1) x (y0,y1); for RECT_MINUS_DISC also
 * minus the closed disc of radius r at (cx, cy); for RECT_MINUS_BOX minus the
 * closed box [cx - r, cx + r] x [cy - ry, cy + ry].  The hole must lie
 * strictly inside the rectangle.  nx, ny >= 3 nodes per side, edges
 * included.  A grid node within 1e-9 grid steps of the box counts as in it
 * (so a box drawn on grid lines keeps its edge nodes whatever the rounding
 * of x0 + i dx).
 *
 * edge: ABSORBING, u = g_outer on the rectangle's edge (Dirichlet); or
 * REFLECTING, d_n u - i k u = g_outer on the edge (Robin, Sec. 2.3): the
 * edge nodes are unknowns, the paths are reflected there and only the hole
 * absorbs them, so a reflecting edge needs a hole, an explicit step cap
 * (fk_params.max_steps) and sides longer than 6 sqrt(2 h).
 *
 * DISC_MINUS_RHOMBUS / DISC_MINUS_DISC (the annular domains of Sec. 2.5 with
 * a disc as the outer boundary): Omega is the open disc inscribed in the
 * square [x0, x1] x [y0, y1] (x1 - x0 = y1 - y0) minus the closed rhombus
 * |x - cx| / r + |y - cy| / ry <= 1 (a node within 1e-9 of its edge counts
 * as in it) or minus the closed disc of radius r at (cx, cy), strictly
 * inside.  The disc's edge reflects (edge = REFLECTING, with the Robin
 * datum g_outer): a path past the circle is mirrored radially, the local
 * time grows by twice the overshoot, the datum is taken at the move's foot
 * on the circle (outward normal radial).  Grid nodes outside the closed disc
 * are exterior: no unknowns; each carries the value of its nearest unknown
 * node (fk_helmholtz_exterior_nodes), so that the bilinear interpolant of
 * the iterate in the cells the circle cuts reads the iterate extended beyond
 * the circle.  Any k, alpha and damping; FP64 or FP32 stepping (FP32: the
 * compensated position is tested and mirrored at the circle in FP64); the
 * single-instance solver and fk_helmholtz_step_static (fk_engine_add rejects
 * them). */
typedef enum {
    FK_DOMAIN_RECT = 0, FK_DOMAIN_RECT_MINUS_DISC = 1, FK_DOMAIN_RECT_MINUS_BOX = 2,
    FK_DOMAIN_DISC_MINUS_RHOMBUS = 3, FK_DOMAIN_DISC_MINUS_DISC = 4
} fk_domain_kind;
typedef enum { FK_EDGE_ABSORBING = 0, FK_EDGE_REFLECTING = 1 } fk_edge_kind;
typedef struct {
    int32_t kind;
    int32_t nx, ny;
    int32_t edge;          /* fk_edge_kind */
    double x0, x1, y0, y1;
    double cx, cy, r;
    double ry;             /* RECT_MINUS_BOX: half-height of the box */
} fk_domain;

/* Source f: ZERO; CONST f = amp; GAUSSIAN f = amp exp(-|x-c|^2 / (2 sigma^2)). */
typedef enum { FK_SRC_ZERO = 0, FK_SRC_CONST = 1, FK_SRC_GAUSSIAN = 2 } fk_source_kind;
typedef struct {
    int32_t kind;
    int32_t reserved;
    double amp_re, amp_im, cx, cy, sigma;
} fk_source;

/* Datum on one boundary part: the Dirichlet value g, or on a reflecting
 * edge the Robin datum g2 of d_n u - i k u = g2.
 *   PLANE_WAVE  c = {amp_re, amp_im, theta}: g = amp exp(i kappa (x cos th + y sin th)),
 *               kappa = sqrt(k^2 + i p) (k without damping)
 *   BILINEAR    c = {c0re, c0im, c1re, c1im, c2re, c2im, c3re, c3im}:
 *               g = c0 + c1 x + c2 y + c3 x y
 *   TABLE       (outer boundary only) table_len complex samples (re, im
 *               interleaved; host pointer, copied at create) at equal
 *               arclength steps round the rectangle, counter-clockwise from
 *               (x0, y0), linearly interpolated, periodic.
 *   PLANE_WAVE_ROBIN  (reflecting edge only) c as PLANE_WAVE: the Robin
 *               datum of that plane wave w, g2 = d_n w - i k w
 *               = i (kappa (n . (cos th, sin th)) - k) w with n the face's
 *               outward normal, so that w solves the Robin problem.
 * On hole nodes the grid carries the inner datum's own formula (a smooth
 * extension); TABLE and PLANE_WAVE_ROBIN are not allowed there. */
typedef enum {
    FK_BC_ZERO = 0, FK_BC_PLANE_WAVE = 1, FK_BC_BILINEAR = 2, FK_BC_TABLE = 3, FK_BC_PLANE_WAVE_ROBIN = 4
} fk_bc_kind;
typedef struct {
    int32_t kind;
    int32_t reserved;
    double c[8];
    const double *table;
    int64_t table_len;
} fk_bc;

/* Layout of the copy of the iterate read by the bilinear gather.
 * NODES: row-major nodes (the cell's two rows are two cache lines); the
 *        FP32 path reads an FP32 copy (8 B per node), the FP64 path the
 *        FP64 master itself.
 * CELLS: per cell (p, q) the four corners u(p,q), u(p+1,q), u(p,q+1),
 *        u(p+1,q+1) in one block: 32 B per cell (FP32) or 64 B (FP64), one
 *        cache line per step, 4x the bytes.
 * AUTO:  NODES while the row-major data fit the vector L1 cache (80 KiB),
 *        CELLS above.  The interpolated values are identical. */
typedef enum { FK_GATHER_AUTO = 0, FK_GATHER_NODES = 1, FK_GATHER_CELLS = 2 } fk_gather_layout;

typedef struct {
    double k;              /* wavenumber (real, >= 0)                          */
    double h;              /* Euler-Maruyama time step (> 0)                  */
    int64_t M;             /* paths per node per iteration (>= 2)             */
    uint64_t seed;         /* Philox key                                       */
    int32_t precision;     /* 64: FP64 stepping; 32: FP32 stepping with
                              compensated sums (node sums always FP64)        */
    int32_t max_iters;     /* for fk_helmholtz_solve                          */
    double tol;            /* stop when max |u_{n+1} - u_n| < tol (0: never)  */
    int64_t max_steps;     /* step cap per path; 0 = ceil(40/(lambda1 h)),
                              lambda1 of the bounding rectangle (absorbing
                              edge only: a reflecting edge needs it set)     */
    int32_t crn;           /* 1: same paths every iteration (counter n -> 0)  */
    int32_t g_unprojected; /* verification variant: g at X_J itself           */
    int32_t paths_per_item;/* paths per wavefront work item; 0 = auto         */
    int32_t gather_layout; /* layout of the copy of u_n that the paths read
                              (fk_gather_layout)                           */
    int32_t waves_per_cu;  /* single-instance solver: resident waves of the
                              path kernel per CU, a multiple of 4 in [4, 32];
                              0 = 16.  (The engine takes it from its config.) */
    int32_t reserved;      /* must be 0 */
    double alpha;          /* shift of the iteration, >= k^2; 0 = k^2.  With
                              damping p the equation is
                              Delta u + (k^2 + i p) u = f and the iteration
                              Delta U_{n+1} - (alpha - k^2) U_{n+1}
                                = f - (alpha + i p) U_n  (Sec. 2.2, the
                              partial sums of (2.6)-(2.8)); each step is a
                              Feynman-Kac solve with killing rate
                              alpha - k^2                                   */
    double damping;        /* p >= 0; plane-wave data then use the wavenumber
                              sqrt(k^2 + i p)                               */
} fk_params;

/* Per-iteration report (after the iteration that produced u_n). */
typedef struct {
    int32_t n;             /* iterations completed (index of the iterate)     */
    int32_t diverging;     /* divergence rule fired at this iteration          */
    double max_du;         /* max over unknown nodes |u_n - u_{n-1}|           */
    double sup;            /* max over unknown nodes |u_n|                     */
    double max_se;         /* max node standard error (|SE_re + i SE_im|)      */
    double noise_floor;    /* 4 * max_se                                       */
    int64_t path_steps;    /* sum of exit-step indices over all paths          */
    int64_t capped;        /* paths stopped by the step cap                    */
    int64_t nonfinite;     /* nodes whose estimate is not finite               */
    double step_ms;        /* device time of the path kernel (HIP events)      */
    double noise_ratio;    /* mean over unknown nodes of |u_n - u_{n-1}|^2 /
                              (2 |SE_n|^2), each node's term capped at 4096:
                              about 1/(1+rho) once the change is Monte Carlo
                              noise alone (fresh paths), large while the
                              iterate still contracts                       */
} fk_iter_report;

typedef struct fk_solver fk_solver;

/* Device bytes a solver needs for this problem (the arena size to pass to
 * fk_helmholtz_create).  g_outer may be NULL unless it is a TABLE. */
fk_status fk_helmholtz_arena_bytes(const fk_domain *domain, const fk_bc *g_outer,
                                   const fk_params *params, size_t *bytes);

/* The work items a solver launches for this problem (the persistent stream
 * kernel's queue).  Every unknown node's M paths are split into
 * *items_large items of *paths_large paths first (0 and 0 when the caller
 * fixed paths_per_item, or when too few nodes would share them), then
 * *items_small items of up to *paths_small paths; *n_items = unknown nodes x
 * (*items_large + *items_small).  The queue hands out every large item before
 * the first small one.  Host-only like fk_helmholtz_arena_bytes; g_outer may
 * be NULL unless it is a TABLE; any output pointer may be NULL.  The split
 * never changes results (node sums are exact integers). */
fk_status fk_helmholtz_work_items(const fk_domain *domain, const fk_bc *g_outer, const fk_params *params,
                                  int64_t *n_items, int32_t *paths_large, int32_t *items_large,
                                  int32_t *paths_small, int32_t *items_small);

/* Disc domains (Sec. 2.5's annular problems with a disc as the outer
 * boundary): the grid nodes outside the disc and, for each, the unknown node
 * whose value it carries in the iterate (its nearest unknown node; ties: the
 * lowest node id), so that the bilinear interpolant reads the iterate
 * extended beyond the circle in the cells the circle cuts.  *n_pairs
 * receives their count; pairs (host, may be NULL) receives 2 *n_pairs ints
 * (exterior node id, unknown node id) when cap >= *n_pairs.  Other domains:
 * *n_pairs = 0.  Host-only like fk_helmholtz_arena_bytes; g_outer may be
 * NULL unless it is a TABLE.  FK_EINVAL: an invalid problem, n_pairs NULL,
 * or pairs given with cap < *n_pairs (*n_pairs is still set). */
fk_status fk_helmholtz_exterior_nodes(const fk_domain *domain, const fk_bc *g_outer, const fk_params *params,
                                      int32_t *pairs, int64_t cap, int64_t *n_pairs);

/* Validates the problem, classifies the grid nodes (unknown: interior or on
 * a reflecting edge; absorbing edge; hole), uploads the boundary data and
 * sets u_0 = 0.  device_arena: device memory of at least
 * fk_helmholtz_arena_bytes bytes, 256-byte aligned, owned by the caller and
 * kept alive until destroy; NULL makes the library allocate (and free) its
 * own.  FK_EINVAL: bad geometry, nx or ny < 3, h <= 0, M < 2, precision not
 * 32/64, hole not strictly inside, TABLE or PLANE_WAVE_ROBIN as inner datum,
 * PLANE_WAVE_ROBIN on an absorbing edge, table_len < 2, a reflecting edge
 * without a hole, without max_steps, with g_unprojected or with a side not
 * longer than 6 sqrt(2 h); a disc domain in a box that is not square, with
 * an absorbing edge, with a diameter not longer than 12 sqrt(2 h) or with no
 * unknown node.  FK_ENOMEM: arena too small. */
fk_status fk_helmholtz_create(const fk_domain *domain, const fk_source *f, const fk_bc *g_outer,
                              const fk_bc *g_inner, const fk_params *params, void *device_arena,
                              size_t arena_bytes, void *hip_stream, fk_solver **out);

/* Runs n_iters fixed-point iterations on the device (u_n -> u_{n+1}: one
 * Feynman-Kac solve at every unknown node, then the update of the iterate)
 * and fills *last (may be NULL) with the report of the last one.  Returns
 * FK_EDIVERGED as soon as the divergence rule fires: the change is not
 * finite, or five iterations apart both max |u| and max |du| grew by 25%. */
fk_status fk_helmholtz_iterate(fk_solver *s, int32_t n_iters, fk_iter_report *last);

/* Iterates until max |du| < tol or max_iters iterations in total (Sec. 3's
 * sup-norm control).  FK_ENOTCONVERGED if tol > 0 was not reached. */
fk_status fk_helmholtz_solve(fk_solver *s, fk_iter_report *final_report);

/* Asks the fk_helmholtz_iterate or fk_helmholtz_solve call running on s (in
 * another thread), or else the next such call, to stop before its next
 * iteration: that call returns FK_ECANCELLED with the report of the last
 * completed iteration, the iterate stays readable and a later call resumes
 * the run (the same results as without the stop: the random numbers depend
 * only on the iteration index).  The request is taken by that one call.  The
 * only entry point that may be called concurrently with others on the same
 * handle (not with or after fk_helmholtz_destroy). */
fk_status fk_helmholtz_cancel(fk_solver *s);

/* Copies the current iterate u_n (nx*ny complex; a disc domain's exterior
 * nodes hold their nearest unknown node's value) and, if se_reim is not NULL,
 * the per-node standard errors (SE_re, SE_im; 0 on nodes that are not
 * unknowns) of the last iteration.  on_device != 0: the pointers are device pointers. */
fk_status fk_helmholtz_get(fk_solver *s, double *u_reim, double *se_reim, int32_t on_device);

/* Per-node sum of exit-step indices and capped-path counts of the last
 * iteration (nx*ny each, host pointers; 0 on nodes that are not unknowns). */
fk_status fk_helmholtz_node_stats(fk_solver *s, int64_t *sum_j, int64_t *capped);

/* Replaces the iterate by u_reim (nx*ny complex, host or device) on unknown
 * nodes and sets the iteration index to n (the next iteration uses counter
 * word n).  Absorbing-edge and hole nodes keep their data; a disc domain's
 * exterior nodes take their nearest unknown node's value.  Used to resume from a
 * checkpoint and to feed the same u_n to another implementation. */
fk_status fk_helmholtz_set_iterate(fk_solver *s, const double *u_reim, int32_t n, int32_t on_device);

/* Probabilistic domain decomposition (the two-stage procedure of Sec. 3,
 * motivated in Sec. 1): from the next iteration on, Feynman-Kac paths run
 * only from the unknown nodes on the listed grid lines (x index in cuts_x,
 * y index in cuts_y: the subdomain interfaces), and every block of unknown
 * nodes between consecutive lines (or the edge) is then solved on the
 * device as its own Dirichlet problem of the same Poisson step,
 *   (Delta_h - (alpha - k^2)) u_{n+1} = f - (alpha + i p) u_n,
 * 5-point Laplacian, boundary values = the new interface values and g, by
 * fast diagonalisation (DST-I in x and y).  With a hole (disc or box), a
 * block with a hole node in it or on its frame is not a rectangle's
 * Dirichlet problem: its unknown nodes keep their own paths, like the
 * interface.  The iteration report's statistics (max_du, sup, max_se,
 * noise_ratio, path_steps) cover the nodes that run paths.  Host arrays,
 * copied.  FK_EINVAL: a reflecting edge, called after the first iteration or
 * twice, no cut,
 * cuts not strictly increasing within [1, nx-2] / [1, ny-2], or a block
 * wider than 64 nodes (a second call is rejected even when the cuts left no
 * block).  Allocates its device tables (freed at destroy).  FK_ENOMEM (the
 * allocation failed) or FK_EDEVICE (a copy failed): the solver is left as it
 * was, with no buffers of the call kept, and the call may be repeated. */
fk_status fk_helmholtz_set_pdd(fk_solver *s, const int32_t *cuts_x, int32_t n_cuts_x, const int32_t *cuts_y,
                               int32_t n_cuts_y);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): one
 * fixed-point iteration u_n -> u_{n+1} of the problem given by value, the same
 * computation as fk_helmholtz_create + fk_helmholtz_set_iterate(u_n, n) +
 * fk_helmholtz_iterate(1) + fk_helmholtz_get (bit-identical results), with
 * every working buffer of the library in one static device array of
 * FK_STATIC_SCRATCH_BYTES per GPU (held until the process ends): no device
 * allocation, no pinned host memory, no events.
 *   u_n     device, nx*ny complex (unknown nodes read; edge and hole nodes
 *           take the problem's data, a disc domain's exterior nodes their
 *           nearest unknown node's value), or NULL for u_0 = 0 (then n must
 *           be 0)
 *   n       index of u_n (the Philox counter word of the iteration)
 *   u_next  device, nx*ny complex: receives u_{n+1}; se: device or NULL,
 *           nx*ny complex standard errors; report (host, may be NULL):
 *           report->n = n + 1, step_ms = 0 (not timed).
 * Ordered on hip_stream and synchronised before returning (host staging
 * copies are made from pageable memory).  Every call on a GPU reuses that
 * GPU's array, so calls that overlap on one GPU (other threads, other
 * streams) race and must be serialised by the caller.  FK_EINVAL: as
 * fk_helmholtz_create, or the problem needs more working memory than the
 * array holds (about 212 bytes per grid node: every grid up to 257 x 257
 * fits); FK_EDIVERGED: u_{n+1} is not finite (still written). */
#define FK_STATIC_SCRATCH_BYTES (16u * 1024u * 1024u)
fk_status fk_helmholtz_step_static(const fk_domain *domain, const fk_source *f, const fk_bc *g_outer,
                                   const fk_bc *g_inner, const fk_params *params, const double *u_n, int32_t n,
                                   double *u_next, double *se, void *hip_stream, fk_iter_report *report);

/* Accumulated device time of the path kernel since creation or the last
 * reset (HIP events recorded on the solver's stream around each launch). */
fk_status fk_helmholtz_timing(fk_solver *s, double *step_ms_total, int64_t *launches, int32_t reset);

fk_status fk_helmholtz_destroy(fk_solver *s);

const char *fk_helmholtz_last_error(void);

/* ---------------------------------------------------------------- debug -- */

/* Philox4x32-10 words computed on the device: for each of the n counters
 * (4 words each) with key (seed mod 2^32, seed div 2^32), 4 output words. */
fk_status fk_debug_philox(uint64_t seed, const uint32_t *ctrs, int64_t n, uint32_t *out);

/* Box-Muller normals computed on the device in the given precision (32|64)
 * from n word pairs (ra, rb): z = sqrt(-2 ln U(ra)) (cos 2pi U(rb), sin 2pi U(rb)). */
fk_status fk_debug_normals(int32_t precision, const uint32_t *words, int64_t n, double *z);

/* Runs the listed paths (node id, path index m) of the next iteration of s
 * with the solver's kernels and current iterate: exit-step index J, score
 * (re, im) and exit point X_J (x, y) per path.  Host pointers, count each. */
fk_status fk_helmholtz_debug_paths(fk_solver *s, const int32_t *node_ids, const int64_t *ms,
                                   int64_t count, int64_t *J, double *score_reim, double *xj);

/* --------------------------------------------------------------- engine -- */
/*
 * Batched, continuous-batching engine: many instances (each its own domain,
 * k, M, seed, grid) advanced together, one fixed-point iteration per tick,
 * by one persistent work-stealing kernel launch replayed from a HIP graph.
 * Instances are admitted into free slots between ticks and retire on
 * convergence; the result of an instance does not depend on what else is in
 * the batch (fixed per-(node, chunk) result slots, fixed reduction order).
 */
typedef struct fk_engine fk_engine;

typedef struct {
    int32_t max_instances;     /* slots                                           */
    int32_t precision;         /* 32 | 64 for every instance                      */
    int64_t max_grid_nodes;    /* sum of nx*ny over resident instances            */
    int64_t max_items;         /* sum of work items over resident instances       */
    int64_t max_table;         /* sum of TABLE lengths over resident instances    */
    int32_t waves_per_cu;      /* persistent grid = CUs * waves_per_cu; 0 = auto  */
    int32_t max_instance_nodes;/* largest nx*ny of one instance; 0 = 257*257      */
} fk_engine_config;

/* Creates an engine with its own device memory (sized by cfg) on hip_stream. */
fk_status fk_engine_create(const fk_engine_config *cfg, void *hip_stream, fk_engine **out);

/* Admits an instance into a free slot (*slot).  FK_EBUSY: no free slot;
 * FK_ENOMEM: the resident instances leave too little room; FK_EINVAL as in
 * fk_helmholtz_create (precision must match the engine's). */
fk_status fk_engine_add(fk_engine *e, const fk_domain *domain, const fk_source *f,
                        const fk_bc *g_outer, const fk_bc *g_inner, const fk_params *params,
                        int32_t *slot);

/* One iteration of every active instance (one persistent launch).  reports:
 * max_instances entries, filled for active slots; active_mask: max_instances
 * bytes, 1 where the slot was active in this tick.  Instances whose report
 * says converged (max_du < tol), diverging or max_iters stay resident until
 * fk_engine_remove. */
fk_status fk_engine_tick(fk_engine *e, fk_iter_report *reports, uint8_t *active_mask);

/* Copies the iterate and SE of a slot (host pointers, nx*ny complex each). */
fk_status fk_engine_get(fk_engine *e, int32_t slot, double *u_reim, double *se_reim);

/* Per-node sum of exit-step indices and capped-path counts of the slot's last
 * iteration (nx*ny each, host pointers; 0 on nodes that are not unknowns). */
fk_status fk_engine_node_stats(fk_engine *e, int32_t slot, int64_t *sum_j, int64_t *capped);

/* Replaces the slot's iterate as fk_helmholtz_set_iterate does (resume from a
 * checkpoint; also used to inject a fault in tests).  Between ticks. */
fk_status fk_engine_set_iterate(fk_engine *e, int32_t slot, const double *u_reim, int32_t n, int32_t on_device);

/* Probabilistic domain decomposition of a resident instance (the two-stage
 * procedure of Sec. 3), as fk_helmholtz_set_pdd: from its next tick on, paths
 * run only from the unknown nodes on the cut lines, and its blocks are solved
 * on the device in the same tick (one launch for the blocks of all
 * instances, inside the tick's graph).  Before the instance's first tick,
 * once.  Takes its DST tables and right-hand sides from the engine pool.
 * FK_EINVAL as fk_helmholtz_set_pdd; FK_ENOMEM: the pool cannot hold them
 * now, or more than 16384 blocks would be resident. */
fk_status fk_engine_set_pdd(fk_engine *e, int32_t slot, const int32_t *cuts_x, int32_t n_cuts_x,
                            const int32_t *cuts_y, int32_t n_cuts_y);

/* Frees a slot and its memory for new instances. */
fk_status fk_engine_remove(fk_engine *e, int32_t slot);

/* Device time of the persistent kernel (HIP events around each launch). */
fk_status fk_engine_timing(fk_engine *e, double *kernel_ms_total, int64_t *launches, int32_t reset);

fk_status fk_engine_destroy(fk_engine *e);

#ifdef __cplusplus
}
#endif

#endif /* FK_HELMHOLTZ_H */
