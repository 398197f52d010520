// fk_solver.cpp -- single-instance solver behind the C ABI.
//
// One fixed-point iteration u_n -> u_{n+1} (Sec. 1 eq. (1.4) with alpha = k^2)
// is four launches on the solver's stream: reset of the status record and the
// queue head, the path kernel (waves pull (node, chunk) work items from a
// one-instance queue), the update kernel (node statistics, new iterate,
// status) and the iteration-index advance; then one 64-byte status copy to
// pinned host memory.  The host applies the
// sup-norm stopping rule (Sec. 3) and the divergence rule.
#include <algorithm>
#include <atomic>
#include <cmath>
#include <cstring>
#include <new>
#include <utility>
#include <vector>

#include "fk_internal.hpp"
#include "fk_problem.hpp"

namespace fkh {
const char *last_error_cstr();
}

using namespace fkh;

struct fk_solver {
    HostProblem P;
    hipStream_t stream = nullptr;
    char *arena = nullptr;
    bool own_arena = false;
    InstanceBuffers B{};
    fkd::Inst *d_inst = nullptr;      // device copy of the instance record (in the arena)
    fkd::EngineQueue *d_queue = nullptr;  // one-segment work queue (in the arena)
    unsigned long long *d_head = nullptr; // queue head (in the arena)
    int n_blocks = 0;
    fkd::DevState *h_status = nullptr;  // pinned
    hipEvent_t ev0 = nullptr, ev1 = nullptr;
    double step_ms_total = 0.0;
    int64_t launches = 0;
    int32_t iter = 0;
    std::vector<double> hist_sup, hist_du;
    fk_iter_report last{};
    // probabilistic domain decomposition (library-owned device memory)
    bool pdd = false;   // set_pdd succeeded (the blocks may be none: every line a cut)
    int32_t pdd_blocks = 0, pdd_max_nodes = 0;
    fkd::PddTask *d_pdd_tasks = nullptr;
    double *d_pdd_tables = nullptr;
    double2 *d_pdd_rhs = nullptr;
    // set by fk_helmholtz_cancel (any thread), taken by the next iteration
    std::atomic<int> cancel{0};
};

static size_t align256(size_t b) { return (b + 255) & ~(size_t)255; }

// arena: instance record | queue | head | instance buffers
static size_t solver_bytes(const HostProblem &P)
{
    return align256(sizeof(fkd::Inst)) + align256(sizeof(fkd::EngineQueue)) + 256 + instance_bytes(P);
}

extern "C" {

const char *fk_helmholtz_last_error(void) { return last_error_cstr(); }

fk_status fk_helmholtz_arena_bytes(const fk_domain *domain, const fk_bc *g_outer, const fk_params *params,
                                   size_t *bytes)
{
    if (!bytes) return fail(FK_EINVAL, "bytes is NULL");
    HostProblem P;
    fk_status st = setup_problem(domain, nullptr, g_outer, nullptr, params, P, true);
    if (st != FK_OK) return st;
    *bytes = solver_bytes(P);
    return FK_OK;
}

fk_status fk_helmholtz_work_items(const fk_domain *domain, const fk_bc *g_outer, const fk_params *params,
                                  int64_t *n_items, int32_t *paths_large, int32_t *items_large,
                                  int32_t *paths_small, int32_t *items_small)
{
    HostProblem P;
    fk_status st = setup_problem(domain, nullptr, g_outer, nullptr, params, P, true);
    if (st != FK_OK) return st;
    if (n_items) *n_items = P.n_items;
    if (paths_large) *paths_large = P.ppi_a;
    if (items_large) *items_large = P.items_a;
    if (paths_small) *paths_small = P.ppi;
    if (items_small) *items_small = P.items_per_node;
    return FK_OK;
}

fk_status fk_helmholtz_exterior_nodes(const fk_domain *domain, const fk_bc *g_outer, const fk_params *params,
                                      int32_t *pairs, int64_t cap, int64_t *n_pairs)
{
    if (!n_pairs) return fail(FK_EINVAL, "n_pairs is NULL");
    HostProblem P;
    fk_status st = setup_problem(domain, nullptr, g_outer, nullptr, params, P, true);
    if (st != FK_OK) return st;
    const int64_t n = (int64_t)(P.ext.size() / 2);
    *n_pairs = n;
    if (pairs) {
        if (cap < n) return fail(FK_EINVAL, "pairs holds fewer than n_pairs entries");
        std::memcpy(pairs, P.ext.data(), P.ext.size() * sizeof(int32_t));
    }
    return FK_OK;
}

fk_status fk_helmholtz_create(const fk_domain *domain, const fk_source *f, const fk_bc *g_outer,
                              const fk_bc *g_inner, const fk_params *params, void *device_arena,
                              size_t arena_bytes, void *hip_stream, fk_solver **out)
{
    if (!out) return fail(FK_EINVAL, "out is NULL");
    *out = nullptr;
    fk_solver *s = new (std::nothrow) fk_solver();
    if (!s) return fail(FK_ENOMEM, "host allocation failed");
    fk_status st = setup_problem(domain, f, g_outer, g_inner, params, s->P, true);
    if (st != FK_OK) {
        delete s;
        return st;
    }
    s->stream = (hipStream_t)hip_stream;
    const size_t need = solver_bytes(s->P);
    if (device_arena) {
        if (((uintptr_t)device_arena & 255u) != 0) {
            delete s;
            return fail(FK_EINVAL, "device_arena must be 256-byte aligned");
        }
        if (arena_bytes < need) {
            delete s;
            return fail(FK_ENOMEM, "arena too small: need " + std::to_string(need) + " bytes");
        }
        s->arena = (char *)device_arena;
    } else {
        hipError_t e = hipMalloc((void **)&s->arena, need);
        if (e != hipSuccess) {
            delete s;
            return hip_fail(e, "hipMalloc(arena)");
        }
        s->own_arena = true;
    }
    char *p = s->arena;
    s->d_inst = (fkd::Inst *)p;
    p += align256(sizeof(fkd::Inst));
    s->d_queue = (fkd::EngineQueue *)p;
    p += align256(sizeof(fkd::EngineQueue));
    s->d_head = (unsigned long long *)p;
    p += 256;
    s->B = carve(s->P, p);
    s->n_blocks = path_kernel_blocks(s->P.par.waves_per_cu);
    fkd::Inst D = make_inst(s->P, s->B);
    auto cleanup = [&](fk_status code) {
        fk_helmholtz_destroy(s);
        return code;
    };
    hipError_t e = hipHostMalloc((void **)&s->h_status, sizeof(fkd::DevState), hipHostMallocDefault);
    if (e != hipSuccess) return cleanup(hip_fail(e, "hipHostMalloc(status)"));
    if ((e = hipEventCreate(&s->ev0)) != hipSuccess || (e = hipEventCreate(&s->ev1)) != hipSuccess)
        return cleanup(hip_fail(e, "hipEventCreate"));
    if ((st = upload_instance(s->P, s->B, s->stream)) != FK_OK) return cleanup(st);
    if ((e = hipMemcpyAsync(s->d_inst, &D, sizeof(D), hipMemcpyHostToDevice, s->stream)) != hipSuccess)
        return cleanup(hip_fail(e, "hipMemcpyAsync(inst)"));
    {
        fkd::EngineQueue q;
        std::memset(&q, 0, sizeof(q));
        q.n_seg = 1;
        q.seg_end[0] = s->P.n_items;
        q.seg_inst[0] = 0;
        if ((e = hipMemcpyAsync(s->d_queue, &q, sizeof(q), hipMemcpyHostToDevice, s->stream)) != hipSuccess ||
            (e = hipStreamSynchronize(s->stream)) != hipSuccess)
            return cleanup(hip_fail(e, "hipMemcpyAsync(queue)"));
    }
    if ((e = hipStreamSynchronize(s->stream)) != hipSuccess) return cleanup(hip_fail(e, "hipStreamSynchronize"));
    *out = s;
    return FK_OK;
}

static fk_status run_one(fk_solver *s, fk_iter_report *rep)
{
    const int prec = s->P.par.precision;
    FK_HIP(fkk::launch_reset(s->d_inst, nullptr, 1, nullptr, s->d_head, s->stream));
    FK_HIP(hipEventRecord(s->ev0, s->stream));
    FK_HIP(fkk::launch_stream(prec, s->P.features(), s->d_inst, s->d_queue, s->d_head, s->n_blocks, s->stream,
                              s->P.cells == 0, s->P.lds_grid ? s->P.n_nodes() * 8 : 0));
    FK_HIP(hipEventRecord(s->ev1, s->stream));
    FK_HIP(fkk::launch_update(s->d_inst, nullptr, 1, nullptr, (int32_t)s->P.interior.size(), s->stream));
    FK_HIP(fkk::launch_extend(s->d_inst, (int32_t)(s->P.ext.size() / 2), s->stream));
    if (s->pdd_blocks > 0)
        FK_HIP(fkk::launch_pdd(s->d_inst, s->d_pdd_tasks, s->pdd_blocks, nullptr, s->pdd_blocks, s->pdd_max_nodes,
                               s->stream));
    FK_HIP(fkk::launch_advance(s->d_inst, nullptr, 1, nullptr, s->stream));
    FK_HIP(hipMemcpyAsync(s->h_status, s->B.state, sizeof(fkd::DevState), hipMemcpyDeviceToHost, s->stream));
    FK_HIP(hipStreamSynchronize(s->stream));
    float ms = 0.0f;
    FK_HIP(hipEventElapsedTime(&ms, s->ev0, s->ev1));
    s->step_ms_total += ms;
    s->launches += 1;
    s->iter += 1;
    const fkd::DevState &h = *s->h_status;
    double du, sup, se;
    std::memcpy(&du, &h.max_du, 8);
    std::memcpy(&sup, &h.sup, 8);
    std::memcpy(&se, &h.max_se, 8);
    fk_iter_report r{};
    r.n = s->iter;
    r.max_du = du;
    r.sup = sup;
    r.max_se = se;
    r.noise_floor = 4.0 * se;
    r.path_steps = (int64_t)h.path_steps;
    r.capped = (int64_t)h.capped;
    r.nonfinite = (int64_t)h.nonfinite;
    r.step_ms = ms;
    r.noise_ratio = h.ratio_n ? (double)h.ratio_fx * 0x1p-20 / (double)h.ratio_n : 0.0;
    bool div = !(std::isfinite(du) && std::isfinite(sup)) || r.nonfinite > 0;
    const size_t nh = s->hist_du.size();
    if (!div && nh >= 5)
        div = sup >= 1.25 * s->hist_sup[nh - 5] && du >= 1.25 * s->hist_du[nh - 5];
    r.diverging = div ? 1 : 0;
    s->hist_sup.push_back(sup);
    s->hist_du.push_back(du);
    s->last = r;
    if (rep) *rep = r;
    return div ? fail(FK_EDIVERGED, "divergence rule fired at iteration " + std::to_string(r.n)) : FK_OK;
}

fk_status fk_helmholtz_set_pdd(fk_solver *s, const int32_t *cuts_x, int32_t n_cuts_x, const int32_t *cuts_y,
                               int32_t n_cuts_y)
{
    if (!s) return fail(FK_EINVAL, "solver is NULL");
    if (s->iter != 0 || s->pdd) return fail(FK_EINVAL, "set PDD once, before the first iteration");
    PddPlan plan;
    fk_status st = plan_pdd(s->P, cuts_x, n_cuts_x, cuts_y, n_cuts_y, plan);
    if (st != FK_OK) return st;
    // on any failure below the solver is left as it was: no partial buffers
    // behind a retry, the host record unchanged
    auto drop = [s]() {
        for (void **b : {(void **)&s->d_pdd_tasks, (void **)&s->d_pdd_tables, (void **)&s->d_pdd_rhs})
            if (*b) {
                (void)hipFree(*b);
                *b = nullptr;
            }
    };
    const size_t nb = plan.blocks.size();
    hipError_t e = hipSuccess;
    const char *what = nullptr;
    if (nb > 0) {
        if ((e = hipMalloc((void **)&s->d_pdd_tasks, nb * sizeof(fkd::PddTask))) != hipSuccess ||
            (e = hipMalloc((void **)&s->d_pdd_tables, plan.tables.size() * sizeof(double))) != hipSuccess ||
            (e = hipMalloc((void **)&s->d_pdd_rhs, s->P.n_nodes() * sizeof(double2))) != hipSuccess) {
            what = "hipMalloc(pdd)";
        } else {
            std::vector<fkd::PddTask> tasks(nb);
            for (size_t i = 0; i < nb; ++i) {
                const PddPlan::Block &B = plan.blocks[i];
                tasks[i] = fkd::PddTask{0, B.i0, B.i1, B.j0, B.j1, 0, s->d_pdd_tables + B.tx,
                                        s->d_pdd_tables + B.ty, s->d_pdd_rhs};
            }
            if ((e = hipMemcpyAsync(s->d_pdd_tasks, tasks.data(), nb * sizeof(fkd::PddTask), hipMemcpyHostToDevice,
                                    s->stream)) != hipSuccess ||
                (e = hipMemcpyAsync(s->d_pdd_tables, plan.tables.data(), plan.tables.size() * sizeof(double),
                                    hipMemcpyHostToDevice, s->stream)) != hipSuccess ||
                (e = hipStreamSynchronize(s->stream)) != hipSuccess)
                what = "hipMemcpyAsync(pdd tables)";
        }
    }
    // the host record changes only once the device has the new node list,
    // instance record and queue; items sized for at least two per wave of
    // the launch
    HostProblem P2 = s->P;
    apply_pdd(P2, plan, 2 * (int64_t)s->n_blocks * 4);
    fkd::Inst D = make_inst(P2, s->B);
    fkd::EngineQueue q;
    std::memset(&q, 0, sizeof(q));
    q.n_seg = 1;
    q.seg_end[0] = P2.n_items;
    q.seg_inst[0] = 0;
    const bool touched = !what;   // the device node list is being rewritten
    if (!what &&
        ((e = hipMemcpyAsync(s->B.nodes, P2.interior.data(), P2.interior.size() * sizeof(int32_t),
                             hipMemcpyHostToDevice, s->stream)) != hipSuccess ||
         (e = hipMemcpyAsync(s->d_inst, &D, sizeof(D), hipMemcpyHostToDevice, s->stream)) != hipSuccess ||
         (e = hipMemcpyAsync(s->d_queue, &q, sizeof(q), hipMemcpyHostToDevice, s->stream)) != hipSuccess ||
         (e = hipStreamSynchronize(s->stream)) != hipSuccess))
        what = "hipMemcpyAsync(pdd node list)";
    if (what) {
        (void)hipStreamSynchronize(s->stream);
        drop();
        if (touched) {
            // best effort: the device node list, record and queue back to the
            // host record's (unchanged)
            const fkd::Inst D0 = make_inst(s->P, s->B);
            fkd::EngineQueue q0 = q;
            q0.seg_end[0] = s->P.n_items;
            (void)hipMemcpyAsync(s->B.nodes, s->P.interior.data(), s->P.interior.size() * sizeof(int32_t),
                                 hipMemcpyHostToDevice, s->stream);
            (void)hipMemcpyAsync(s->d_inst, &D0, sizeof(D0), hipMemcpyHostToDevice, s->stream);
            (void)hipMemcpyAsync(s->d_queue, &q0, sizeof(q0), hipMemcpyHostToDevice, s->stream);
            (void)hipStreamSynchronize(s->stream);
        }
        return hip_fail(e, what);
    }
    s->P = std::move(P2);
    s->pdd = true;
    s->pdd_blocks = (int32_t)nb;
    s->pdd_max_nodes = plan.max_nodes;
    return FK_OK;
}

fk_status fk_helmholtz_cancel(fk_solver *s)
{
    if (!s) return fail(FK_EINVAL, "solver is NULL");
    s->cancel.store(1);
    return FK_OK;
}

// Takes a pending cancel request (true: the caller stops with FK_ECANCELLED).
static bool take_cancel(fk_solver *s) { return s->cancel.exchange(0) != 0; }

fk_status fk_helmholtz_iterate(fk_solver *s, int32_t n_iters, fk_iter_report *last)
{
    if (!s) return fail(FK_EINVAL, "solver is NULL");
    if (n_iters < 0) return fail(FK_EINVAL, "n_iters must be >= 0");
    for (int32_t i = 0; i < n_iters; ++i) {
        if (take_cancel(s)) {
            if (last) *last = s->last;
            return fail(FK_ECANCELLED, "cancelled after iteration " + std::to_string(s->iter));
        }
        fk_status st = run_one(s, last);
        if (st != FK_OK) return st;
    }
    if (n_iters == 0 && last) *last = s->last;
    return FK_OK;
}

fk_status fk_helmholtz_solve(fk_solver *s, fk_iter_report *final_report)
{
    if (!s) return fail(FK_EINVAL, "solver is NULL");
    const double tol = s->P.par.tol;
    while (s->iter < s->P.par.max_iters) {
        if (take_cancel(s)) {
            if (final_report) *final_report = s->last;
            return fail(FK_ECANCELLED, "cancelled after iteration " + std::to_string(s->iter));
        }
        fk_iter_report r;
        fk_status st = run_one(s, &r);
        if (final_report) *final_report = r;
        if (st != FK_OK) return st;
        if (tol > 0.0 && r.max_du < tol) return FK_OK;
    }
    if (final_report) *final_report = s->last;
    if (tol > 0.0) return fail(FK_ENOTCONVERGED, "max_iters reached above tol");
    return FK_OK;
}

fk_status fk_helmholtz_get(fk_solver *s, double *u_reim, double *se_reim, int32_t on_device)
{
    if (!s) return fail(FK_EINVAL, "solver is NULL");
    const size_t nn = s->P.n_nodes();
    const hipMemcpyKind kind = on_device ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost;
    if (u_reim) FK_HIP(hipMemcpyAsync(u_reim, s->B.u64, nn * sizeof(double2), kind, s->stream));
    if (se_reim) FK_HIP(hipMemcpyAsync(se_reim, s->B.se, nn * sizeof(double2), kind, s->stream));
    FK_HIP(hipStreamSynchronize(s->stream));
    return FK_OK;
}

fk_status fk_helmholtz_node_stats(fk_solver *s, int64_t *sum_j, int64_t *capped)
{
    if (!s) return fail(FK_EINVAL, "solver is NULL");
    const size_t nn = s->P.n_nodes();
    if (sum_j) FK_HIP(hipMemcpyAsync(sum_j, s->B.sum_j, nn * sizeof(int64_t), hipMemcpyDeviceToHost, s->stream));
    if (capped) FK_HIP(hipMemcpyAsync(capped, s->B.capped, nn * sizeof(int64_t), hipMemcpyDeviceToHost, s->stream));
    FK_HIP(hipStreamSynchronize(s->stream));
    return FK_OK;
}

fk_status fk_helmholtz_set_iterate(fk_solver *s, const double *u_reim, int32_t n, int32_t on_device)
{
    if (!s || !u_reim) return fail(FK_EINVAL, "solver and u_reim are required");
    if (n < 0) return fail(FK_EINVAL, "n must be >= 0");
    const fk_status st = load_iterate(s->P, s->B, u_reim, n, on_device != 0, s->stream);
    if (st != FK_OK) return st;
    s->iter = n;
    s->hist_du.clear();
    s->hist_sup.clear();
    return FK_OK;
}

fk_status fk_helmholtz_timing(fk_solver *s, double *step_ms_total, int64_t *launches, int32_t reset)
{
    if (!s) return fail(FK_EINVAL, "solver is NULL");
    if (step_ms_total) *step_ms_total = s->step_ms_total;
    if (launches) *launches = s->launches;
    if (reset) {
        s->step_ms_total = 0.0;
        s->launches = 0;
    }
    return FK_OK;
}

fk_status fk_helmholtz_destroy(fk_solver *s)
{
    if (!s) return FK_OK;
    if (s->stream || s->arena) (void)hipStreamSynchronize(s->stream);
    if (s->ev0) (void)hipEventDestroy(s->ev0);
    if (s->ev1) (void)hipEventDestroy(s->ev1);
    if (s->h_status) (void)hipHostFree(s->h_status);
    if (s->d_pdd_tasks) (void)hipFree(s->d_pdd_tasks);
    if (s->d_pdd_tables) (void)hipFree(s->d_pdd_tables);
    if (s->d_pdd_rhs) (void)hipFree(s->d_pdd_rhs);
    if (s->own_arena && s->arena) (void)hipFree(s->arena);
    delete s;
    return FK_OK;
}

// ------------------------------------------------------------------ debug

fk_status fk_debug_philox(uint64_t seed, const uint32_t *ctrs, int64_t n, uint32_t *out)
{
    if (n < 0 || (n > 0 && (!ctrs || !out))) return fail(FK_EINVAL, "bad arguments");
    if (n == 0) return FK_OK;
    uint4 *d_c = nullptr, *d_o = nullptr;
    FK_HIP(hipMalloc((void **)&d_c, n * sizeof(uint4)));
    hipError_t e = hipMalloc((void **)&d_o, n * sizeof(uint4));
    if (e == hipSuccess) e = hipMemcpy(d_c, ctrs, n * sizeof(uint4), hipMemcpyHostToDevice);
    if (e == hipSuccess) e = fkk::launch_debug_philox((uint32_t)seed, (uint32_t)(seed >> 32), d_c, n, d_o, nullptr);
    if (e == hipSuccess) e = hipMemcpy(out, d_o, n * sizeof(uint4), hipMemcpyDeviceToHost);
    (void)hipFree(d_c);
    if (d_o) (void)hipFree(d_o);
    if (e != hipSuccess) return hip_fail(e, "fk_debug_philox");
    return FK_OK;
}

fk_status fk_debug_normals(int32_t precision, const uint32_t *words, int64_t n, double *z)
{
    if (n < 0 || (n > 0 && (!words || !z)) || (precision != 32 && precision != 64))
        return fail(FK_EINVAL, "bad arguments");
    if (n == 0) return FK_OK;
    uint2 *d_w = nullptr;
    double2 *d_z = nullptr;
    FK_HIP(hipMalloc((void **)&d_w, n * sizeof(uint2)));
    hipError_t e = hipMalloc((void **)&d_z, n * sizeof(double2));
    if (e == hipSuccess) e = hipMemcpy(d_w, words, n * sizeof(uint2), hipMemcpyHostToDevice);
    if (e == hipSuccess) e = fkk::launch_debug_normals(precision, d_w, n, d_z, nullptr);
    if (e == hipSuccess) e = hipMemcpy(z, d_z, n * sizeof(double2), hipMemcpyDeviceToHost);
    (void)hipFree(d_w);
    if (d_z) (void)hipFree(d_z);
    if (e != hipSuccess) return hip_fail(e, "fk_debug_normals");
    return FK_OK;
}

fk_status fk_helmholtz_debug_paths(fk_solver *s, const int32_t *node_ids, const int64_t *ms, int64_t count,
                                   int64_t *J, double *score_reim, double *xj)
{
    if (!s || count < 0 || (count > 0 && (!node_ids || !ms || !J || !score_reim || !xj)))
        return fail(FK_EINVAL, "bad arguments");
    if (count == 0) return FK_OK;
    const size_t nn = s->P.n_nodes();
    for (int64_t i = 0; i < count; ++i) {
        if (node_ids[i] < 0 || (size_t)node_ids[i] >= nn || s->P.cls[node_ids[i]] != 0)
            return fail(FK_EINVAL, "debug path node is not an interior node");
        if (ms[i] < 0 || ms[i] > 0xFFFFFFFFll) return fail(FK_EINVAL, "debug path index out of range");
    }
    int32_t *d_n = nullptr;
    int64_t *d_m = nullptr;
    long long *d_J = nullptr;
    double2 *d_s = nullptr, *d_x = nullptr;
    hipError_t e = hipMalloc((void **)&d_n, count * sizeof(int32_t));
    if (e == hipSuccess) e = hipMalloc((void **)&d_m, count * sizeof(int64_t));
    if (e == hipSuccess) e = hipMalloc((void **)&d_J, count * sizeof(long long));
    if (e == hipSuccess) e = hipMalloc((void **)&d_s, count * sizeof(double2));
    if (e == hipSuccess) e = hipMalloc((void **)&d_x, count * sizeof(double2));
    if (e == hipSuccess) e = hipMemcpyAsync(d_n, node_ids, count * sizeof(int32_t), hipMemcpyHostToDevice, s->stream);
    if (e == hipSuccess) e = hipMemcpyAsync(d_m, ms, count * sizeof(int64_t), hipMemcpyHostToDevice, s->stream);
    if (e == hipSuccess)
        e = fkk::launch_debug_paths(s->P.par.precision, s->d_inst, d_n, d_m, count, d_J, d_s, d_x, s->stream);
    if (e == hipSuccess) e = hipMemcpyAsync(J, d_J, count * sizeof(long long), hipMemcpyDeviceToHost, s->stream);
    if (e == hipSuccess) e = hipMemcpyAsync(score_reim, d_s, count * sizeof(double2), hipMemcpyDeviceToHost, s->stream);
    if (e == hipSuccess) e = hipMemcpyAsync(xj, d_x, count * sizeof(double2), hipMemcpyDeviceToHost, s->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(s->stream);
    (void)hipFree(d_n);
    (void)hipFree(d_m);
    (void)hipFree(d_J);
    (void)hipFree(d_s);
    (void)hipFree(d_x);
    if (e != hipSuccess) return hip_fail(e, "fk_helmholtz_debug_paths");
    return FK_OK;
}

}  // extern "C"
