// fk_engine.cpp -- batched, continuous-batching engine behind the C ABI.
//
// Device-resident tables hold, per slot, the instance record and its status;
// a segment table numbers the work items of the active instances (longest
// expected paths first).  One tick = one fixed-point iteration of every active
// instance = one replay of a HIP graph captured at creation:
//   reset (status + queue head) -> path kernel (persistent waves pulling work
//   items from the queue) -> update (all active instances) -> iteration
//   advance -> status copy.
// One graph is captured per set of optional path-kernel features (hole,
// source term, shift or damping, reflecting edge); a tick replays the one for the union of the active
// instances' features.  Admitting or retiring an instance edits the tables
// between ticks; the graphs are never re-captured.  Instance memory comes from one device pool managed by
// a first-fit allocator; admission fails with FK_ENOMEM when the pool cannot
// hold the instance's footprint, so callers admit by HBM footprint.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <map>
#include <new>
#include <vector>

#include "fk_internal.hpp"
#include "fk_problem.hpp"

using namespace fkh;

namespace {

struct Region {
    size_t off, size;
};

// First-fit allocator over [0, capacity) in 256-byte units.
class PoolAllocator {
public:
    explicit PoolAllocator(size_t cap = 0) { reset(cap); }
    void reset(size_t cap)
    {
        free_.clear();
        if (cap) free_[0] = cap;
    }
    bool alloc(size_t bytes, size_t &off)
    {
        bytes = (bytes + 255) & ~(size_t)255;
        for (auto it = free_.begin(); it != free_.end(); ++it) {
            if (it->second >= bytes) {
                off = it->first;
                const size_t rest = it->second - bytes;
                free_.erase(it);
                if (rest) free_[off + bytes] = rest;
                return true;
            }
        }
        return false;
    }
    void release(size_t off, size_t bytes)
    {
        bytes = (bytes + 255) & ~(size_t)255;
        auto it = free_.emplace(off, bytes).first;
        auto nx = std::next(it);
        if (nx != free_.end() && it->first + it->second == nx->first) {
            it->second += nx->second;
            free_.erase(nx);
        }
        if (it != free_.begin()) {
            auto pv = std::prev(it);
            if (pv->first + pv->second == it->first) {
                pv->second += it->second;
                free_.erase(it);
            }
        }
    }

private:
    std::map<size_t, size_t> free_;  // offset -> size
};

struct SlotInfo {
    bool used = false;
    HostProblem P;
    Region region{};
    InstanceBuffers B{};
    int32_t iter = 0;
    double est_cost = 0.0;           // expected path steps per item (ordering)
    std::vector<double> hist_sup, hist_du;
    // probabilistic domain decomposition: the block solves of the instance
    // (pointers into its own pool region: DST tables, right-hand sides)
    bool pdd = false;
    Region pdd_region{};
    std::vector<fkd::PddTask> tasks;
};

// Block solves of the probabilistic domain decomposition per tick, over all
// instances (the graph's launch loops over the listed tasks).
constexpr int32_t kMaxPddTasks = 16384;

}  // namespace

struct fk_engine {
    fk_engine_config cfg{};
    hipStream_t user_stream = nullptr;
    hipStream_t cap_stream = nullptr;   // private stream used for capture
    int n_blocks = 0;
    int32_t max_interior_cap = 0;
    // device
    fkd::Inst *d_insts = nullptr;       // [max_instances]
    fkd::DevState *d_states = nullptr;  // [max_instances]
    int32_t *d_active = nullptr;        // [max_instances]
    int32_t *d_n_active = nullptr;
    fkd::EngineQueue *d_queue = nullptr;
    unsigned long long *d_head = nullptr;
    char *d_pool = nullptr;
    size_t pool_bytes = 0;
    // host mirrors
    fkd::DevState *h_states = nullptr;  // pinned [max_instances]
    fkd::EngineQueue *h_queue = nullptr;  // pinned
    int32_t *h_active = nullptr;        // pinned [max_instances + 1]
    fkd::PddTask *d_tasks = nullptr;    // [kMaxPddTasks] + count
    int32_t *d_n_tasks = nullptr;
    fkd::PddTask *h_tasks = nullptr;    // pinned [kMaxPddTasks]
    int32_t *h_n_tasks = nullptr;       // pinned
    int32_t pdd_grid = 0;               // workgroups of the block-solve launch
    std::vector<SlotInfo> slots;
    std::vector<fkd::Inst> h_insts;
    PoolAllocator pool;
    bool tables_dirty = true;
    int32_t n_active = 0;
    hipGraph_t graph[16] = {};        // per feature set of the path kernel
    hipGraphExec_t exec[16] = {};
    hipEvent_t ev0 = nullptr, ev1 = nullptr;
    double kernel_ms_total = 0.0;
    int64_t launches = 0;
};

static size_t align256(size_t b) { return (b + 255) & ~(size_t)255; }

// Feature sets that occur: a reflecting edge (bit 3) always comes with a
// hole (bit 0), so a union of instances' sets with bit 3 has bit 0 too.
static bool valid_feature_set(int f) { return (f & 8) == 0 || (f & 1) != 0; }

static fk_status capture_graph(fk_engine *e, int features)
{
    const int prec = e->cfg.precision;
    const int32_t cap = e->cfg.max_instances;
    FK_HIP(hipStreamBeginCapture(e->cap_stream, hipStreamCaptureModeThreadLocal));
    hipError_t err = fkk::launch_reset(e->d_insts, e->d_active, cap, e->d_n_active, e->d_head, e->cap_stream);
    if (err == hipSuccess)
        err = fkk::launch_stream(prec, features, e->d_insts, e->d_queue, e->d_head, e->n_blocks, e->cap_stream);
    if (err == hipSuccess)
        err = fkk::launch_update(e->d_insts, e->d_active, cap, e->d_n_active, e->max_interior_cap, e->cap_stream);
    // block solves of the instances with a domain decomposition (none: the
    // launch finds no task and ends at once)
    if (err == hipSuccess)
        err = fkk::launch_pdd(e->d_insts, e->d_tasks, 0, e->d_n_tasks, e->pdd_grid,
                              fkd::kPddMaxSide * fkd::kPddMaxSide, e->cap_stream);
    if (err == hipSuccess) err = fkk::launch_advance(e->d_insts, e->d_active, cap, e->d_n_active, e->cap_stream);
    if (err == hipSuccess)
        err = hipMemcpyAsync(e->h_states, e->d_states, cap * sizeof(fkd::DevState), hipMemcpyDeviceToHost,
                             e->cap_stream);
    hipGraph_t g = nullptr;
    hipError_t end = hipStreamEndCapture(e->cap_stream, &g);
    if (err != hipSuccess) {
        if (g) (void)hipGraphDestroy(g);
        return hip_fail(err, "engine graph capture");
    }
    if (end != hipSuccess) return hip_fail(end, "hipStreamEndCapture");
    e->graph[features] = g;
    FK_HIP(hipGraphInstantiate(&e->exec[features], g, nullptr, nullptr, 0));
    return FK_OK;
}

// Rebuilds the active list and the segment table (longest expected paths first).
static void rebuild_tables(fk_engine *e)
{
    std::vector<int32_t> act;
    for (int32_t i = 0; i < e->cfg.max_instances; ++i)
        if (e->slots[i].used) act.push_back(i);
    std::stable_sort(act.begin(), act.end(), [&](int32_t a, int32_t b) {
        return e->slots[a].est_cost > e->slots[b].est_cost;
    });
    e->n_active = (int32_t)act.size();
    e->h_queue->n_seg = e->n_active;
    int64_t acc = 0;
    for (int32_t s = 0; s < e->n_active; ++s) {
        acc += e->slots[act[s]].P.n_items;
        e->h_queue->seg_end[s] = acc;
        e->h_queue->seg_inst[s] = act[s];
        e->h_active[s] = act[s];
    }
    e->h_active[e->cfg.max_instances] = e->n_active;
    int32_t nt = 0;
    for (int32_t s = 0; s < e->n_active; ++s)
        for (const fkd::PddTask &t : e->slots[act[s]].tasks) e->h_tasks[nt++] = t;
    *e->h_n_tasks = nt;
    e->tables_dirty = true;
}

static int32_t pdd_task_count(const fk_engine *e)
{
    int32_t n = 0;
    for (const SlotInfo &o : e->slots)
        if (o.used) n += (int32_t)o.tasks.size();
    return n;
}

extern "C" {

fk_status fk_engine_destroy(fk_engine *e);

fk_status fk_engine_create(const fk_engine_config *cfg, void *hip_stream, fk_engine **out)
{
    if (!cfg || !out) return fail(FK_EINVAL, "cfg and out are required");
    *out = nullptr;

    if (cfg->max_instances < 1 || cfg->max_instances > fkd::kMaxSlots)
        return fail(FK_EINVAL, "max_instances must be in [1, " + std::to_string(fkd::kMaxSlots) + "]");
    if (cfg->precision != 32 && cfg->precision != 64) return fail(FK_EINVAL, "precision must be 32 or 64");
    if (cfg->max_grid_nodes < 9 || cfg->max_items < 1 || cfg->max_table < 0 || cfg->waves_per_cu < 0 ||
        cfg->max_instance_nodes < 0)
        return fail(FK_EINVAL, "engine capacities out of range");
    fk_engine *e = new (std::nothrow) fk_engine();
    if (!e) return fail(FK_ENOMEM, "host allocation failed");
    e->cfg = *cfg;
    e->user_stream = (hipStream_t)hip_stream;
    e->slots.resize(cfg->max_instances);
    e->h_insts.resize(cfg->max_instances);
    auto bail = [&](fk_status st) {
        fk_engine_destroy(e);
        return st;
    };
    hipError_t err;
    e->n_blocks = path_kernel_blocks(cfg->waves_per_cu);
    // largest interior count of one instance (sizes the update grid of the graph)
    e->max_interior_cap = cfg->max_instance_nodes > 0 ? cfg->max_instance_nodes : 257 * 257;
    const int32_t cap = cfg->max_instances;
    // pool: per-node arrays (u64 16, gather copy up to 64 when FP64
    // cell-major, nodes 4, se 16, sum_j 8, capped 8, slot, and the block
    // right-hand sides 16 of a domain decomposition), tables, and per
    // instance 11 alignment paddings and the decomposition's DST tables
    e->pool_bytes = (size_t)cfg->max_grid_nodes * (132 + sizeof(fkd::Slot)) + (size_t)cfg->max_table * 16 +
                    (size_t)cap * (11 * 256 + 8192);
    if ((err = hipStreamCreateWithFlags(&e->cap_stream, hipStreamNonBlocking)) != hipSuccess)
        return bail(hip_fail(err, "hipStreamCreateWithFlags"));
    if ((err = hipMalloc((void **)&e->d_insts, cap * sizeof(fkd::Inst))) != hipSuccess ||
        (err = hipMalloc((void **)&e->d_states, cap * sizeof(fkd::DevState))) != hipSuccess ||
        (err = hipMalloc((void **)&e->d_active, (cap + 1) * sizeof(int32_t))) != hipSuccess ||
        (err = hipMalloc((void **)&e->d_queue, sizeof(fkd::EngineQueue))) != hipSuccess ||
        (err = hipMalloc((void **)&e->d_head, 256)) != hipSuccess ||
        (err = hipMalloc((void **)&e->d_pool, e->pool_bytes)) != hipSuccess ||
        (err = hipMalloc((void **)&e->d_tasks, kMaxPddTasks * sizeof(fkd::PddTask) + 256)) != hipSuccess)
        return bail(hip_fail(err, "hipMalloc(engine)"));
    e->d_n_tasks = (int32_t *)((char *)e->d_tasks + kMaxPddTasks * sizeof(fkd::PddTask));
    e->d_n_active = e->d_active + cap;
    if ((err = hipHostMalloc((void **)&e->h_states, cap * sizeof(fkd::DevState), hipHostMallocDefault)) != hipSuccess ||
        (err = hipHostMalloc((void **)&e->h_queue, sizeof(fkd::EngineQueue), hipHostMallocDefault)) != hipSuccess ||
        (err = hipHostMalloc((void **)&e->h_active, (cap + 1) * sizeof(int32_t), hipHostMallocDefault)) != hipSuccess ||
        (err = hipHostMalloc((void **)&e->h_tasks, kMaxPddTasks * sizeof(fkd::PddTask), hipHostMallocDefault)) !=
            hipSuccess ||
        (err = hipHostMalloc((void **)&e->h_n_tasks, sizeof(int32_t), hipHostMallocDefault)) != hipSuccess)
        return bail(hip_fail(err, "hipHostMalloc(engine)"));
    *e->h_n_tasks = 0;
    std::memset(e->h_states, 0, cap * sizeof(fkd::DevState));
    std::memset(e->h_queue, 0, sizeof(fkd::EngineQueue));
    std::memset(e->h_active, 0, (cap + 1) * sizeof(int32_t));
    std::memset(e->h_insts.data(), 0, cap * sizeof(fkd::Inst));
    if ((err = hipMemcpy(e->d_insts, e->h_insts.data(), cap * sizeof(fkd::Inst), hipMemcpyHostToDevice)) != hipSuccess ||
        (err = hipMemcpy(e->d_states, e->h_states, cap * sizeof(fkd::DevState), hipMemcpyHostToDevice)) != hipSuccess ||
        (err = hipMemcpy(e->d_active, e->h_active, (cap + 1) * sizeof(int32_t), hipMemcpyHostToDevice)) != hipSuccess ||
        (err = hipMemcpy(e->d_queue, e->h_queue, sizeof(fkd::EngineQueue), hipMemcpyHostToDevice)) != hipSuccess ||
        (err = hipMemcpy(e->d_n_tasks, e->h_n_tasks, sizeof(int32_t), hipMemcpyHostToDevice)) != hipSuccess)
        return bail(hip_fail(err, "hipMemcpy(engine tables)"));
    {
        int dev = 0, n_cu = 0;
        if (hipGetDevice(&dev) != hipSuccess ||
            hipDeviceGetAttribute(&n_cu, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || n_cu <= 0)
            n_cu = 256;
        e->pdd_grid = n_cu;
    }
    if ((err = hipEventCreate(&e->ev0)) != hipSuccess || (err = hipEventCreate(&e->ev1)) != hipSuccess)
        return bail(hip_fail(err, "hipEventCreate"));
    e->pool.reset(e->pool_bytes);
    for (int f = 0; f < 16; ++f) {
        if (!valid_feature_set(f)) continue;
        fk_status st = capture_graph(e, f);
        if (st != FK_OK) return bail(st);
    }
    e->tables_dirty = false;
    *out = e;
    return FK_OK;
}

fk_status fk_engine_add(fk_engine *e, const fk_domain *domain, const fk_source *f, const fk_bc *g_outer,
                        const fk_bc *g_inner, const fk_params *params, int32_t *slot)
{
    if (!e || !slot) return fail(FK_EINVAL, "engine and slot are required");
    *slot = -1;
    int32_t free_slot = -1;
    for (int32_t i = 0; i < e->cfg.max_instances; ++i)
        if (!e->slots[i].used) {
            free_slot = i;
            break;
        }
    HostProblem P;
    fk_status st = setup_problem(domain, f, g_outer, g_inner, params, P);
    if (st != FK_OK) return st;
    if (P.par.precision != e->cfg.precision) return fail(FK_EINVAL, "instance precision differs from the engine's");
    // the disc kernels mirror every path radially (they serve disc domains
    // alone) and an engine launch mixes instances, so disc domains stay in
    // the single-instance solver
    if (P.disc_domain()) return fail(FK_EINVAL, "disc domains run in the single-instance solver, not the engine");
    if ((int64_t)P.interior.size() > e->max_interior_cap) return fail(FK_ENOMEM, "instance grid exceeds the engine");
    if (free_slot < 0) return fail(FK_EBUSY, "no free engine slot");
    int64_t resident_items = 0;
    for (const SlotInfo &o : e->slots)
        if (o.used) resident_items += o.P.n_items;
    if (resident_items + P.n_items > e->cfg.max_items) return fail(FK_ENOMEM, "engine work-item capacity reached");
    const size_t bytes = instance_bytes(P);
    size_t off = 0;
    if (!e->pool.alloc(bytes, off)) return fail(FK_ENOMEM, "engine pool cannot hold the instance now");
    SlotInfo &S = e->slots[free_slot];
    S.P = std::move(P);
    S.region = {off, bytes};
    S.B = carve(S.P, e->d_pool + off);
    S.B.state = e->d_states + free_slot;    // states live in one contiguous array
    S.iter = 0;
    S.hist_du.clear();
    S.hist_sup.clear();
    S.pdd = false;
    S.tasks.clear();
    const double a = S.P.dom.x1 - S.P.dom.x0, b = S.P.dom.y1 - S.P.dom.y0;
    // mean exit time of a rectangle ~ 0.0351 * 2 a^2 b^2 / (a^2 + b^2) (unit square: 0.0351)
    S.est_cost = 0.0351 * 2.0 * a * a * b * b / (a * a + b * b) / S.P.par.h * (double)S.P.par.M /
                 (double)(S.P.items_a + S.P.items_per_node);
    fkd::Inst D = make_inst(S.P, S.B);
    const hipStream_t s = e->cap_stream;
    st = upload_instance(S.P, S.B, s);
    if (st == FK_OK) {
        hipError_t err = hipMemcpyAsync(e->d_insts + free_slot, &D, sizeof(D), hipMemcpyHostToDevice, s);
        if (err == hipSuccess) err = hipStreamSynchronize(s);
        if (err != hipSuccess) st = hip_fail(err, "engine add");
    }
    if (st != FK_OK) {
        e->pool.release(off, bytes);
        return st;
    }
    e->h_insts[free_slot] = D;
    S.used = true;
    rebuild_tables(e);
    *slot = free_slot;
    return FK_OK;
}

fk_status fk_engine_remove(fk_engine *e, int32_t slot)
{
    if (!e || slot < 0 || slot >= e->cfg.max_instances || !e->slots[slot].used)
        return fail(FK_EINVAL, "no instance in that slot");
    SlotInfo &S = e->slots[slot];
    // the slot's memory may be reused right away: no tick is in flight here
    e->pool.release(S.region.off, S.region.size);
    if (S.pdd) e->pool.release(S.pdd_region.off, S.pdd_region.size);
    S.used = false;
    S.pdd = false;
    S.tasks.clear();
    S.P = HostProblem();
    rebuild_tables(e);
    return FK_OK;
}

fk_status fk_engine_tick(fk_engine *e, fk_iter_report *reports, uint8_t *active_mask)
{
    if (!e) return fail(FK_EINVAL, "engine is NULL");
    const int32_t cap = e->cfg.max_instances;
    if (active_mask) std::memset(active_mask, 0, cap);
    if (e->n_active == 0) return FK_OK;
    const hipStream_t s = e->user_stream ? e->user_stream : e->cap_stream;
    if (e->tables_dirty) {
        FK_HIP(hipMemcpyAsync(e->d_active, e->h_active, (cap + 1) * sizeof(int32_t), hipMemcpyHostToDevice, s));
        FK_HIP(hipMemcpyAsync(e->d_queue, e->h_queue, sizeof(fkd::EngineQueue), hipMemcpyHostToDevice, s));
        if (*e->h_n_tasks > 0)
            FK_HIP(hipMemcpyAsync(e->d_tasks, e->h_tasks, *e->h_n_tasks * sizeof(fkd::PddTask), hipMemcpyHostToDevice,
                                  s));
        FK_HIP(hipMemcpyAsync(e->d_n_tasks, e->h_n_tasks, sizeof(int32_t), hipMemcpyHostToDevice, s));
        e->tables_dirty = false;
    }
    int features = 0;
    for (int32_t a = 0; a < e->n_active; ++a) features |= e->slots[e->h_active[a]].P.features();
    FK_HIP(hipEventRecord(e->ev0, s));
    FK_HIP(hipGraphLaunch(e->exec[features], s));
    FK_HIP(hipEventRecord(e->ev1, s));
    FK_HIP(hipStreamSynchronize(s));
    float ms = 0.0f;
    FK_HIP(hipEventElapsedTime(&ms, e->ev0, e->ev1));
    e->kernel_ms_total += ms;
    e->launches += 1;
    for (int32_t a = 0; a < e->n_active; ++a) {
        const int32_t i = e->h_active[a];
        SlotInfo &S = e->slots[i];
        const fkd::DevState &h = e->h_states[i];
        S.iter += 1;
        double du, sup, se;
        std::memcpy(&du, &h.max_du, 8);
        std::memcpy(&sup, &h.sup, 8);
        std::memcpy(&se, &h.max_se, 8);
        fk_iter_report r{};
        r.n = S.iter;
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
        const size_t nh = S.hist_du.size();
        if (!div && nh >= 5) div = sup >= 1.25 * S.hist_sup[nh - 5] && du >= 1.25 * S.hist_du[nh - 5];
        r.diverging = div ? 1 : 0;
        S.hist_sup.push_back(sup);
        S.hist_du.push_back(du);
        // measured path length orders the next ticks (longest first)
        if (S.P.par.M > 0 && !S.P.interior.empty())
            S.est_cost = (double)r.path_steps / (double)S.P.n_items;
        if (reports) reports[i] = r;
        if (active_mask) active_mask[i] = 1;
    }
    rebuild_tables(e);
    return FK_OK;
}

fk_status fk_engine_get(fk_engine *e, int32_t slot, double *u_reim, double *se_reim)
{
    if (!e || slot < 0 || slot >= e->cfg.max_instances || !e->slots[slot].used)
        return fail(FK_EINVAL, "no instance in that slot");
    const SlotInfo &S = e->slots[slot];
    const size_t nn = S.P.n_nodes();
    const hipStream_t s = e->user_stream ? e->user_stream : e->cap_stream;
    if (u_reim) FK_HIP(hipMemcpyAsync(u_reim, S.B.u64, nn * sizeof(double2), hipMemcpyDeviceToHost, s));
    if (se_reim) FK_HIP(hipMemcpyAsync(se_reim, S.B.se, nn * sizeof(double2), hipMemcpyDeviceToHost, s));
    FK_HIP(hipStreamSynchronize(s));
    return FK_OK;
}

fk_status fk_engine_set_pdd(fk_engine *e, int32_t slot, const int32_t *cuts_x, int32_t n_cuts_x,
                            const int32_t *cuts_y, int32_t n_cuts_y)
{
    if (!e || slot < 0 || slot >= e->cfg.max_instances || !e->slots[slot].used)
        return fail(FK_EINVAL, "no instance in that slot");
    SlotInfo &S = e->slots[slot];
    if (S.iter != 0 || S.pdd) return fail(FK_EINVAL, "set PDD once, before the instance's first tick");
    PddPlan plan;
    fk_status st = plan_pdd(S.P, cuts_x, n_cuts_x, cuts_y, n_cuts_y, plan);
    if (st != FK_OK) return st;
    if (pdd_task_count(e) + (int64_t)plan.blocks.size() > kMaxPddTasks)
        return fail(FK_ENOMEM, "engine block-solve capacity reached");
    // tables, then the right-hand sides (one complex value per grid node)
    const size_t tab_bytes = align256(plan.tables.size() * sizeof(double));
    const size_t bytes = tab_bytes + S.P.n_nodes() * sizeof(double2);
    size_t off = 0;
    if (!e->pool.alloc(bytes, off)) return fail(FK_ENOMEM, "engine pool cannot hold the decomposition now");
    double *tables = (double *)(e->d_pool + off);
    double2 *rhs = (double2 *)(e->d_pool + off + tab_bytes);
    HostProblem P2 = S.P;
    apply_pdd(P2, plan, 2 * (int64_t)e->n_blocks * 4);
    const fkd::Inst D = make_inst(P2, S.B);
    const hipStream_t s = e->cap_stream;
    hipError_t err = hipSuccess;
    if (!plan.tables.empty())
        err = hipMemcpyAsync(tables, plan.tables.data(), plan.tables.size() * sizeof(double), hipMemcpyHostToDevice, s);
    if (err == hipSuccess && !P2.interior.empty())
        err = hipMemcpyAsync(S.B.nodes, P2.interior.data(), P2.interior.size() * sizeof(int32_t),
                             hipMemcpyHostToDevice, s);
    if (err == hipSuccess) err = hipMemcpyAsync(e->d_insts + slot, &D, sizeof(D), hipMemcpyHostToDevice, s);
    if (err == hipSuccess) err = hipStreamSynchronize(s);
    if (err != hipSuccess) {
        // best effort: the device node list and record back to the host's
        const fkd::Inst D0 = make_inst(S.P, S.B);
        (void)hipMemcpyAsync(S.B.nodes, S.P.interior.data(), S.P.interior.size() * sizeof(int32_t),
                             hipMemcpyHostToDevice, s);
        (void)hipMemcpyAsync(e->d_insts + slot, &D0, sizeof(D0), hipMemcpyHostToDevice, s);
        (void)hipStreamSynchronize(s);
        e->pool.release(off, bytes);
        return hip_fail(err, "engine set_pdd");
    }
    S.tasks.clear();
    for (const PddPlan::Block &B : plan.blocks)
        S.tasks.push_back(fkd::PddTask{slot, B.i0, B.i1, B.j0, B.j1, 0, tables + B.tx, tables + B.ty, rhs});
    S.P = std::move(P2);
    S.pdd = true;
    S.pdd_region = {off, bytes};
    e->h_insts[slot] = D;
    rebuild_tables(e);
    return FK_OK;
}

fk_status fk_engine_node_stats(fk_engine *e, int32_t slot, int64_t *sum_j, int64_t *capped)
{
    if (!e || slot < 0 || slot >= e->cfg.max_instances || !e->slots[slot].used)
        return fail(FK_EINVAL, "no instance in that slot");
    const SlotInfo &S = e->slots[slot];
    const size_t nn = S.P.n_nodes();
    const hipStream_t s = e->user_stream ? e->user_stream : e->cap_stream;
    if (sum_j) FK_HIP(hipMemcpyAsync(sum_j, S.B.sum_j, nn * sizeof(int64_t), hipMemcpyDeviceToHost, s));
    if (capped) FK_HIP(hipMemcpyAsync(capped, S.B.capped, nn * sizeof(int64_t), hipMemcpyDeviceToHost, s));
    FK_HIP(hipStreamSynchronize(s));
    return FK_OK;
}

fk_status fk_engine_set_iterate(fk_engine *e, int32_t slot, const double *u_reim, int32_t n, int32_t on_device)
{
    if (!e || slot < 0 || slot >= e->cfg.max_instances || !e->slots[slot].used)
        return fail(FK_EINVAL, "no instance in that slot");
    if (!u_reim || n < 0) return fail(FK_EINVAL, "u_reim is required and n must be >= 0");
    SlotInfo &S = e->slots[slot];
    const hipStream_t s = e->user_stream ? e->user_stream : e->cap_stream;
    const fk_status st = load_iterate(S.P, S.B, u_reim, n, on_device != 0, s);
    if (st != FK_OK) return st;
    S.iter = n;
    S.hist_du.clear();
    S.hist_sup.clear();
    return FK_OK;
}

fk_status fk_engine_timing(fk_engine *e, double *kernel_ms_total, int64_t *launches, int32_t reset)
{
    if (!e) return fail(FK_EINVAL, "engine is NULL");
    if (kernel_ms_total) *kernel_ms_total = e->kernel_ms_total;
    if (launches) *launches = e->launches;
    if (reset) {
        e->kernel_ms_total = 0.0;
        e->launches = 0;
    }
    return FK_OK;
}

fk_status fk_engine_destroy(fk_engine *e)
{
    if (!e) return FK_OK;
    if (e->user_stream) (void)hipStreamSynchronize(e->user_stream);
    if (e->cap_stream) (void)hipStreamSynchronize(e->cap_stream);
    for (int f = 0; f < 16; ++f) {
        if (e->exec[f]) (void)hipGraphExecDestroy(e->exec[f]);
        if (e->graph[f]) (void)hipGraphDestroy(e->graph[f]);
    }
    if (e->ev0) (void)hipEventDestroy(e->ev0);
    if (e->ev1) (void)hipEventDestroy(e->ev1);
    (void)hipFree(e->d_insts);
    (void)hipFree(e->d_states);
    (void)hipFree(e->d_active);
    (void)hipFree(e->d_queue);
    (void)hipFree(e->d_head);
    (void)hipFree(e->d_pool);
    (void)hipFree(e->d_tasks);
    if (e->h_states) (void)hipHostFree(e->h_states);
    if (e->h_queue) (void)hipHostFree(e->h_queue);
    if (e->h_active) (void)hipHostFree(e->h_active);
    if (e->h_tasks) (void)hipHostFree(e->h_tasks);
    if (e->h_n_tasks) (void)hipHostFree(e->h_n_tasks);
    if (e->cap_stream) (void)hipStreamDestroy(e->cap_stream);
    delete e;
    return FK_OK;
}

}  // extern "C"
