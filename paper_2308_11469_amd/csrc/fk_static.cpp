// fk_static.cpp -- one fixed-point iteration with no device allocation.
//
// fk_helmholtz_step_static runs the iteration of fk_helmholtz_iterate
// (reset, path kernel, update, index advance) for a problem given by value,
// with all its working memory (instance record, work queue and head, the
// iterate's master and gather copies, node list, node slots, statistics,
// boundary table, status) in one file-scope device array of fixed size.  The
// caller passes u_n and receives u_{n+1} in its own device buffers.
//
// The array's name is a host-side stand-in in host code: its device address
// comes from hipGetSymbolAddress, taken once per device with that device
// current, and only that address is used on the host.
#include <cmath>
#include <cstring>
#include <mutex>
#include <vector>

#include "fk_internal.hpp"
#include "fk_problem.hpp"

using namespace fkh;

namespace {

static __device__ __align__(256) unsigned char scratch[FK_STATIC_SCRATCH_BYTES];

constexpr int kMaxDevices = 64;
std::mutex g_mu;
void *g_scratch[kMaxDevices] = {};

size_t align256(size_t b) { return (b + 255) & ~(size_t)255; }

// The device address of the current device's copy of the array.
fk_status scratch_address(void **out)
{
    int dev = 0;
    FK_HIP(hipGetDevice(&dev));
    if (dev < 0 || dev >= kMaxDevices) return fail(FK_EDEVICE, "device index beyond the static scratch table");
    std::lock_guard<std::mutex> lock(g_mu);
    if (!g_scratch[dev]) {
        void *ptr = nullptr;
        FK_HIP(hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)));
        if (!ptr) return fail(FK_EDEVICE, "hipGetSymbolAddress returned no address for the static scratch");
        g_scratch[dev] = ptr;
    }
    *out = g_scratch[dev];
    return FK_OK;
}

}  // namespace

extern "C" {

fk_status fk_helmholtz_step_static(const fk_domain *domain, const fk_source *f, const fk_bc *g_outer,
                                   const fk_bc *g_inner, const fk_params *params, const double *u_n, int32_t n,
                                   double *u_next, double *se, void *hip_stream, fk_iter_report *report)
{
    if (!u_next) return fail(FK_EINVAL, "u_next is required");
    if (n < 0) return fail(FK_EINVAL, "n must be >= 0");
    if (n > 0 && !u_n) return fail(FK_EINVAL, "u_n is required for n > 0 (NULL means u_0 = 0)");
    HostProblem P;
    fk_status st = setup_problem(domain, f, g_outer, g_inner, params, P, true);
    if (st != FK_OK) return st;
    // record | queue | head | instance buffers, as in a solver's arena
    const size_t need = align256(sizeof(fkd::Inst)) + align256(sizeof(fkd::EngineQueue)) + 256 + instance_bytes(P);
    if (need > (size_t)FK_STATIC_SCRATCH_BYTES)
        return fail(FK_EINVAL, "the problem needs " + std::to_string(need) + " bytes of working memory; the static "
                    "scratch holds " + std::to_string((size_t)FK_STATIC_SCRATCH_BYTES));
    void *base = nullptr;
    if ((st = scratch_address(&base)) != FK_OK) return st;
    const hipStream_t s = (hipStream_t)hip_stream;
    char *p = (char *)base;
    fkd::Inst *d_inst = (fkd::Inst *)p;
    p += align256(sizeof(fkd::Inst));
    fkd::EngineQueue *d_queue = (fkd::EngineQueue *)p;
    p += align256(sizeof(fkd::EngineQueue));
    unsigned long long *d_head = (unsigned long long *)p;
    p += 256;
    const InstanceBuffers B = carve(P, p);
    const fkd::Inst D = make_inst(P, B);
    // the previous call's contents are overwritten: grid, node list, table,
    // zeroed slots and statistics, fresh status (u_0 = 0)
    if ((st = upload_instance(P, B, s)) != FK_OK) return st;
    if (u_n && (st = load_iterate(P, B, u_n, n, true, s)) != FK_OK) return st;
    fkd::EngineQueue q;
    std::memset(&q, 0, sizeof(q));
    q.n_seg = 1;
    q.seg_end[0] = P.n_items;
    q.seg_inst[0] = 0;
    FK_HIP(hipMemcpyAsync(d_inst, &D, sizeof(D), hipMemcpyHostToDevice, s));
    FK_HIP(hipMemcpyAsync(d_queue, &q, sizeof(q), hipMemcpyHostToDevice, s));
    FK_HIP(fkk::launch_reset(d_inst, nullptr, 1, nullptr, d_head, s));
    FK_HIP(fkk::launch_stream(P.par.precision, P.features(), d_inst, d_queue, d_head,
                              path_kernel_blocks(P.par.waves_per_cu), s, P.cells == 0,
                              P.lds_grid ? P.n_nodes() * 8 : 0));
    FK_HIP(fkk::launch_update(d_inst, nullptr, 1, nullptr, (int32_t)P.interior.size(), s));
    FK_HIP(fkk::launch_extend(d_inst, (int32_t)(P.ext.size() / 2), s));
    FK_HIP(fkk::launch_advance(d_inst, nullptr, 1, nullptr, s));
    const size_t nn = P.n_nodes();
    FK_HIP(hipMemcpyAsync(u_next, B.u64, nn * sizeof(double2), hipMemcpyDeviceToDevice, s));
    if (se) FK_HIP(hipMemcpyAsync(se, B.se, nn * sizeof(double2), hipMemcpyDeviceToDevice, s));
    fkd::DevState h;
    FK_HIP(hipMemcpyAsync(&h, B.state, sizeof(h), hipMemcpyDeviceToHost, s));
    FK_HIP(hipStreamSynchronize(s));
    if (report) {
        fk_iter_report r{};
        double du, sup, sem;
        std::memcpy(&du, &h.max_du, 8);
        std::memcpy(&sup, &h.sup, 8);
        std::memcpy(&sem, &h.max_se, 8);
        r.n = n + 1;
        r.max_du = du;
        r.sup = sup;
        r.max_se = sem;
        r.noise_floor = 4.0 * sem;
        r.path_steps = (int64_t)h.path_steps;
        r.capped = (int64_t)h.capped;
        r.nonfinite = (int64_t)h.nonfinite;
        r.step_ms = 0.0;
        r.noise_ratio = h.ratio_n ? (double)h.ratio_fx * 0x1p-20 / (double)h.ratio_n : 0.0;
        r.diverging = (!(std::isfinite(du) && std::isfinite(sup)) || r.nonfinite > 0) ? 1 : 0;
        *report = r;
    }
    double du;
    std::memcpy(&du, &h.max_du, 8);
    if (!std::isfinite(du) || h.nonfinite > 0)
        return fail(FK_EDIVERGED, "the iterate is not finite after iteration " + std::to_string(n + 1));
    return FK_OK;
}

}  // extern "C"
