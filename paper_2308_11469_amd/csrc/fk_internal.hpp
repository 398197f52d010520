// fk_internal.hpp -- declarations shared by the kernels and the host runtime
// of the HIP library (not part of the C ABI).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace fkd {
struct Inst;
struct DevState;
struct Slot;

// Segment table of a path launch (device): segment s covers the items of
// instance seg_inst[s]; seg_end is the inclusive prefix sum of item counts.
constexpr int kMaxSlots = 1024;
struct EngineQueue {
    int32_t n_seg;
    int32_t pad;
    int64_t seg_end[kMaxSlots];
    int32_t seg_inst[kMaxSlots];
};

// One subdomain of the probabilistic domain decomposition: the unknown nodes
// [i0, i1) x [j0, j1) of instance `inst` (an index into the instance array)
// between two interface lines (or the edge), the DST tables of its sides
// i1 - i0 and j1 - j0 (2 (m + 1) sines, then m eigenvalue factors), and the
// right-hand-side buffer of its instance (one complex value per grid node).
constexpr int kPddMaxSide = 64;
struct PddTask {
    int32_t inst, i0, i1, j0, j1, pad;
    const double *tx, *ty;
    double2 *rhs;
};
}  // namespace fkd

namespace fkk {
// features: bit 0 some instance has a hole, bit 1 a source term, bit 2 a
// shift alpha != k^2 or a damping, bit 3 a reflecting edge
// l1_grid: every instance reads a row-major copy (picks the four-wave build
// of the plain FP64 kernel)
// lds_bytes > 0: one FP32 instance without a reflecting edge whose row-major
// copy (lds_bytes) is staged in LDS by 1024-thread blocks (n_blocks / 4 of them)
hipError_t launch_stream(int precision, int features, const fkd::Inst *d_insts, const fkd::EngineQueue *Q,
                         unsigned long long *head, int n_blocks, hipStream_t s, bool l1_grid = false,
                         size_t lds_bytes = 0);
hipError_t launch_reset(const fkd::Inst *d_insts, const int32_t *which, int32_t n, const int32_t *n_dev,
                        unsigned long long *head, hipStream_t s);
hipError_t launch_update(const fkd::Inst *d_insts, const int32_t *which, int32_t n_inst, const int32_t *n_dev,
                         int32_t max_interior, hipStream_t s);
hipError_t launch_advance(const fkd::Inst *d_insts, const int32_t *which, int32_t n, const int32_t *n_dev,
                          hipStream_t s);
// Disc domains: the exterior nodes of one instance take the values of their
// nearest unknown nodes (after launch_update, on the same stream).
hipError_t launch_extend(const fkd::Inst *d_inst, int32_t n_ext, hipStream_t s);
// The blocks of one PDD step: right-hand sides into each task's rhs buffer,
// then the fast-diagonalisation solve of every block and component, written
// into the iterate and its gather copy.  The task count is *n_dev when given
// (graph replays read it from the device), else n; `grid` workgroups (per
// component) loop over the tasks; max_nodes bounds the largest block.
hipError_t launch_pdd(const fkd::Inst *d_insts, const fkd::PddTask *tasks, int32_t n, const int32_t *n_dev,
                      int32_t grid, int32_t max_nodes, hipStream_t s);
hipError_t launch_debug_philox(uint32_t k0, uint32_t k1, const uint4 *ctr, int64_t n, uint4 *out, hipStream_t s);
hipError_t launch_debug_normals(int precision, const uint2 *words, int64_t n, double2 *z, hipStream_t s);
hipError_t launch_debug_paths(int precision, const fkd::Inst *d_inst, const int32_t *nodes, const int64_t *ms,
                              int64_t n, long long *J, double2 *score, double2 *xj, hipStream_t s);
}  // namespace fkk
