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
// [i0, i1) x [j0, j1) between two interface lines (or the edge), and the
// offsets of its DST tables for the sizes i1 - i0 and j1 - j0.
constexpr int kPddMaxSide = 64;
struct PddBlock {
    int32_t i0, i1, j0, j1;
    int32_t tx, ty;
};
}  // namespace fkd

namespace fkk {
// features: bit 0 some instance has a hole, bit 1 a source term, bit 2 a
// shift alpha != k^2 or a damping, bit 3 a reflecting edge
// l1_grid: every instance reads a row-major copy (picks the four-wave build
// of the plain FP64 kernel)
hipError_t launch_stream(int precision, int features, const fkd::Inst *d_insts, const fkd::EngineQueue *Q,
                         unsigned long long *head, int n_blocks, hipStream_t s, bool l1_grid = false);
hipError_t launch_reset(const fkd::Inst *d_insts, const int32_t *which, int32_t n, const int32_t *n_dev,
                        unsigned long long *head, hipStream_t s);
hipError_t launch_update(const fkd::Inst *d_insts, const int32_t *which, int32_t n_inst, const int32_t *n_dev,
                         int32_t max_interior, hipStream_t s);
hipError_t launch_advance(const fkd::Inst *d_insts, const int32_t *which, int32_t n, const int32_t *n_dev,
                          hipStream_t s);
// The blocks of one PDD step: right-hand sides into rhs (per grid node),
// then the fast-diagonalisation solve of every block and component, written
// into the iterate and its gather copy.  max_nodes: the largest block.
hipError_t launch_pdd_blocks(const fkd::Inst *d_inst, const fkd::PddBlock *blocks, int32_t n_blocks,
                             int32_t max_nodes, const double *tables, double2 *rhs, hipStream_t s);
hipError_t launch_debug_philox(uint32_t k0, uint32_t k1, const uint4 *ctr, int64_t n, uint4 *out, hipStream_t s);
hipError_t launch_debug_normals(int precision, const uint2 *words, int64_t n, double2 *z, hipStream_t s);
hipError_t launch_debug_paths(int precision, const fkd::Inst *d_inst, const int32_t *nodes, const int64_t *ms,
                              int64_t n, long long *J, double2 *score, double2 *xj, hipStream_t s);
}  // namespace fkk
