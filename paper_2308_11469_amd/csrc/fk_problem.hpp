// fk_problem.hpp -- host-side problem setup shared by the single-instance
// solver and the batched engine: validation, node classification, boundary
// values of the grid, work decomposition and the device instance record.
#pragma once

#include <string>
#include <vector>

#include "../../include/fk_helmholtz.h"
#include "fk_device.hpp"

namespace fkh {

void set_error(const std::string &msg);
fk_status fail(fk_status st, const std::string &msg);
fk_status hip_fail(hipError_t e, const char *what);

#define FK_HIP(call)                                                  \
    do {                                                              \
        hipError_t e_ = (call);                                       \
        if (e_ != hipSuccess) return ::fkh::hip_fail(e_, #call);      \
    } while (0)

// Largest row-major copy of u_n (FP32 copy, or the FP64 master) that the
// automatic gather layout keeps row-major.  The vector L1 cache of a CU holds 32 KiB; measured on the
// unit square (FP32, M = 1024), row-major is ahead up to 97x97 (75 KB:
// 2.40e11 against 2.28e11 path-steps/s) and cell-major from 129x129 on
// (257x257: 2.39e11 against 1.35e11).
constexpr size_t kL1GatherBytes = 80 * 1024;
// Largest FP32 row-major copy a single-instance launch stages in LDS (a
// 1024-thread block per CU holds it beside the 16 waves' node accumulators,
// 6 KiB, within the CU's 160 KiB): about 139 x 139 nodes.
constexpr size_t kLdsGridBytes = 152 * 1024;

struct HostProblem {
    fk_domain dom{};
    fk_source src{};
    fk_bc outer{}, inner{};
    fk_params par{};
    std::vector<double> table;        // outer TABLE samples (re, im), copied
    std::vector<uint8_t> cls;         // 0 unknown (interior or reflecting edge), 1 absorbing edge, 2 hole,
                                      // 3 outside a disc domain's disc
    std::vector<int32_t> interior;    // unknown node ids, longest expected paths first
    std::vector<double> grid0;        // initial grid (re, im): 0 interior, g elsewhere
    std::vector<int32_t> ext;         // disc domains: pairs (exterior node, its nearest unknown node)
    int64_t jmax = 0;
    int32_t ppi = 0;                  // paths per (small) work item
    int32_t items_per_node = 0;       // small items per node
    int32_t ppi_a = 0;                // paths per large item (0: none)
    int32_t items_a = 0;              // large items per node, ahead of the small ones
    int64_t n_items = 0;              // all items: nodes x (items_a + items_per_node)
    int32_t cells = 0;                // the gather copy of u_n is cell-major
    int32_t lds_grid = 0;             // single-instance FP32: the row-major copy is staged in LDS
    // optional parts of the stepping loop this instance needs (bit 0 a hole,
    // bit 1 a source term, bit 2 a shift alpha != k^2 or damping, bit 3 a
    // reflecting edge); the path kernel is compiled per set
    int features() const
    {
        return (dom.kind != FK_DOMAIN_RECT ? 1 : 0) | (src.kind != FK_SRC_ZERO ? 2 : 0) |
               (alpha() != par.k * par.k || par.damping != 0.0 ? 4 : 0) | (reflect() ? 8 : 0) |
               (disc_domain() ? fkd::kFeatCurved : 0);
    }
    bool reflect() const { return dom.edge == FK_EDGE_REFLECTING; }
    bool disc_domain() const
    {
        return dom.kind == FK_DOMAIN_DISC_MINUS_RHOMBUS || dom.kind == FK_DOMAIN_DISC_MINUS_DISC;
    }
    double alpha() const { return par.alpha == 0.0 ? par.k * par.k : par.alpha; }
    size_t n_nodes() const { return (size_t)dom.nx * (size_t)dom.ny; }
    size_t n_cells() const { return (size_t)(dom.nx - 1) * (size_t)(dom.ny - 1); }
    // bytes of the gather copy of the iterate: FP32 row-major 8 per node or
    // cells 32 per cell; FP64 cells 64 per cell; none for FP64 row-major
    // (those paths read the FP64 master)
    size_t gather_bytes() const
    {
        if (par.precision == 32) return cells ? 32 * n_cells() : 8 * n_nodes();
        return cells ? 64 * n_cells() : 0;
    }
};

// Validates and prepares a problem.  Returns FK_OK or FK_EINVAL (message set).
// single_instance: the problem runs alone in its launches (the solver), so an
// FP32 iterate that fits LDS is staged there (row-major copy; the automatic
// layout picks it), which a batched launch of mixed instances cannot do.
fk_status setup_problem(const fk_domain *domain, const fk_source *f, const fk_bc *g_outer, const fk_bc *g_inner,
                        const fk_params *params, HostProblem &out, bool single_instance = false);

// Device bytes of one instance's buffers (grids, node list, slots, stats,
// table, state), each part 256-byte aligned.
size_t instance_bytes(const HostProblem &P);

// Carves the instance buffers out of base (device, 256-byte aligned) and
// fills the instance record; uploads nothing.
struct InstanceBuffers {
    double2 *u64;
    void *gather;
    int32_t *nodes;
    fkd::Slot *slots;
    double2 *se;
    int64_t *sum_j, *capped;
    double2 *table;
    fkd::DevState *state;
    int32_t *ext;
};
InstanceBuffers carve(const HostProblem &P, char *base);
fkd::Inst make_inst(const HostProblem &P, const InstanceBuffers &B);

// Uploads the initial grid (FP64 and FP32 copies), node list, table and a
// fresh state (iteration 0, u_0 = 0) on stream s.
fk_status upload_instance(const HostProblem &P, const InstanceBuffers &B, hipStream_t s);

// The gather copy (bytes, gather_bytes() of them) of a grid of complex
// values (re, im interleaved, row-major nodes) in the instance's precision
// and layout.
void gather_copy(const HostProblem &P, const double *grid, std::vector<uint8_t> &out);

// Replaces the iterate on the unknown nodes by u_reim (nx*ny complex, host, or
// device when on_device) and sets the iteration index to n (use_u = 1):
// absorbing-edge and hole nodes keep the problem's data, a disc domain's
// exterior nodes take their nearest unknown node's value, the gather copy is
// rebuilt from the FP64 values, the status record is cleared.  Synchronises s.
fk_status load_iterate(const HostProblem &P, const InstanceBuffers &B, const double *u_reim, int32_t n,
                       bool on_device, hipStream_t s);

// Probabilistic domain decomposition of a problem (Sec. 3's two-stage
// procedure): the interface is the unknown nodes on the grid lines x index in
// cuts_x, y index in cuts_y; the blocks are the unknown nodes between
// consecutive lines (or the edge), each with the DST tables of its two sides
// (offsets into `tables`: 2 (m + 1) sines sqrt(2/(m+1)) sin(pi t/(m+1)),
// then m factors 4 sin^2(pi (q+1) / (2 (m+1)))).
struct PddPlan {
    struct Block {
        int32_t i0, i1, j0, j1;   // unknown nodes [i0, i1) x [j0, j1)
        int32_t tx, ty;           // table offsets of the sides i1 - i0, j1 - j0
    };
    std::vector<Block> blocks;
    std::vector<double> tables;
    std::vector<int32_t> iface;   // the nodes that run paths: the interface and the unknown nodes of
                                  // blocks touching the hole, in the problem's work order
    int32_t max_nodes = 0;        // largest block
};
// A block with a hole node in it or on its frame is not solved: its unknown
// nodes run paths.  FK_EINVAL: a reflecting edge, no cut, cuts not strictly
// increasing within [1, n - 2], or a block wider than 64 nodes.
fk_status plan_pdd(const HostProblem &P, const int32_t *cuts_x, int32_t n_cuts_x, const int32_t *cuts_y,
                   int32_t n_cuts_y, PddPlan &out);
// Makes the PDD node list the problem's work list.  With the automatic item
// size, items are re-sized for the shorter list: the item size is rounded
// down to 64 times a power of two and halved (not below 64) while the
// instance has fewer than target_items items.
void apply_pdd(HostProblem &P, const PddPlan &plan, int64_t target_items);

// Paths per work item when the caller leaves it to the library.
int32_t auto_paths_per_item(int64_t n_interior, int64_t M);

// Resident waves of the path kernel: CUs x (waves per CU), in blocks of four.
int path_kernel_blocks(int waves_per_cu);

double lambda1_bounding_rect(const fk_domain &d);

}  // namespace fkh
