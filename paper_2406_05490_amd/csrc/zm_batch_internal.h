// Internal interface of the batched kernels (zm_batch.hip) and their host
// side (zm_batch_api.hip).  Not part of the public ABI.
#pragma once

#include "zm_host.h"
#include "zm_internal.h"

#include <hip/hip_runtime.h>

#include <vector>

namespace zm {

// Device descriptor of one instance of a batch.
struct InstDesc {
    Mesh m;
    PairShape sh;
    int precision;       // 0 = FP64 pairs, 1 = FP32 pairs
    int block_begin;     // first block of this instance in the point kernels
    int blocks;          // ceil(N / 256)
    int tie_block_begin; // first block of this instance in the tie kernel
    int reduce_block_begin; // first block of this instance in the reduction
    double* Y[3];        // RK3 stage states, 5 planes each
    double* gam;         // 3 planes
    double* q;           // 1 plane
    double* part;        // splits x 3 planes
    double* tie;         // 2 x 3 planes
    double* u;           // 3 planes
    double* V;           // 1 plane
    int* fold;           // tangent-map statistics and far-form flag (kFoldWords ints)
    int* flag;           // set to 1 by the update if this instance's state is not finite (may be NULL)
};

// One unit of the persistent pair sweep.
struct WorkItem {
    int inst;
    int patch;
    int split;
    int pad_;
};

// Items of one persistent pair launch: same precision, targets per lane and
// patch width (one kernel body per launch, so each keeps the register count,
// and with it the occupancy, of the single-instance kernel of that shape).
struct PairGroup {
    int precision;
    int R;
    int px;
    int item_begin;
    int nitems;
};

constexpr int kMaxPairGroups = 18;   // 2 precisions x R in {1, 2, 4} x patch width in {32, 16, 8}

// Everything one batched RK3 stage needs (device pointers + host counts).
struct BatchLaunch {
    const InstDesc* table;   // device, count entries, block_begin ascending
    int count;
    int total_blocks;
    int total_tie_blocks;
    int total_reduce_blocks;
    const WorkItem* items;   // device; grouped by PairGroup, each group longest first
    PairGroup groups[kMaxPairGroups];
    int ngroups;
    int* counters;           // device, one work counter per group
    int persistent_groups;   // workgroups of a persistent pair launch
    bool any_even;           // some instance has an even side (tie pass needed)
};

// Workgroups of the tie kernel for an n1 x n2 mesh (host mirror of the
// device rule in zm_device.h's tie_blocks).
int dev_tie_blocks(int n1, int n2);

// Lanes per point of the split reduction (host mirror of zm_device.h's
// reduce_lanes).
int dev_reduce_lanes(int N, int splits);

// Enqueue one RK3 stage (surface, pairs, ties, reduce, update) for every
// instance of the batch.  Non-finite results are flagged per instance
// through InstDesc::flag.
hipError_t launch_batch_stage(const BatchLaunch& b, int stage, hipStream_t s);

// Enqueue only the persistent pair launches of one stage (one per group),
// each preceded by its work-counter reset.
hipError_t launch_batch_pairs(const BatchLaunch& b, int stage, hipStream_t s);

// Host-side tables for a set of instances: descriptors, pair work items
// grouped by (precision, targets per lane, patch width) and ordered longest
// first within a group, block offsets of the point kernels.
struct TableBuild {
    std::vector<InstDesc> table;
    std::vector<WorkItem> items;
    std::vector<PairGroup> groups;
    int total_blocks = 0;
    int total_tie_blocks = 0;
    int total_reduce_blocks = 0;
    bool any_even = false;
};

// Member i: parameters, pair shape, workspace layout, base address of its
// region and its non-finite flag (may be NULL).
void build_tables(const zm_params* params, const PairShape* shapes, const Layout* layouts,
                  char* const* bases, int* const* flags, int count, TableBuild& out);

}  // namespace zm
