// Internal interface of the batched kernels (zm_batch.hip) and their host
// side (zm_batch_api.hip).  Not part of the public ABI.
#pragma once

#include "zm_internal.h"

#include <hip/hip_runtime.h>

namespace zm {

// Device descriptor of one instance of a batch.
struct InstDesc {
    Mesh m;
    PairShape sh;
    int precision;       // 0 = FP64 pairs, 1 = FP32 pairs
    int block_begin;     // first block of this instance in the point kernels
    int blocks;          // ceil(N / 256)
    int pad_;
    double* Y[3];        // RK3 stage states, 5 planes each
    double* gam;         // 3 planes
    double* q;           // 1 plane
    double* part;        // splits x 3 planes
    double* tie;         // 2 x 3 planes
    double* u;           // 3 planes
    double* V;           // 1 plane
};

// One unit of the persistent pair sweep.
struct WorkItem {
    int inst;
    int patch;
    int split;
    int pad_;
};

// Everything one batched RK3 stage needs (device pointers + host counts).
struct BatchLaunch {
    const InstDesc* table;   // device, count entries, block_begin ascending
    int count;
    int total_blocks;
    const WorkItem* items;   // device; FP64 items then FP32 items, each longest first
    int nitems[2];
    int item_begin[2];
    int* counters;           // device, one work counter per precision
    int persistent_groups;   // workgroups of a persistent pair launch
    bool any_even;           // some instance has an even side (tie pass needed)
};

// Enqueue one RK3 stage (surface, pairs, ties, reduce, update) for every
// instance of the batch.
hipError_t launch_batch_stage(const BatchLaunch& b, int stage, int* nonfinite, hipStream_t s);

}  // namespace zm
