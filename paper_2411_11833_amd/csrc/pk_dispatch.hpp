// Launch interface shared by the host library and the kernel objects.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "ct_tables.hpp"

struct AdamArgs {
    float lr = 0, b1 = 0, b2 = 0, eps = 0, gs = 0;
};

struct PkArgs {
    float *X, *M, *V, *G, *cost, *terms;
    uint8_t* mask;
    int32_t* first_sat;
    const uint8_t* frozen;
    int64_t n, ld;
    AdamArgs a;
    int32_t t;               // update number, used when t_in is null
    const int32_t* t_in;     // device counter of applied updates (t = *t_in + 1), or null
    int32_t* t_out;          // receives t (the other counter slot), or null
    int32_t stop_at_first;   // skip the step if an earlier iteration satisfied
    const float* gw;         // per-particle gradient weights (gradient mode), or null
    const float* wts;        // per-particle term weights [n_terms][ld] (extended kernels), or null
    int32_t* hits;           // cost mode: touching sphere-box pairs per particle, or null
};

// one skeleton of a given length (each length has its own kernels)
using PkFn = hipError_t (*)(const ct::Tables*, const PkArgs&, hipStream_t);

// persistent many-skeleton step
struct BatchArgs {
    const void* skels;       // device ct::BatchSkel[count]
    const int2* items;       // device (skeleton, tile) list
    int32_t n_items;
    int32_t* queue;          // device int[2], zero between launches
    int32_t n_workgroups;
    AdamArgs a;
    int32_t t;
    const int32_t* t_in;
    int32_t* t_out;
};
using BatchFn = hipError_t (*)(const BatchArgs&, hipStream_t);

// defined in pk_instances.hip, compiled once per split (-DCT_SPLIT=1, 2, 4)
// plain (-DCT_EXT=0) and extended (_ext, -DCT_EXT=1: the self-collision pass
// and per-particle term weights compiled in)
PkFn ct_pick_s1(int K, int mode);
PkFn ct_pick_s2(int K, int mode);
PkFn ct_pick_s4(int K, int mode);
PkFn ct_pick_s1_ext(int K, int mode);
PkFn ct_pick_s2_ext(int K, int mode);
PkFn ct_pick_s4_ext(int K, int mode);
BatchFn ct_batch_s1();
BatchFn ct_batch_s2();
BatchFn ct_batch_s4();
BatchFn ct_batch_s1_ext();
BatchFn ct_batch_s2_ext();
BatchFn ct_batch_s4_ext();
