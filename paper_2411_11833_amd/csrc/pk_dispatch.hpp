// Launch interface shared by the host library and the per-K kernel objects.
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
};

using PkFn = hipError_t (*)(const ct::Tables*, const PkArgs&, hipStream_t);

// kernel launcher for `split` lanes per configuration and mode (ct::Mode);
// defined in pk_instances.hip compiled once per K
PkFn ct_pick_k1(int split, int mode);
PkFn ct_pick_k2(int split, int mode);
PkFn ct_pick_k3(int split, int mode);
PkFn ct_pick_k4(int split, int mode);
PkFn ct_pick_k5(int split, int mode);
PkFn ct_pick_k6(int split, int mode);
