// Instantiations of the fused particle kernels for one lane split, plain or
// extended (the robot self-collision pass and per-particle term weights
// compiled in), once per combination with -DCT_SPLIT=<1|2|4> -DCT_EXT=<0|1>,
// so the objects build in parallel.
#include "particle_kernel.hpp"
#include "pk_dispatch.hpp"

#ifndef CT_SPLIT
#error "compile with -DCT_SPLIT=<lanes per configuration>"
#endif
#ifndef CT_EXT
#error "compile with -DCT_EXT=<0|1> (extended kernels)"
#endif

namespace {

template <int S, int MODE, int K>
hipError_t launch_pk(const ct::Tables* T, const PkArgs& g, hipStream_t st) {
    constexpr int P = ct::tile_particles(K, S);
    const dim3 grid((unsigned)((g.n + P - 1) / P));
    hipLaunchKernelGGL((ct::particle_kernel<S, MODE, K, CT_EXT != 0>), grid, dim3(ct::WG), 0, st, T, g.X, g.M, g.V, g.G, g.cost,
                       g.terms, g.mask, g.first_sat, g.frozen, g.n, g.ld, g.a.lr, g.a.b1, g.a.b2, g.a.eps, g.a.gs,
                       g.t, g.t_in, g.t_out, g.stop_at_first, g.gw, g.wts, g.hits);
    return hipGetLastError();
}

template <int S>
hipError_t launch_batch(const BatchArgs& g, hipStream_t st) {
    hipLaunchKernelGGL((ct::batch_kernel<S, CT_EXT != 0>), dim3((unsigned)g.n_workgroups), dim3(ct::WG), 0, st,
                       static_cast<const ct::BatchSkel*>(g.skels), g.items, g.n_items, g.queue, g.a.lr, g.a.b1,
                       g.a.b2, g.a.eps, g.t, g.t_in, g.t_out);
    return hipGetLastError();
}

template <int S, int K>
PkFn pick_k(int mode) {
    static const PkFn tab[3] = {launch_pk<S, ct::MODE_COST, K>, launch_pk<S, ct::MODE_GRAD, K>,
                                launch_pk<S, ct::MODE_STEP, K>};
    return (mode >= 0 && mode <= 2) ? tab[mode] : nullptr;
}

template <int S>
PkFn pick(int K, int mode) {
    switch (K) {
        case 1: return pick_k<S, 1>(mode);
        case 2: return pick_k<S, 2>(mode);
        case 3: return pick_k<S, 3>(mode);
        case 4: return pick_k<S, 4>(mode);
        case 5: return pick_k<S, 5>(mode);
        case 6: return pick_k<S, 6>(mode);
        default: return nullptr;
    }
}

}  // namespace

#define CT_CAT2(a, b) a##b
#define CT_CAT(a, b) CT_CAT2(a, b)
#if CT_EXT
#define CT_SUFFIX _ext
#else
#define CT_SUFFIX
#endif
PkFn CT_CAT(CT_CAT(ct_pick_s, CT_SPLIT), CT_SUFFIX)(int K, int mode) { return pick<CT_SPLIT>(K, mode); }
BatchFn CT_CAT(CT_CAT(ct_batch_s, CT_SPLIT), CT_SUFFIX)() { return launch_batch<CT_SPLIT>; }
