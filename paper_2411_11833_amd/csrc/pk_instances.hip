// Instantiations of the fused particle kernel for one skeleton length K
// (compiled once per K with -DCT_K=<K>, so the six objects build in parallel).
#include "particle_kernel.hpp"
#include "pk_dispatch.hpp"

#ifndef CT_K
#error "compile with -DCT_K=<steps>"
#endif

namespace {

template <int K, int S, int MODE>
hipError_t launch_pk(const ct::Tables* T, const PkArgs& g, hipStream_t st) {
    constexpr int P = ct::WG / (2 * K * S);
    const dim3 grid((unsigned)((g.n + P - 1) / P));
    hipLaunchKernelGGL((ct::particle_kernel<K, S, MODE>), grid, dim3(ct::WG), 0, st, T, g.X, g.M, g.V, g.G,
                       g.cost, g.terms, g.mask, g.first_sat, g.frozen, g.n, g.ld, g.a.lr, g.a.b1, g.a.b2,
                       g.a.eps, g.a.gs, g.t, g.t_in, g.t_out, g.stop_at_first, g.gw);
    return hipGetLastError();
}

template <int K>
PkFn pick(int split, int mode) {
    const int s = split == 4 ? 2 : (split == 2 ? 1 : 0);
    static const PkFn tab[3][3] = {
        {launch_pk<K, 1, ct::MODE_COST>, launch_pk<K, 1, ct::MODE_GRAD>, launch_pk<K, 1, ct::MODE_STEP>},
        {launch_pk<K, 2, ct::MODE_COST>, launch_pk<K, 2, ct::MODE_GRAD>, launch_pk<K, 2, ct::MODE_STEP>},
        {launch_pk<K, 4, ct::MODE_COST>, launch_pk<K, 4, ct::MODE_GRAD>, launch_pk<K, 4, ct::MODE_STEP>},
    };
    if (mode < 0 || mode > 2) return nullptr;
    return tab[s][mode];
}

}  // namespace

#define CT_CAT2(a, b) a##b
#define CT_CAT(a, b) CT_CAT2(a, b)
PkFn CT_CAT(ct_pick_k, CT_K)(int split, int mode) { return pick<CT_K>(split, mode); }
