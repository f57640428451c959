// lbm_features.hip -- the learned closure's six inputs of every cell of a
// lattice, from its current state (the subgrid model of the Section 5.1 LES
// channel).  They are computed exactly as the fused stream-collide kernel
// computes them before it runs the network: the non-equilibrium momentum
// flux P_c of the canonical populations (with the forcing correction), the
// Smagorinsky excess tau_s - tau from |P_c|, and the invariants of P_c / rho.
// Training data taken from a coarse lattice's own populations therefore has
// the distribution the network meets when it runs inside the lattice.
//
// Bytes per cell: q s read (the populations; the mask word with flags) and
// 24 written.
#include "lattice.h"

namespace lbm {

template <int Q, int ST>
__global__ void __launch_bounds__(LBM_LB_THREADS) k_closure_features(LatticeArgs a, SparseArgs sp, int odd, float *xout)
{
    const int x = blockIdx.x * blockDim.x + threadIdx.x;
    const int y = blockIdx.y * blockDim.y + threadIdx.y;
    const int z = blockIdx.z;
    if (x >= a.nx || y >= a.ny) return;
    const Geom g = make_geom(a, x, y, z);
    float *o = xout + 6 * cidx(a, g);
    const uint32_t m = a.mask ? a.mask[cidx(a, g)] : 0u;
    if (m & SELF_SOLID) {
#pragma unroll
        for (int k = 0; k < 6; ++k) o[k] = __builtin_nanf("");
        return;
    }
    float d[Q];
    load_state<Q, ST>(a, sp, g, m, odd, d);
    float drho;
    const Macro M = moments<Q>(a, d, drho);
    float P[6], Pn[6], xf[6];
    noneq_flux<Q>(a, d, drho, M, P);
    const float excess = smag_excess(a.tau, a.cs, flux_norm(P), M.rho);
    const float ir = rcp(M.rho);
#pragma unroll
    for (int k = 0; k < 6; ++k) Pn[k] = P[k] * ir;
    closure_features(Pn, M.rho, a.tau, excess, xf);
#pragma unroll
    for (int k = 0; k < 6; ++k) o[k] = xf[k];
}

hipError_t launch_closure_features(const LatticeArgs &a, const SparseArgs &sp, int q, int st, int odd, float *x,
                                   hipStream_t s)
{
    const Launch L = lattice_launch(a);
    return dispatch(q, st, [&](auto Q, auto ST) {
        k_closure_features<Q.value, ST.value><<<L.grid, L.block, 0, s>>>(a, sp, odd, x);
        return hipGetLastError();
    });
}

}  // namespace lbm
