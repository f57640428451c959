// lbm_et.hip -- fused in-place stream-collide with the Esoteric Twist.
//
// The in-place streaming scheme the paper's LAGOON runs use (Section 5.2),
// as an alternative to the AA pattern of lbm_kernels.hip, on the same store
// ([z][y][q][x] rows of direction segments, deviations f_i - w_i) and with
// the same collision operators.
//
// Every step has the same access pattern.  Cell x reads f_i from location
// x + max(-c_i, 0) and writes its post-collision value of direction i to
// location x + max(c_i, 0): only the cell itself and its positive
// neighbours are touched.  Which of the two slots i, opposite(i) at a
// location holds direction i alternates from step to step (the twist):
// after an even number of steps f_i sits in slot i, after an odd number in
// slot opposite(i).  So on a step that starts from time t,
//   read  f_i   from slot P(i)           at x + max(-c_i, 0),
//   write f*_i  into slot P(opposite(i)) at x + max(c_i, 0),
// with P the identity for even t and opposite() for odd t.  The slot
// written at x + max(c_i, 0) is the one cell x + c_i reads next step, and the
// set of slots a cell reads equals the set it writes, so the update is race
// free in place.
//
// A link cut by a solid neighbour or a non-periodic face is closed by
// writing into slot P(i) at the same location instead: that is the slot
// from which the cell reads direction opposite(i) on the next step, and on
// this step no other cell touches it (it belongs to the solid neighbour, or
// to a ghost layer one cell thick beyond each non-periodic + face).  Reads
// therefore need no boundary logic at all.  Velocity and pressure faces
// modify the returned value with the emitting cell's own velocity, as on the
// AA path.  Solid cells do nothing.
#include "lattice.h"

namespace lbm {

// Slot holding direction i after an even (P = identity) or odd (P =
// opposite) number of steps.
__device__ inline int twist(int i, int odd) { return odd ? opp(i) : i; }

template <int Q, int ST, int CL, bool MASK, int COLL>
__global__ void __launch_bounds__(LBM_LB_THREADS, LBM_MIN_WAVES) k_stream_collide_et(LatticeArgs a, int odd)
{
    using S = Store<ST>;
    const int x = blockIdx.x * blockDim.x + threadIdx.x;
    const int y = blockIdx.y * blockDim.y + threadIdx.y;
    const int z = blockIdx.z;
    // With the learned closure every lane stays to the end (the network runs
    // across the wavefront); otherwise lanes outside the domain or on solid
    // cells leave at once.
    bool active = x < a.nx && y < a.ny;
    if constexpr (CL != CL_MLP) {
        if (!active) return;
    }
    [[maybe_unused]] const uint32_t *tab = nullptr;
    if constexpr (CL == CL_MLP) {
        __shared__ uint32_t tab_lds[TAB_WORDS * 64];
        stage_mlp_table(a, tab_lds);
        __syncthreads();
        tab = tab_lds;
    }
    const Geom g = make_geom(a, active ? x : 0, active ? y : 0, z);
    uint32_t m = 0;
    if constexpr (MASK) {
        m = active ? a.mask[cidx(a, g)] : 0u;
        if (m & SELF_SOLID) {
            if constexpr (CL != CL_MLP) return;
            active = false;
        }
    }
    typename S::T *A = (typename S::T *)a.pdf;
    float d[Q];
    // read side: a line is shared with the neighbouring wavefront only when
    // shifted along x (c_x < 0); the others stream with the nontemporal hint
    for_dirs<0, Q>([&](auto I) {
        constexpr int i = decltype(I)::value;
        constexpr bool nt = LBM_NT_POLICY == 2 || (LBM_NT_POLICY == 1 && cdir(i, 0) >= 0);
        const uint64_t k = et_index<Q>(a, g, twist(i, odd), cdir(i, 0) < 0, cdir(i, 1) < 0, cdir(i, 2) < 0);
        d[i] = (CL != CL_MLP || active) ? S::template ld<nt>(A + k) : 0.f;
    });

    float drho;
    const Macro M = moments<Q>(a, d, drho);
    float wp, wm;
    closure_rates<Q, CL>(a, tab, d, drho, M, active, wp, wm);
    if constexpr (COLL == COLL_MRT)
        mrt_collide<Q>(a, d, drho, M, wp);
    else
        trt_collide<Q>(a, d, drho, M, wp, wm);
    if constexpr (CL == CL_MLP) {
        if (!active) return;
    }

    for_dirs<0, Q>([&](auto I) {
        constexpr int i = decltype(I)::value;
        constexpr int dx = cdir(i, 0), dy = cdir(i, 1), dz = cdir(i, 2);
        constexpr bool nt = LBM_NT_POLICY == 2 || (LBM_NT_POLICY == 1 && dx <= 0);
        const bool fcut = face_cut(g, dx, dy, dz);
        const bool cut = fcut || (MASK && ((m >> i) & 1u));
        float v = d[i];
        if (a.any_vp && fcut) v = wall_value<Q>(a, deciding_face(a, g, dx, dy, dz), i, v, M);
        const int slot = cut ? twist(i, odd) : twist(opp(i), odd);
        S::template st<nt>(A + et_index<Q>(a, g, slot, dx > 0, dy > 0, dz > 0), v);
    });
}

template <int Q, int ST, int COLL>
static void et_coll(const LatticeArgs &a, int cl, bool mk, int odd, const Launch &L, hipStream_t s)
{
    if constexpr (COLL == COLL_TRT) {
        if (cl == CL_MLP) {  // the learned closure runs with the TRT collision
            if (mk)
                k_stream_collide_et<Q, ST, CL_MLP, true, COLL><<<L.grid, L.block, 0, s>>>(a, odd);
            else
                k_stream_collide_et<Q, ST, CL_MLP, false, COLL><<<L.grid, L.block, 0, s>>>(a, odd);
            return;
        }
    }
    if (cl == CL_NONE) {
        if (mk)
            k_stream_collide_et<Q, ST, CL_NONE, true, COLL><<<L.grid, L.block, 0, s>>>(a, odd);
        else
            k_stream_collide_et<Q, ST, CL_NONE, false, COLL><<<L.grid, L.block, 0, s>>>(a, odd);
    } else {
        if (mk)
            k_stream_collide_et<Q, ST, CL_SMAG, true, COLL><<<L.grid, L.block, 0, s>>>(a, odd);
        else
            k_stream_collide_et<Q, ST, CL_SMAG, false, COLL><<<L.grid, L.block, 0, s>>>(a, odd);
    }
}

hipError_t launch_step_et(const LatticeArgs &a, int q, int st, int cl, int coll, int odd, hipStream_t s)
{
    if (cl == CL_MLP && coll == COLL_MRT) return hipErrorInvalidValue;
    if (coll == COLL_HRR) return hipErrorInvalidValue;  // HRR runs with the dense AA pattern only
    const Launch L = lattice_launch(a);
    const bool mk = a.mask != nullptr;
    return dispatch(q, st, [&](auto Qc, auto STc) {
        constexpr int Q = decltype(Qc)::value, ST = decltype(STc)::value;
        if (coll == COLL_MRT)
            et_coll<Q, ST, COLL_MRT>(a, cl, mk, odd, L, s);
        else
            et_coll<Q, ST, COLL_TRT>(a, cl, mk, odd, L, s);
        return hipGetLastError();
    });
}

}  // namespace lbm
