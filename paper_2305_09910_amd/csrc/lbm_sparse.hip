// lbm_sparse.hip -- fused in-place stream-collide over the fluid cells only
// (sparse indirect addressing), for domains where solids take much of the
// volume.
//
// The dense kernels move every cell's populations, solid or not: solid
// lanes keep their slots on the even step so that wavefronts write whole
// cache lines.  Here only fluid cells are stored.  They are numbered in row
// order (z, y, x) and kept in chunks of 64, one wavefront each, with the q
// direction segments of a chunk side by side ([chunk][q][64]).  The update
// is the AA pattern of lbm_kernels.hip applied to the fluid index:
//   even step: read slot i of cell k, write slot opposite(i) of cell k;
//   odd step:  read slot opposite(i) of the neighbour x - c_i, write slot i
//              of the neighbour x + c_i;
// where a link is cut (solid neighbour or non-periodic face) the cell's own
// slot stands in, exactly as in the dense kernel.  The neighbours come from
// a table of q - 1 indices per fluid cell ([chunk][q - 1][64], 4 bytes
// each), read on the odd step; on the even step it is read only when the
// domain has velocity or pressure faces, whose cut links need the face.
//
// Bytes per fluid-cell update: 2 q s of populations (s = 4 or 2) on both
// steps, plus 4 (q - 1) of table on odd steps: 152 + 36 = 188 B on average
// for D3Q19 FP32, against 152 B per cell -- fluid or solid -- of the dense
// kernel's even step.  By bytes it pays once solids fill more than about 30%
// of the box; on a 70%-solid porous medium it runs 2.7-2.8 times faster.
#include "lattice.h"

namespace lbm {

// Chunk order over the XCDs: 0 grid order (workgroup b on XCD b mod 8), 1 a
// contiguous range of workgroups per XCD on odd steps, 2 on every step.
// Measured on the 256^3 porous medium (70% solid): 1 is 12-13% faster than 0
// in FP32 and FP16 (the odd step 9-16% faster); 2 gains less in FP32.
#ifndef LBM_SPARSE_REMAP
#define LBM_SPARSE_REMAP 1
#endif

// Workgroup b runs on XCD b mod 8.  The remap hands XCD x the contiguous
// block range of its share (the first nb mod 8 XCDs take one more block), so
// the y and z neighbours that a wavefront gathers on the odd step, a few rows
// further along the fluid order, are read through the same L2.  A bijection
// of [0, nb).
__device__ inline uint32_t sparse_block(int odd)
{
    uint32_t b = blockIdx.x;
    if (LBM_SPARSE_REMAP == 2 || (LBM_SPARSE_REMAP == 1 && odd)) {
        const uint32_t nb = gridDim.x, q = nb / 8u, r = nb % 8u, x = b % 8u, slot = b / 8u;
        b = (x < r ? x * (q + 1u) : r * (q + 1u) + (x - r) * q) + slot;
    }
    return b;
}

template <int Q, int ST, int CL, int COLL>
__global__ void __launch_bounds__(256) k_stream_collide_sparse(LatticeArgs a, SparseArgs sp, int odd)
{
    using S = Store<ST>;
    const uint32_t k = sparse_block(odd) * 256u + threadIdx.x;
    // With the learned closure every lane stays to the end (the network runs
    // across the wavefront), but lanes past the last fluid cell touch no
    // memory; otherwise they leave at once.
    const bool active = k < sp.nf;
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
    const bool mem = CL != CL_MLP || active;
    typename S::T *A = (typename S::T *)a.pdf;
    // neighbour table: all q - 1 entries on the odd step (each serves one
    // read and one write), only with velocity/pressure faces on the even one
    // (entry 0 is unused: the rest population stays in the cell's own slot)
    uint32_t t[Q];
    t[0] = NB_SOLID;
    const bool need = odd || a.any_vp;
    for_dirs<1, Q>([&](auto J) {
        constexpr int j = decltype(J)::value;
        t[j] = need && mem ? __builtin_nontemporal_load(sp.nbt + sp_table<Q>(k, j)) : NB_SOLID;
    });
    float d[Q];
    for_dirs<0, Q>([&](auto I) {
        constexpr int i = decltype(I)::value;
        if (!mem) {
            d[i] = 0.f;
        } else if (i == 0 || !odd) {
            d[i] = S::template ld<true>(A + sp_index<Q>(k, i));
        } else {
            const uint32_t s = t[opp(i)];  // neighbour x - c_i
            d[i] = S::ld(A + (s >= NB_FACE0 ? sp_index<Q>(k, i) : sp_index<Q>(s, opp(i))));
        }
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
        if constexpr (i == 0) {
            S::template st<true>(A + sp_index<Q>(k, 0), d[0]);
        } else {
            const uint32_t e = t[i];  // neighbour x + c_i
            float v = d[i];
            // a link through a velocity or pressure face returns the face's value
            if (a.any_vp && e >= NB_FACE0 && e != NB_SOLID) v = wall_value<Q>(a, (int)(e - NB_FACE0), i, v, M);
            if (!odd)
                S::template st<true>(A + sp_index<Q>(k, opp(i)), v);
            else
                S::st(A + (e >= NB_FACE0 ? sp_index<Q>(k, opp(i)) : sp_index<Q>(e, i)), v);
        }
    });
}

// One thread per fluid cell: its neighbour along each c_j (periodic wrap),
// or the code of the face or solid that cuts the link.
template <int Q>
__global__ void __launch_bounds__(256) k_build_sparse_table(LatticeArgs a, SparseArgs sp, const uint32_t *fcell, uint32_t *T)
{
    const uint32_t k = blockIdx.x * 256u + threadIdx.x;
    if (k >= sp.nf) return;
    const uint32_t c = fcell[k];
    const int x = (int)(c % (uint32_t)a.nx), y = (int)((c / (uint32_t)a.nx) % (uint32_t)a.ny);
    const int z = (int)(c / ((uint32_t)a.nx * (uint32_t)a.ny));
    const Geom g = make_geom(a, x, y, z);
#pragma unroll
    for (int j = 1; j < Q; ++j) {
        const int dx = cdir(j, 0), dy = cdir(j, 1), dz = cdir(j, 2);
        uint32_t e;
        if (face_cut(g, dx, dy, dz)) {
            e = NB_FACE0 + (uint32_t)deciding_face(a, g, dx, dy, dz);
        } else {
            const int32_t f = sp.fmap[nbr(a, g, dx, dy, dz)];
            e = f < 0 ? NB_SOLID : (uint32_t)f;
        }
        T[sp_table<Q>(k, j)] = e;
    }
}

hipError_t launch_build_sparse_table(const LatticeArgs &a, const SparseArgs &sp, int q, const uint32_t *fcell,
                                     uint32_t *table, hipStream_t s)
{
    if (sp.nf == 0) return hipSuccess;
    const dim3 grid((sp.nf + 255) / 256), block(256);
    if (q == 19)
        k_build_sparse_table<19><<<grid, block, 0, s>>>(a, sp, fcell, table);
    else
        k_build_sparse_table<27><<<grid, block, 0, s>>>(a, sp, fcell, table);
    return hipGetLastError();
}

template <int Q, int ST, int COLL>
static void sparse_coll(const LatticeArgs &a, const SparseArgs &sp, int cl, int odd, dim3 grid, hipStream_t s)
{
    if constexpr (COLL == COLL_TRT) {
        if (cl == CL_MLP) {  // the learned closure runs with the TRT collision
            k_stream_collide_sparse<Q, ST, CL_MLP, COLL><<<grid, 256, 0, s>>>(a, sp, odd);
            return;
        }
    }
    if (cl == CL_NONE)
        k_stream_collide_sparse<Q, ST, CL_NONE, COLL><<<grid, 256, 0, s>>>(a, sp, odd);
    else
        k_stream_collide_sparse<Q, ST, CL_SMAG, COLL><<<grid, 256, 0, s>>>(a, sp, odd);
}

hipError_t launch_step_sparse(const LatticeArgs &a, const SparseArgs &sp, int q, int st, int cl, int coll, int odd,
                              hipStream_t s)
{
    if (cl == CL_MLP && coll == COLL_MRT) return hipErrorInvalidValue;
    if (coll == COLL_HRR) return hipErrorInvalidValue;  // HRR runs with the dense AA pattern only
    if (sp.nf == 0) return hipSuccess;
    const dim3 grid((sp.nf + 255) / 256);
    return dispatch(q, st, [&](auto Qc, auto STc) {
        constexpr int Q = decltype(Qc)::value, ST = decltype(STc)::value;
        if (coll == COLL_MRT)
            sparse_coll<Q, ST, COLL_MRT>(a, sp, cl, odd, grid, s);
        else
            sparse_coll<Q, ST, COLL_TRT>(a, sp, cl, odd, grid, s);
        return hipGetLastError();
    });
}

}  // namespace lbm
