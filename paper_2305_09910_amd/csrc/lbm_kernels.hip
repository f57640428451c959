// lbm_kernels.hip -- fused in-place stream-collide kernels for gfx950.
//
// One population set lives in HBM as deviations d_i = f_i - w_i, in rows of
// q direction segments [z][y][q][x]: structure of arrays within each row,
// so every wavefront access to one direction is contiguous, with the q
// segments of a row kept together in one block.  Streaming (the paper's Eq. (2)) and collision
// (Eq. (1), read as TRT with Guo forcing) are fused into one kernel per time
// step with the AA access pattern, an in-place scheme of the same family as
// the Esoteric Twist the paper's LAGOON runs use (Section 5.2):
//
//   even step: cell x reads d_i from its own slot i, collides, and writes
//              the post-collision value of direction i into its own slot
//              opposite(i);
//   odd step:  cell x reads d_i from slot opposite(i) of cell x - c_i,
//              collides, and writes direction i into slot i of cell x + c_i.
//
// After an odd step the array holds the canonical post-stream state in the
// natural slots; after an even step the post-collision values sit in
// swapped slots of the emitting cell.  In both steps the set of slots a cell
// reads equals the set it writes, so the update is race free in place.
//
// Walls: a link cut by a wall face or a solid neighbour is closed at write
// time inside the emitting cell: the (possibly modified) value goes into
// the cell's own slot opposite(i), which is exactly where that cell reads
// its returning population next step.  Velocity and pressure faces modify
// the value there with the emitting cell's own velocity.
//
// The kernel is bound by HBM bandwidth (every population is read once and
// written once per step); no matrix cores are used here.  All arithmetic is
// FP32 on deviations, which keeps small forcing increments above the FP32
// rounding of w_i.
#include "lattice.h"

namespace lbm {

// ---------------------------------------------------------------------------
// the fused stream-collide kernel
// ---------------------------------------------------------------------------
// flags: bit 0 the step parity (1: odd step); bit 1 (SC_SOLID_ODD): on the
// odd step solid lanes write zero deviations into their own slots (see
// below); bit 2
// (SC_MASK_RUNS): mask words only in runs that touch a solid
template <int Q, int ST, int CL, bool MASK, int COLL>
__global__ void __launch_bounds__(LBM_LB_THREADS, LBM_MIN_WAVES)
    k_stream_collide(LatticeArgs a, int flags, [[maybe_unused]] HrrArgs h)
{
    using S = Store<ST>;
    const int odd = flags & 1;
    constexpr bool kUnified =
        LBM_UNIFIED == 1 || (LBM_UNIFIED == 2 && (MASK || ST == ST_F32) && CL != CL_MLP);
    const int x = blockIdx.x * blockDim.x + threadIdx.x;
    const int y = blockIdx.y * blockDim.y + threadIdx.y;
    const int z = blockIdx.z;
    bool active = x < a.nx && y < a.ny;
    // The learned closure runs on the matrix cores across the whole
    // wavefront, so with it every lane stays to the end; otherwise lanes
    // outside the domain or on solid cells leave at once.
    if constexpr (CL != CL_MLP) {
        if (!active) return;
    }
    [[maybe_unused]] const uint32_t *tab = nullptr;
    if constexpr (CL == CL_MLP) {
        // the per-lane operand table of the network, staged once per workgroup
        __shared__ uint32_t tab_lds[TAB_WORDS * 64];
        stage_mlp_table(a, tab_lds);
        __syncthreads();
        tab = tab_lds;
    }
    // Solid cells on the even step: their lanes load and store their own
    // slots unchanged, in the same instructions as the fluid lanes of the
    // wavefront.  No other cell touches a solid cell's slots, so this is race
    // free, and every cache line the wavefront writes is then written whole;
    // lanes that skip would leave holes in the lines along sphere surfaces,
    // and partially written lines cost ~20% of the even step's time on the
    // 384^3 obstacle flow.  On the odd step no fluid cell reads or writes a
    // solid cell's slots either (links into a solid are cut, and cut links
    // use the fluid cell's own slots), so with SC_SOLID_ODD a solid lane
    // writes zero deviations into its own slots on the odd step, filling the
    // holes that solid cells leave in the lines its row's neighbours write
    // (no cell ever reads a solid cell's slots, and the state readers report
    // solid cells as at rest).  That costs the solid cells' store bytes: it
    // pays on sparse solids (384^3 obstacle flow, 10% solid: odd step -4%
    // against no fill) and not on dense ones (70%-solid porous medium), so
    // the host sets the flag by the solid fraction.
    constexpr bool kKeepSolid = MASK && kUnified && CL != CL_MLP;
    bool keep = false;
    const Geom g = make_geom(a, active ? x : 0, active ? y : 0, z);
    uint32_t m = 0;
    if constexpr (MASK) {
        // with SC_MASK_RUNS the cell's mask word only where its run of 64
        // cells touches a solid
        if (active && (!(flags & SC_MASK_RUNS) || a.mask[cells(a) + (uint64_t)g.frow * mask_runs(a.nx) + ((uint32_t)x >> 6)]))
            m = a.mask[cidx(a, g)];
        if (m & SELF_SOLID) {
            if constexpr (kKeepSolid) {
                if (odd) {
                    if (flags & SC_SOLID_ODD) {
                        // no cell reads a solid cell's slots (state readers
                        // report solids as at rest), so zero deviations do
                        typename S::T *A = (typename S::T *)a.pdf;
#pragma unroll
                        for (int i = 0; i < Q; ++i) S::st(A + pidx<Q>(a, i, g.row, g.x), 0.0f);
                    }
                    return;
                }
                keep = true;
            } else {
                if constexpr (CL != CL_MLP) return;
                active = false;
            }
        }
    }
    // no link of this cell crosses a non-periodic face: the common case,
    // without face logic (solid neighbours are handled inside the plain path)
    const bool plain = !(g.cxl || g.cxh || g.cyl || g.cyh || g.czl || g.czh);
    float d[Q];
    if (CL == CL_MLP && !active) {
#pragma unroll
        for (int i = 0; i < Q; ++i) d[i] = 0.f;
    } else if (kUnified) {
        load_all<Q, ST, MASK>(a, g, m, odd, d);
    } else if (plain) {
        load_plain<Q, ST, MASK>(a, g, m, odd, d);
    } else {
        load_canonical<Q, ST>(a, g, m, odd, d);
    }

    float drho;
    const Macro M = moments<Q>(a, d, drho);
    float wp, wm;
    closure_rates<Q, CL>(a, tab, d, drho, M, active, wp, wm);
    if constexpr (COLL == COLL_MRT) {
        mrt_collide<Q>(a, d, drho, M, wp, keep);
    } else if constexpr (COLL == COLL_HRR) {
        // finite-difference gradient of the previous step's velocities; this
        // step's velocities go to the other field (solid cells keep zeros)
        float G[3][3] = {};
        if (!keep) {
            fd_gradient<Q>(a, h, g, m, G);
            h.unext[cidx(a, g)] = M.ux;
            h.unext[cells(a) + cidx(a, g)] = M.uy;
            h.unext[2 * cells(a) + cidx(a, g)] = M.uz;
        }
        hrr_collide<Q>(a, h.sigma, G, d, drho, M, keep);
    } else {
        trt_collide<Q>(a, d, drho, M, wp, wm, keep);
    }
    if constexpr (CL == CL_MLP) {
        if (!active) return;
    }

    typename S::T *A = (typename S::T *)a.pdf;
    if (kUnified) {
        store_all<Q, ST, MASK, COLL != COLL_TRT>(a, g, m, odd, d, M, keep);
    } else if (plain) {
        store_plain<Q, ST, MASK>(a, g, m, odd, d);
    } else if (!odd) {
#pragma unroll
        for (int i = 0; i < Q; ++i) {
            float v = d[i];
            if (a.any_vp) {
                const int dx = cdir(i, 0), dy = cdir(i, 1), dz = cdir(i, 2);
                if (face_cut(g, dx, dy, dz)) v = wall_value<Q>(a, deciding_face(a, g, dx, dy, dz), i, v, M);
            }
            S::st(A + pidx<Q>(a, opp(i), g.row, g.x), v);
        }
    } else {
#pragma unroll
        for (int i = 0; i < Q; ++i) {
            const int dx = cdir(i, 0), dy = cdir(i, 1), dz = cdir(i, 2);
            const bool fcut = face_cut(g, dx, dy, dz);
            const bool cut = fcut || ((m >> i) & 1u);
            float v = d[i];
            if (a.any_vp && fcut) v = wall_value<Q>(a, deciding_face(a, g, dx, dy, dz), i, v, M);
            const uint64_t own = pidx<Q>(a, opp(i), g.row, g.x);
            const uint64_t dst = pidx_nbr<Q>(a, g, i, dx, dy, dz);
            S::st(A + (cut ? own : dst), v);
        }
    }
}

// Even step of 16-bit storage without a solid mask, two neighbouring cells
// per thread.  A wavefront access of one 16-bit value per lane covers a
// single 128-byte line, and such accesses reach only ~93% of the bandwidth of
// 4-byte ones; here each lane loads and stores one aligned 32-bit word per
// direction (cells x0 and x0 + 1, x0 even), so a wavefront moves two lines
// per instruction as the FP32 kernel does (even step 2-6% faster, the whole
// step 2-4% on the FP16/BF16 channels).  The per-cell arithmetic is the
// step kernel's: moments, closure rates, collision, wall values of cut links.
// Needs nx a multiple of 128 (whole wavefronts of pairs; rows start on lines).
#ifndef LBM_PAIR16
#define LBM_PAIR16 1
#endif

template <int Q, int ST, int CL, int COLL>
__global__ void __launch_bounds__(256, LBM_MIN_WAVES) k_even_pair16(LatticeArgs a)
{
    using S = Store<ST>;
    const int x0 = 2 * (int)(blockIdx.x * blockDim.x + threadIdx.x);
    const int y = blockIdx.y * blockDim.y + threadIdx.y;
    const int z = blockIdx.z;
    if (x0 >= a.nx || y >= a.ny) return;
    const Geom g[2] = {make_geom(a, x0, y, z), make_geom(a, x0 + 1, y, z)};
    // the row's direction segments start on 128-byte lines and x0 is even:
    // every word below is 4-byte aligned
    uint32_t *R = (uint32_t *)((typename S::T *)a.pdf + pidx<Q>(a, 0, g[0].row, x0));
    const uint32_t pitch = (uint32_t)a.sx / 2u;
    float d[2][Q];
    for_dirs<0, Q>([&](auto I) {
        constexpr int i = decltype(I)::value;
        const uint32_t w = __builtin_nontemporal_load(R + (uint64_t)i * pitch);
        d[0][i] = S::from_bits(w);
        d[1][i] = S::from_bits(w >> 16);
    });
#pragma unroll
    for (int c = 0; c < 2; ++c) {
        float drho;
        const Macro M = moments<Q>(a, d[c], drho);
        float wp, wm;
        closure_rates<Q, CL>(a, nullptr, d[c], drho, M, true, wp, wm);
        if constexpr (COLL == COLL_MRT)
            mrt_collide<Q>(a, d[c], drho, M, wp);
        else
            trt_collide<Q>(a, d[c], drho, M, wp, wm);
        if (a.any_vp) {
#pragma unroll
            for (int i = 1; i < Q; ++i) {
                const int dx = cdir(i, 0), dy = cdir(i, 1), dz = cdir(i, 2);
                if (face_cut(g[c], dx, dy, dz))
                    d[c][i] = wall_value<Q>(a, deciding_face(a, g[c], dx, dy, dz), i, d[c][i], M);
            }
        }
    }
    // direction i goes into slot opposite(i) of the same cell
    for_dirs<0, Q>([&](auto I) {
        constexpr int i = decltype(I)::value;
        const uint32_t w = S::to_bits(d[0][i]) | (S::to_bits(d[1][i]) << 16);
        __builtin_nontemporal_store(w, R + (uint64_t)opp(i) * pitch);
    });
}

// ---------------------------------------------------------------------------
// set-up and state kernels
// ---------------------------------------------------------------------------
template <int Q>
__global__ void __launch_bounds__(LBM_LB_THREADS) k_build_mask(LatticeArgs a, const uint8_t *flags, uint32_t *mask)
{
    const int x = blockIdx.x * blockDim.x + threadIdx.x;
    const int y = blockIdx.y * blockDim.y + threadIdx.y;
    const int z = blockIdx.z;
    if (x >= a.nx || y >= a.ny) return;
    const Geom g = make_geom(a, x, y, z);
    uint32_t m = flags[cidx(a, g)] ? SELF_SOLID : 0u;
#pragma unroll
    for (int i = 1; i < Q; ++i) {
        const int dx = cdir(i, 0), dy = cdir(i, 1), dz = cdir(i, 2);
        if (!face_cut(g, dx, dy, dz) && flags[nbr(a, g, dx, dy, dz)]) m |= 1u << i;
    }
    mask[cidx(a, g)] = m;
}

// the run words after the mask (one thread per row and run of 64 cells)
__global__ void __launch_bounds__(256) k_build_mask_runs(LatticeArgs a, uint32_t *mask)
{
    const uint64_t t = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const uint32_t nr = mask_runs(a.nx);
    if (t >= (uint64_t)a.nrows * nr) return;
    const uint64_t row = t / nr;
    const int x0 = (int)(t - row * nr) * 64, x1 = min(x0 + 64, a.nx);
    uint32_t any = 0;
    for (int x = x0; x < x1; ++x) any |= mask[row * (uint32_t)a.nx + (uint32_t)x];
    mask[cells(a) + t] = any != 0u;
}

template <int Q, int ST>
__global__ void __launch_bounds__(LBM_LB_THREADS) k_init_eq(LatticeArgs a, SparseArgs sp, const double *rho, const double *u)
{
    using S = Store<ST>;
    const int x = blockIdx.x * blockDim.x + threadIdx.x;
    const int y = blockIdx.y * blockDim.y + threadIdx.y;
    const int z = blockIdx.z;
    if (x >= a.nx || y >= a.ny) return;
    const Geom g = make_geom(a, x, y, z);
    const bool solid = a.mask && (a.mask[cidx(a, g)] & SELF_SOLID);
    if (sp.on && sp.fmap[cidx(a, g)] < 0) return;  // sparse addressing stores fluid cells only
    const double r = rho[cidx(a, g)], ux = u[cidx(a, g)], uy = u[cells(a) + cidx(a, g)], uz = u[2 * cells(a) + cidx(a, g)];
    const double usq = ux * ux + uy * uy + uz * uz;
    typename S::T *A = (typename S::T *)a.pdf;
#pragma unroll
    for (int i = 0; i < Q; ++i) {
        const double cu = cdir(i, 0) * ux + cdir(i, 1) * uy + cdir(i, 2) * uz;
        const double dev = wgt<Q>(i) * ((r - 1.0) + r * (3.0 * cu + 4.5 * cu * cu - 1.5 * usq));
        A[index_t0<Q>(a, sp, g, i)] = S::cvt(solid ? 0.f : (float)dev);
    }
}

template <int Q, int ST>
__global__ void __launch_bounds__(LBM_LB_THREADS) k_set_pdfs(LatticeArgs a, SparseArgs sp, const double *f)
{
    using S = Store<ST>;
    const int x = blockIdx.x * blockDim.x + threadIdx.x;
    const int y = blockIdx.y * blockDim.y + threadIdx.y;
    const int z = blockIdx.z;
    if (x >= a.nx || y >= a.ny) return;
    const Geom g = make_geom(a, x, y, z);
    if (sp.on && sp.fmap[cidx(a, g)] < 0) return;  // sparse addressing stores fluid cells only
    typename S::T *A = (typename S::T *)a.pdf;
#pragma unroll
    for (int i = 0; i < Q; ++i) {
        A[index_t0<Q>(a, sp, g, i)] = S::cvt((float)(f[(uint64_t)i * cells(a) + cidx(a, g)] - wgt<Q>(i)));
    }
}

template <int Q, int ST>
__global__ void __launch_bounds__(LBM_LB_THREADS) k_get_pdfs(LatticeArgs a, SparseArgs sp, int odd, double *f)
{
    const int x = blockIdx.x * blockDim.x + threadIdx.x;
    const int y = blockIdx.y * blockDim.y + threadIdx.y;
    const int z = blockIdx.z;
    if (x >= a.nx || y >= a.ny) return;
    const Geom g = make_geom(a, x, y, z);
    const uint32_t m = a.mask ? a.mask[cidx(a, g)] : 0u;
    float d[Q];
    if (m & SELF_SOLID) {
#pragma unroll
        for (int i = 0; i < Q; ++i) d[i] = 0.f;
    } else {
        load_state<Q, ST>(a, sp, g, m, odd, d);
    }
#pragma unroll
    for (int i = 0; i < Q; ++i) f[(uint64_t)i * cells(a) + cidx(a, g)] = wgt<Q>(i) + (double)d[i];
}

template <int Q, int ST>
__global__ void __launch_bounds__(256) k_gather(LatticeArgs a, SparseArgs sp, int odd, const int64_t *cells, int64_t ncell,
                                                double *out)
{
    const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= ncell) return;
    const int64_t c = cells[r];
    if (c < 0 || c >= (int64_t)lbm::cells(a)) {
#pragma unroll
        for (int i = 0; i < Q; ++i) out[r * Q + i] = __builtin_nan("");
        return;
    }
    const int x = (int)(c % a.nx), y = (int)((c / a.nx) % a.ny), z = (int)(c / ((int64_t)a.nx * a.ny));
    const Geom g = make_geom(a, x, y, z);
    const uint32_t m = a.mask ? a.mask[cidx(a, g)] : 0u;
    float d[Q];
    if (m & SELF_SOLID) {
#pragma unroll
        for (int i = 0; i < Q; ++i) d[i] = 0.f;
    } else {
        load_state<Q, ST>(a, sp, g, m, odd, d);
    }
#pragma unroll
    for (int i = 0; i < Q; ++i) out[r * Q + i] = wgt<Q>(i) + (double)d[i];
}

template <int Q, int ST>
__global__ void __launch_bounds__(LBM_LB_THREADS) k_moments(LatticeArgs a, SparseArgs sp, int odd, float *rho, float *u)
{
    const int x = blockIdx.x * blockDim.x + threadIdx.x;
    const int y = blockIdx.y * blockDim.y + threadIdx.y;
    const int z = blockIdx.z;
    if (x >= a.nx || y >= a.ny) return;
    const Geom g = make_geom(a, x, y, z);
    const uint32_t m = a.mask ? a.mask[cidx(a, g)] : 0u;
    if (m & SELF_SOLID) {
        rho[cidx(a, g)] = 1.f;
        u[cidx(a, g)] = u[cells(a) + cidx(a, g)] = u[2 * cells(a) + cidx(a, g)] = 0.f;
        return;
    }
    float d[Q];
    load_state<Q, ST>(a, sp, g, m, odd, d);
    float drho;
    const Macro M = moments<Q>(a, d, drho);
    rho[cidx(a, g)] = M.rho;
    u[cidx(a, g)] = M.ux;
    u[cells(a) + cidx(a, g)] = M.uy;
    u[2 * cells(a) + cidx(a, g)] = M.uz;
}

// Deterministic FP64 totals: each block owns a fixed slice of cells and
// reduces it in a fixed order (lanes, then wavefronts); a second kernel sums
// the block partials in index order.
constexpr int TOT_BLOCKS = 1024;

__device__ inline double wave_sum(double v)
{
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

template <int Q, int ST>
__global__ void __launch_bounds__(256) k_totals(LatticeArgs a, SparseArgs sp, int odd, double *partial)
{
    double acc[5] = {0, 0, 0, 0, 0};
    const uint64_t n = cells(a);
    const uint64_t per_block = (n + TOT_BLOCKS - 1) / TOT_BLOCKS;
    const uint64_t lo = (uint64_t)blockIdx.x * per_block;
    const uint64_t hi = lo + per_block < n ? lo + per_block : n;
    const uint64_t plane = (uint64_t)a.nx * (uint64_t)a.ny;
    for (uint64_t c = lo + threadIdx.x; c < hi; c += blockDim.x) {
        const int z = (int)(c / plane);
        const uint64_t r = c - (uint64_t)z * plane;
        const int y = (int)(r / (uint64_t)a.nx);
        const int x = (int)(r - (uint64_t)y * (uint64_t)a.nx);
        const Geom g = make_geom(a, x, y, z);
        const uint32_t m = a.mask ? a.mask[cidx(a, g)] : 0u;
        if (m & SELF_SOLID) continue;
        float d[Q];
        load_state<Q, ST>(a, sp, g, m, odd, d);
        float s = 0.f, jx = 0.f, jy = 0.f, jz = 0.f;
#pragma unroll
        for (int i = 0; i < Q; ++i) {
            s += d[i];
            jx += cdir(i, 0) * d[i];
            jy += cdir(i, 1) * d[i];
            jz += cdir(i, 2) * d[i];
        }
        acc[0] += (double)s;
        acc[1] += (double)jx;
        acc[2] += (double)jy;
        acc[3] += (double)jz;
        acc[4] += isfinite(s) ? 0.0 : 1.0;
    }
    __shared__ double red[4][5];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
    for (int k = 0; k < 5; ++k) {
        const double v = wave_sum(acc[k]);
        if (lane == 0) red[wave][k] = v;
    }
    __syncthreads();
    if (threadIdx.x < 5) {
        double v = 0.0;
        for (int w = 0; w < (int)(blockDim.x >> 6); ++w) v += red[w][threadIdx.x];
        partial[blockIdx.x * 5 + threadIdx.x] = v;
    }
}

__global__ void __launch_bounds__(64) k_totals_final(const double *partial, double *out)
{
    const int k = threadIdx.x;
    if (k >= 5) return;
    double v = 0.0;
    for (int b = 0; b < TOT_BLOCKS; ++b) v += partial[b * 5 + k];
    out[k] = v;
}

// Copy: one 16-byte vector per thread, loaded and stored with the
// nontemporal hint (each line is touched once).  Of the shapes measured on
// MI355X (1 or 4 vectors per thread, with and without the hint) this one
// moves the most bytes per second.
typedef float f32x4 __attribute__((ext_vector_type(4)));

__global__ void __launch_bounds__(256) k_copy(const f32x4 *__restrict__ src, f32x4 *__restrict__ dst, size_t n)
{
    const size_t i = (size_t)blockIdx.x * 256 + threadIdx.x;
    if (i < n) __builtin_nontemporal_store(__builtin_nontemporal_load(src + i), dst + i);
}

// ---------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------
Launch lattice_launch(const LatticeArgs &a)
{
    // LBM_BLOCK threads: BX cells along x (a row segment) times BY rows,
    // BX the largest power of two up to LBM_BLOCK that divides nx.  When a
    // row fits one workgroup, the +-1 shifted accesses of the odd step stay
    // in it; wider rows share a line at each seam between workgroups.
    int bx = LBM_BLOCK;
    if (LBM_ROW_MAX > 0 && a.nx <= LBM_ROW_MAX && a.nx % 64 == 0) {
        Launch L;
        L.block = dim3(a.nx, 1, 1);
        L.grid = dim3(1, a.ny, a.nz);
        return L;
    }
    if (LBM_WIDE > 0 && a.nx % LBM_WIDE == 0) {
        Launch L;
        L.block = dim3(LBM_WIDE, 1, 1);
        L.grid = dim3(a.nx / LBM_WIDE, a.ny, a.nz);
        return L;
    }
    while (bx > 32 && a.nx % bx != 0) bx >>= 1;
    if (a.nx % bx != 0) bx = 64;  // ragged rows: masked tail
    if (bx > a.nx) bx = a.nx <= 32 ? 32 : 64;
    const int by = LBM_BLOCK / bx;
    Launch L;
    L.block = dim3(bx, by, 1);
    L.grid = dim3((a.nx + bx - 1) / bx, (a.ny + by - 1) / by, a.nz);
    return L;
}

hipError_t launch_build_mask(const LatticeArgs &a, int q, const uint8_t *flags, uint32_t *mask, hipStream_t s)
{
    const Launch L = lattice_launch(a);
    if (q == 19)
        k_build_mask<19><<<L.grid, L.block, 0, s>>>(a, flags, mask);
    else
        k_build_mask<27><<<L.grid, L.block, 0, s>>>(a, flags, mask);
    const uint64_t nruns = (uint64_t)a.nrows * mask_runs(a.nx);
    k_build_mask_runs<<<(unsigned)((nruns + 255) / 256), 256, 0, s>>>(a, mask);
    return hipGetLastError();
}

template <int Q, int ST, int CL, bool MASK, int COLL>
static void launch_sc(const LatticeArgs &a, const HrrArgs &h, int odd, const Launch &L, hipStream_t s)
{
    k_stream_collide<Q, ST, CL, MASK, COLL><<<L.grid, L.block, 0, s>>>(a, odd, h);
}

template <int Q, int ST, int COLL>
static void step_coll(const LatticeArgs &a, const HrrArgs &h, int cl, bool mk, int odd, const Launch &L,
                      hipStream_t s)
{
    if (cl == CL_NONE) {
        if (mk)
            launch_sc<Q, ST, CL_NONE, true, COLL>(a, h, odd, L, s);
        else
            launch_sc<Q, ST, CL_NONE, false, COLL>(a, h, odd, L, s);
    } else {
        if (mk)
            launch_sc<Q, ST, CL_SMAG, true, COLL>(a, h, odd, L, s);
        else
            launch_sc<Q, ST, CL_SMAG, false, COLL>(a, h, odd, L, s);
    }
}

// Launch of the paired even step: nx / 2 threads per row, rows of whole
// wavefronts (nx a multiple of 128).
template <int Q, int ST>
static bool even_pair16(const LatticeArgs &a, int cl, int coll, hipStream_t s)
{
    if constexpr (ST == ST_F32 || !LBM_PAIR16) {
        return false;
    } else {
        // TRT only: with MRT the two collisions per thread cost more than
        // the wider accesses gain (measured +5% even-step time on 512x256x256)
        if (a.mask || a.et || cl == CL_MLP || coll != COLL_TRT || a.nx % 128 != 0) return false;
        int bx = 256;
        while ((a.nx / 2) % bx != 0) bx >>= 1;  // nx / 2 is a multiple of 64
        const int by = 256 / bx;
        const dim3 grid(a.nx / 2 / bx, (a.ny + by - 1) / by, a.nz), block(bx, by, 1);
        if (cl == CL_NONE)
            k_even_pair16<Q, ST, CL_NONE, COLL_TRT><<<grid, block, 0, s>>>(a);
        else
            k_even_pair16<Q, ST, CL_SMAG, COLL_TRT><<<grid, block, 0, s>>>(a);
        return true;
    }
}

template <int Q, int ST>
static hipError_t step_q_st(const LatticeArgs &a, const HrrArgs &h, int cl, int coll, int odd, hipStream_t s)
{
    if (!(odd & 1) && even_pair16<Q, ST>(a, cl, coll, s)) return hipGetLastError();
    const Launch L = lattice_launch(a);
    const bool mk = a.mask != nullptr;
    if (cl == CL_MLP) {  // the learned closure runs with the TRT collision
        if (coll != COLL_TRT) return hipErrorInvalidValue;
        if (mk)
            launch_sc<Q, ST, CL_MLP, true, COLL_TRT>(a, h, odd, L, s);
        else
            launch_sc<Q, ST, CL_MLP, false, COLL_TRT>(a, h, odd, L, s);
    } else if (coll == COLL_HRR) {  // D3Q19, no closure
        if constexpr (Q == 19) {
            if (cl != CL_NONE) return hipErrorInvalidValue;
            if (mk)
                launch_sc<Q, ST, CL_NONE, true, COLL_HRR>(a, h, odd, L, s);
            else
                launch_sc<Q, ST, CL_NONE, false, COLL_HRR>(a, h, odd, L, s);
        } else {
            return hipErrorInvalidValue;
        }
    } else if (coll == COLL_MRT) {
        step_coll<Q, ST, COLL_MRT>(a, h, cl, mk, odd, L, s);
    } else {
        step_coll<Q, ST, COLL_TRT>(a, h, cl, mk, odd, L, s);
    }
    return hipGetLastError();
}

hipError_t launch_step(const LatticeArgs &a, const HrrArgs &h, int q, int st, int cl, int coll, int odd, hipStream_t s)
{
    return dispatch(q, st, [&](auto Q, auto ST) { return step_q_st<Q.value, ST.value>(a, h, cl, coll, odd, s); });
}

hipError_t launch_init_eq(const LatticeArgs &a, const SparseArgs &sp, int q, int st, const double *rho,
                          const double *u, hipStream_t s)
{
    const Launch L = lattice_launch(a);
    return dispatch(q, st, [&](auto Q, auto ST) {
        k_init_eq<Q.value, ST.value><<<L.grid, L.block, 0, s>>>(a, sp, rho, u);
        return hipGetLastError();
    });
}

hipError_t launch_set_pdfs(const LatticeArgs &a, const SparseArgs &sp, int q, int st, const double *f, hipStream_t s)
{
    const Launch L = lattice_launch(a);
    return dispatch(q, st, [&](auto Q, auto ST) {
        k_set_pdfs<Q.value, ST.value><<<L.grid, L.block, 0, s>>>(a, sp, f);
        return hipGetLastError();
    });
}

hipError_t launch_get_pdfs(const LatticeArgs &a, const SparseArgs &sp, int q, int st, int odd, double *f,
                           hipStream_t s)
{
    const Launch L = lattice_launch(a);
    return dispatch(q, st, [&](auto Q, auto ST) {
        k_get_pdfs<Q.value, ST.value><<<L.grid, L.block, 0, s>>>(a, sp, odd, f);
        return hipGetLastError();
    });
}

hipError_t launch_gather(const LatticeArgs &a, const SparseArgs &sp, int q, int st, int odd, const int64_t *cells,
                         int64_t ncell, double *out, hipStream_t s)
{
    if (ncell <= 0) return hipSuccess;
    const dim3 grid((unsigned)((ncell + 255) / 256)), block(256);
    return dispatch(q, st, [&](auto Q, auto ST) {
        k_gather<Q.value, ST.value><<<grid, block, 0, s>>>(a, sp, odd, cells, ncell, out);
        return hipGetLastError();
    });
}

hipError_t launch_moments(const LatticeArgs &a, const SparseArgs &sp, int q, int st, int odd, float *rho, float *u,
                          hipStream_t s)
{
    const Launch L = lattice_launch(a);
    return dispatch(q, st, [&](auto Q, auto ST) {
        k_moments<Q.value, ST.value><<<L.grid, L.block, 0, s>>>(a, sp, odd, rho, u);
        return hipGetLastError();
    });
}

int totals_blocks() { return TOT_BLOCKS; }

hipError_t launch_totals(const LatticeArgs &a, const SparseArgs &sp, int q, int st, int odd, double *partial,
                         double *final_out, hipStream_t s)
{
    hipError_t e = dispatch(q, st, [&](auto Q, auto ST) {
        k_totals<Q.value, ST.value><<<TOT_BLOCKS, 256, 0, s>>>(a, sp, odd, partial);
        return hipGetLastError();
    });
    if (e != hipSuccess) return e;
    k_totals_final<<<1, 64, 0, s>>>(partial, final_out);
    return hipGetLastError();
}

__global__ void __launch_bounds__(64) k_build_mlp_table(const float *P, uint32_t *T)
{
    build_table_lane(P, threadIdx.x, T);
}

hipError_t launch_build_mlp_table(const float *params, uint32_t *table, hipStream_t s)
{
    k_build_mlp_table<<<1, 64, 0, s>>>(params, table);
    return hipGetLastError();
}

hipError_t launch_copy(const void *src, void *dst, size_t bytes, hipStream_t s)
{
    const size_t n = bytes / 16;
    const size_t blocks = (n + 255) / 256;
    if (n == 0) return hipSuccess;
    if (blocks > 0x7fffffffu) return hipErrorInvalidValue;
    k_copy<<<(unsigned)blocks, 256, 0, s>>>((const f32x4 *)src, (f32x4 *)dst, n);
    return hipGetLastError();
}

}  // namespace lbm
