// lattice.h -- device-side core shared by the stream-collide kernels of every
// scheme (lbm_kernels.hip: AA pattern and the state kernels; lbm_et.hip:
// Esoteric Twist; lbm_sparse.hip: AA pattern over the fluid cells only):
// storage formats, cell geometry, population addressing, canonical reads,
// collision operators and wall values.
#pragma once

#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

#include <algorithm>
#include <type_traits>

#include "internal.h"
#include "mlp_wave.h"
#include "stencil.h"

// Tuning knobs: the minimum number of waves per SIMD the register
// allocation must allow for the stream-collide kernel, the workgroup size,
// and the streaming (nontemporal) hints of the plain path (1: measured
// policy, 0: none, 2: everywhere).
#ifndef LBM_MIN_WAVES
#define LBM_MIN_WAVES 1
#endif
#ifndef LBM_BLOCK
#define LBM_BLOCK 256
#endif
// Row segments of LBM_WIDE cells per workgroup when nx is a multiple of it
// (0: never): a 512-cell row then fits one workgroup and the odd step's
// shifted lines at the seam are fetched once (+2% on 512x256x256).
#ifndef LBM_WIDE
#define LBM_WIDE 512
#endif
// whole rows of up to LBM_ROW_MAX cells per workgroup (0: fixed LBM_BLOCK)
#ifndef LBM_ROW_MAX
#define LBM_ROW_MAX 0
#endif
#define LBM_MAX2(a, b) ((a) > (b) ? (a) : (b))
#define LBM_LB_THREADS LBM_MAX2(LBM_MAX2(LBM_ROW_MAX, LBM_WIDE), LBM_BLOCK)
#ifndef LBM_NT_POLICY
#define LBM_NT_POLICY 1
#endif
// Code paths of the stream-collide kernel.  Unified: one path for every
// cell, cut links handled by address selects (no divergence between cells
// next to faces or solids and open cells).  Split: a plain path for cells
// away from non-periodic faces and a separate boundary path.  Measured on
// MI355X: unified is faster for FP32 storage (+3% on 512x256x256) and for
// masked domains (+6% on the 384^3 D3Q27 obstacles); split is faster for
// 16-bit storage (+14%) and with the MLP closure (+5%).
// LBM_UNIFIED: 0 split, 1 unified, 2 the measured choice per instantiation.
#ifndef LBM_UNIFIED
#define LBM_UNIFIED 2
#endif

namespace lbm {

// Streaming hints.  A population line that only this wavefront touches is
// loaded and stored with the nontemporal hint (no reuse; it should not
// displace other lines).  Lines read with a +-1 shift along x are shared
// with the neighbouring wavefront in the same workgroup, so those keep the
// normal policy and meet in the CU's L1 (or in L2).
template <bool NT, class T>
__device__ inline T ld_pop(const T *p)
{
    if constexpr (NT) return __builtin_nontemporal_load(p);
    return *p;
}

template <bool NT, class T>
__device__ inline void st_pop(T *p, T v)
{
    if constexpr (NT)
        __builtin_nontemporal_store(v, p);
    else
        *p = v;
}

// Hint for a population access along direction i on the even (local) or
// odd (shifted) step of the AA pattern.  With a solid mask the odd step
// keeps every line cached: links cut by solids send lanes to their own
// cell's slots, whose lines other directions of the same rows touch again
// (measured: 4.5% faster odd steps on the 384^3 D3Q27 obstacle flow; the
// Esoteric Twist kernel measured slower that way and keeps its hints).
template <int I, bool MASK = false>
struct Hint {
    static constexpr bool even = LBM_NT_POLICY != 0;
    static constexpr bool odd = LBM_NT_POLICY == 2 || (LBM_NT_POLICY == 1 && !MASK && cdir(I, 0) == 0);
};

// ---------------------------------------------------------------------------
// storage formats
// ---------------------------------------------------------------------------
template <int ST>
struct Store;

template <>
struct Store<ST_F32> {
    using T = float;
    template <bool NT = false>
    __device__ static float ld(const T *p) { return ld_pop<NT>(p); }
    template <bool NT = false>
    __device__ static void st(T *p, float v) { st_pop<NT>(p, v); }
    __device__ static T cvt(float v) { return v; }
};

template <>
struct Store<ST_F16> {
    using T = _Float16;
    template <bool NT = false>
    __device__ static float ld(const T *p) { return (float)ld_pop<NT>(p); }
    template <bool NT = false>
    __device__ static void st(T *p, float v) { st_pop<NT>(p, (_Float16)v); }
    __device__ static T cvt(float v) { return (_Float16)v; }
    // raw 16-bit patterns (two cells packed in one 32-bit access)
    __device__ static float from_bits(uint32_t b) { return (float)__builtin_bit_cast(_Float16, (uint16_t)b); }
    __device__ static uint32_t to_bits(float v) { return __builtin_bit_cast(uint16_t, (_Float16)v); }
};

// bfloat16 as raw bits: widen by a shift, narrow with the hardware
// round-to-nearest-even conversion
__device__ inline uint16_t f32_to_bf16_rne(float v) { return __builtin_bit_cast(uint16_t, (__bf16)v); }

template <>
struct Store<ST_BF16> {
    using T = uint16_t;
    template <bool NT = false>
    __device__ static float ld(const T *p) { return __uint_as_float((uint32_t)ld_pop<NT>(p) << 16); }
    template <bool NT = false>
    __device__ static void st(T *p, float v) { st_pop<NT>(p, f32_to_bf16_rne(v)); }
    __device__ static T cvt(float v) { return f32_to_bf16_rne(v); }
    __device__ static float from_bits(uint32_t b) { return __uint_as_float((b & 0xffffu) << 16); }
    __device__ static uint32_t to_bits(float v) { return f32_to_bf16_rne(v); }
};

// ---------------------------------------------------------------------------
// cell geometry
// ---------------------------------------------------------------------------
struct Geom {
    int x, y, z;
    uint32_t frow; // row z ny + y of the cell fields and the mask (cell index frow nx + x: cidx)
    uint32_t row;  // row index z sy + y of the population store
    int xm, xp, ym, yp, zm, zp;    // wrapped neighbour coordinates
    int xq, yq, zq;                // x + 1 etc. in the store: wrapped on periodic axes, else the ghost layer
    bool cxl, cxh, cyl, cyh, czl, czh;  // link through that face is cut by a non-periodic face
};

__device__ inline Geom make_geom(const LatticeArgs &a, int x, int y, int z)
{
    Geom g;
    g.x = x;
    g.y = y;
    g.z = z;
    g.row = (uint32_t)z * (uint32_t)a.sy + (uint32_t)y;
    g.frow = (uint32_t)z * (uint32_t)a.ny + (uint32_t)y;
    g.xm = x == 0 ? a.nx - 1 : x - 1;
    g.xp = x == a.nx - 1 ? 0 : x + 1;
    g.ym = y == 0 ? a.ny - 1 : y - 1;
    g.yp = y == a.ny - 1 ? 0 : y + 1;
    g.zm = z == 0 ? a.nz - 1 : z - 1;
    g.zp = z == a.nz - 1 ? 0 : z + 1;
    g.xq = a.per[0] ? g.xp : x + 1;
    g.yq = a.per[1] ? g.yp : y + 1;
    g.zq = a.per[2] ? g.zp : z + 1;
    g.cxl = !a.per[0] && x == 0;
    g.cxh = !a.per[0] && x == a.nx - 1;
    g.cyl = !a.per[1] && y == 0;
    g.cyh = !a.per[1] && y == a.ny - 1;
    g.czl = !a.per[2] && z == 0;
    g.czh = !a.per[2] && z == a.nz - 1;
    return g;
}

// 64-bit cell index (z ny + y) nx + x of the fields and the mask, formed
// only where a kernel uses it
__device__ inline uint64_t cidx(const LatticeArgs &a, const Geom &g)
{
    return (uint64_t)g.frow * (uint32_t)a.nx + (uint32_t)g.x;
}

// index of the neighbour at offset (dx, dy, dz), periodic wrap
__device__ inline uint64_t nbr(const LatticeArgs &a, const Geom &g, int dx, int dy, int dz)
{
    const int xx = dx < 0 ? g.xm : (dx > 0 ? g.xp : g.x);
    const int yy = dy < 0 ? g.ym : (dy > 0 ? g.yp : g.y);
    const int zz = dz < 0 ? g.zm : (dz > 0 ? g.zp : g.z);
    return (uint64_t)((uint32_t)zz * (uint32_t)a.ny + (uint32_t)yy) * (uint32_t)a.nx + (uint32_t)xx;
}

// Population store: rows of q direction segments, [z][y][i][x].  Each
// segment holds the sx populations of one direction of one row, so a
// wavefront's accesses for one direction are contiguous, and the q segments
// of a row sit together (one block of q sx elements per row).
template <int Q>
__device__ inline uint64_t pidx(const LatticeArgs &a, int i, uint32_t row, int x)
{
    return ((uint64_t)row * Q + (uint64_t)i) * (uint32_t)a.sx + (uint32_t)x;
}

// row and x of the neighbour at offset (dx, dy, dz), periodic wrap
__device__ inline uint32_t nbr_row(const LatticeArgs &a, const Geom &g, int dy, int dz)
{
    const int yy = dy < 0 ? g.ym : (dy > 0 ? g.yp : g.y);
    const int zz = dz < 0 ? g.zm : (dz > 0 ? g.zp : g.z);
    return (uint32_t)zz * (uint32_t)a.sy + (uint32_t)yy;
}

// Esoteric Twist location x + p of the store, p in {0, 1}^3 (the positive
// neighbourhood of the cell), slot i
template <int Q>
__device__ inline uint64_t et_index(const LatticeArgs &a, const Geom &g, int i, int px, int py, int pz)
{
    const uint32_t row = (uint32_t)(pz ? g.zq : g.z) * (uint32_t)a.sy + (uint32_t)(py ? g.yq : g.y);
    return pidx<Q>(a, i, row, px ? g.xq : g.x);
}

__device__ inline int nbr_x(const Geom &g, int dx) { return dx < 0 ? g.xm : (dx > 0 ? g.xp : g.x); }

template <int Q>
__device__ inline uint64_t pidx_nbr(const LatticeArgs &a, const Geom &g, int i, int dx, int dy, int dz)
{
    return pidx<Q>(a, i, nbr_row(a, g, dy, dz), nbr_x(g, dx));
}

// does the link from this cell along (dx, dy, dz) leave through a non-periodic face?
__device__ inline bool face_cut(const Geom &g, int dx, int dy, int dz)
{
    return (dx < 0 && g.cxl) || (dx > 0 && g.cxh) || (dy < 0 && g.cyl) || (dy > 0 && g.cyh) ||
           (dz < 0 && g.czl) || (dz > 0 && g.czh);
}

// Face that decides a cut link along (dx, dy, dz): among the crossed
// non-periodic faces the first of no-slip, velocity, pressure (lowest face
// index among equals).  Returns -1 when no face is crossed.
__device__ inline int deciding_face(const LatticeArgs &a, const Geom &g, int dx, int dy, int dz)
{
    int best = -1, rank = 0;
    const bool cross[6] = {dx < 0 && g.cxl, dx > 0 && g.cxh, dy < 0 && g.cyl,
                           dy > 0 && g.cyh, dz < 0 && g.czl, dz > 0 && g.czh};
#pragma unroll
    for (int f = 0; f < 6; ++f) {
        if (!cross[f]) continue;
        const int k = a.bc[f];
        const int r = k == BC_NOSLIP ? 3 : (k == BC_VELOCITY ? 2 : (k == BC_PRESSURE ? 1 : 0));
        if (r > rank) {
            rank = r;
            best = f;
        }
    }
    return best;
}

// sparse addressing: population i of fluid cell k, and neighbour-table entry
// j of fluid cell k
template <int Q>
__device__ inline uint64_t sp_index(uint32_t k, int i)
{
    return ((uint64_t)(k / SP_CHUNK) * Q + (uint32_t)i) * SP_CHUNK + k % SP_CHUNK;
}

template <int Q>
__device__ inline uint64_t sp_table(uint32_t k, int j)
{
    return ((uint64_t)(k / SP_CHUNK) * (Q - 1) + (uint32_t)(j - 1)) * SP_CHUNK + k % SP_CHUNK;
}

// ---------------------------------------------------------------------------
// canonical read (shared by the step kernel and every state reader)
// ---------------------------------------------------------------------------
template <int Q, int ST>
__device__ inline void load_canonical(const LatticeArgs &a, const Geom &g, uint32_t m, int odd, float (&d)[Q])
{
    using S = Store<ST>;
    const typename S::T *A = (const typename S::T *)a.pdf;
    if (a.et) {
        // Esoteric Twist: f_i(x) sits at x + max(-c_i, 0) in slot i after an
        // even number of steps, slot opposite(i) after an odd number, cut
        // links included
#pragma unroll
        for (int i = 0; i < Q; ++i)
            d[i] = S::ld(A + et_index<Q>(a, g, odd ? opp(i) : i, cdir(i, 0) < 0, cdir(i, 1) < 0, cdir(i, 2) < 0));
        return;
    }
    if (!odd) {
#pragma unroll
        for (int i = 0; i < Q; ++i) d[i] = S::ld(A + pidx<Q>(a, i, g.row, g.x));
    } else {
#pragma unroll
        for (int i = 0; i < Q; ++i) {
            const int dx = cdir(i, 0), dy = cdir(i, 1), dz = cdir(i, 2);
            // source x - c_i; blocked when that link is cut (mask bit of opposite(i))
            const bool cut = face_cut(g, -dx, -dy, -dz) || ((m >> opp(i)) & 1u);
            const uint64_t own = pidx<Q>(a, i, g.row, g.x);
            const uint64_t src = pidx_nbr<Q>(a, g, opp(i), -dx, -dy, -dz);
            d[i] = S::ld(A + (cut ? own : src));
        }
    }
}

// Compile-time loop over the directions (so each access can take its own
// streaming hint).
template <int I, int Q, class F>
__device__ inline void for_dirs(F &&f)
{
    if constexpr (I < Q) {
        f(std::integral_constant<int, I>{});
        for_dirs<I + 1, Q>(f);
    }
}

// Read of a cell none of whose links crosses a non-periodic face: no face
// logic.  Links cut by a solid neighbour (mask bit of the link) only matter
// on the odd step, where they select the cell's own slot instead of the
// neighbour's -- a per-direction select, not a branch, so wavefronts that
// mix cells next to solids with open cells do not diverge.
template <int Q, int ST, bool MASK>
__device__ inline void load_plain(const LatticeArgs &a, const Geom &g, uint32_t m, int odd, float (&d)[Q])
{
    using S = Store<ST>;
    const typename S::T *A = (const typename S::T *)a.pdf;
    if (!odd) {
        const typename S::T *R = A + pidx<Q>(a, 0, g.row, g.x);
        for_dirs<0, Q>([&](auto I) {
            constexpr int i = decltype(I)::value;
            d[i] = S::template ld<Hint<i, MASK>::even>(R + (uint64_t)i * (uint32_t)a.sx);
        });
    } else {
        for_dirs<0, Q>([&](auto I) {
            constexpr int i = decltype(I)::value;
            uint64_t k = pidx_nbr<Q>(a, g, opp(i), -cdir(i, 0), -cdir(i, 1), -cdir(i, 2));
            if constexpr (MASK) {
                if (i != 0 && ((m >> opp(i)) & 1u)) k = pidx<Q>(a, i, g.row, g.x);
            }
            d[i] = S::template ld<Hint<i, MASK>::odd>(A + k);
        });
    }
}

template <int Q, int ST, bool MASK>
__device__ inline void store_plain(const LatticeArgs &a, const Geom &g, uint32_t m, int odd, const float (&d)[Q])
{
    using S = Store<ST>;
    typename S::T *A = (typename S::T *)a.pdf;
    if (!odd) {
        typename S::T *R = A + pidx<Q>(a, 0, g.row, g.x);
        for_dirs<0, Q>([&](auto I) {
            constexpr int i = decltype(I)::value;
            S::template st<Hint<i, MASK>::even>(R + (uint64_t)opp(i) * (uint32_t)a.sx, d[i]);
        });
    } else {
        for_dirs<0, Q>([&](auto I) {
            constexpr int i = decltype(I)::value;
            uint64_t k = pidx_nbr<Q>(a, g, i, cdir(i, 0), cdir(i, 1), cdir(i, 2));
            if constexpr (MASK) {
                if (i != 0 && ((m >> i) & 1u)) k = pidx<Q>(a, opp(i), g.row, g.x);
            }
            S::template st<Hint<i, MASK>::odd>(A + k, d[i]);
        });
    }
}

// ---------------------------------------------------------------------------
// collision: TRT + Guo on deviations, optional Smagorinsky relaxation time
// ---------------------------------------------------------------------------
struct Macro {
    float rho, ux, uy, uz;
};

template <int Q>
__device__ inline Macro moments(const LatticeArgs &a, const float (&d)[Q], float &drho)
{
    float s = 0.f, jx = 0.f, jy = 0.f, jz = 0.f;
#pragma unroll
    for (int i = 0; i < Q; ++i) {
        s += d[i];
        if (cdir(i, 0)) jx += cdir(i, 0) > 0 ? d[i] : -d[i];
        if (cdir(i, 1)) jy += cdir(i, 1) > 0 ? d[i] : -d[i];
        if (cdir(i, 2)) jz += cdir(i, 2) > 0 ? d[i] : -d[i];
    }
    drho = s;
    Macro M;
    M.rho = 1.f + s;
    const float ir = 1.f / M.rho;
    M.ux = (jx + 0.5f * a.F[0]) * ir;
    M.uy = (jy + 0.5f * a.F[1]) * ir;
    M.uz = (jz + 0.5f * a.F[2]) * ir;
    return M;
}

// Non-equilibrium momentum flux with the forcing correction,
// P_c = sum_i c_i c_i (f_i - f_i^eq) + (u F + F u)/2, packed xx,yy,zz,xy,xz,yz.
// With deviations, sum_i c c f^eq - sum_i c c w = drho/3 I + rho u u.
template <int Q>
__device__ inline void noneq_flux(const LatticeArgs &a, const float (&d)[Q], float drho, const Macro &M,
                                  float (&P)[6])
{
    float pxx = 0.f, pyy = 0.f, pzz = 0.f, pxy = 0.f, pxz = 0.f, pyz = 0.f;
#pragma unroll
    for (int i = 1; i < Q; ++i) {
        const int cx = cdir(i, 0), cy = cdir(i, 1), cz = cdir(i, 2);
        if (cx) pxx += d[i];
        if (cy) pyy += d[i];
        if (cz) pzz += d[i];
        if (cx * cy) pxy += cx * cy > 0 ? d[i] : -d[i];
        if (cx * cz) pxz += cx * cz > 0 ? d[i] : -d[i];
        if (cy * cz) pyz += cy * cz > 0 ? d[i] : -d[i];
    }
    const float third = drho * (1.f / 3.f);
    const float F0 = a.F[0], F1 = a.F[1], F2 = a.F[2];
    P[0] = pxx - third - M.rho * M.ux * M.ux + M.ux * F0;
    P[1] = pyy - third - M.rho * M.uy * M.uy + M.uy * F1;
    P[2] = pzz - third - M.rho * M.uz * M.uz + M.uz * F2;
    P[3] = pxy - M.rho * M.ux * M.uy + 0.5f * (M.ux * F1 + F0 * M.uy);
    P[4] = pxz - M.rho * M.ux * M.uz + 0.5f * (M.ux * F2 + F0 * M.uz);
    P[5] = pyz - M.rho * M.uy * M.uz + 0.5f * (M.uy * F2 + F1 * M.uz);
}

// The closures' square roots and quotients use the hardware square root and
// reciprocal (within 1 ulp each): their operands are positive normal numbers,
// and an ulp of a relaxation time is far below what the FP32 populations
// resolve.
__device__ inline float rcp(float v) { return __builtin_amdgcn_rcpf(v); }

__device__ inline float flux_norm(const float (&P)[6])
{
    return __builtin_amdgcn_sqrtf(P[0] * P[0] + P[1] * P[1] + P[2] * P[2] +
                                  2.f * (P[3] * P[3] + P[4] * P[4] + P[5] * P[5]));
}

// Hou et al. (1996) Smagorinsky relaxation time from |P_c|:
// tau_s = (tau + sqrt(tau^2 + a)) / 2 with a = 18 sqrt(2) Cs^2 |P_c| / rho.
// Returned as the excess tau_s - tau = (a/2) / (sqrt(tau^2 + a) + tau), which
// has no cancellation in FP32 when a << tau^2.
__device__ inline float smag_excess(float tau, float cs, float Qn, float rho)
{
    const float a = 18.f * 1.41421356237f * cs * cs * Qn * rcp(rho);
    return 0.5f * a * rcp(__builtin_amdgcn_sqrtf(tau * tau + a) + tau);
}

// TRT rates of a cell whose relaxation time is tt: omega+ = 1/tt and
// omega- from the magic parameter, 1 / (1/2 + Lambda / (tt - 1/2)).
__device__ inline void trt_rates(float tt, float magic, float &wp, float &wm)
{
    wp = rcp(tt);
    wm = rcp(0.5f + magic * rcp(tt - 0.5f));
}

// keep: exchange each pair instead of colliding (solid lanes on the even
// step, which store direction i into slot opposite(i) and so put every
// slot's own value back; see the stream-collide kernel)
template <int Q>
__device__ inline void trt_collide(const LatticeArgs &a, float (&d)[Q], float drho, const Macro &M, float wp,
                                   float wm, bool keep = false)
{
    const float F0 = a.F[0], F1 = a.F[1], F2 = a.F[2];
    const float usq = M.ux * M.ux + M.uy * M.uy + M.uz * M.uz;
    const float uF = M.ux * F0 + M.uy * F1 + M.uz * F2;
    const float kp = 1.f - 0.5f * wp, km = 1.f - 0.5f * wm;
    const float base = drho - 1.5f * M.rho * usq;  // shared part of the symmetric equilibrium
    {
        constexpr float w0 = (float)wgt<Q>(0);
        const float deq = w0 * base;
        const float S = w0 * (-3.f * uF);
        d[0] = keep ? d[0] : d[0] - wp * (d[0] - deq) + kp * S;
    }
#pragma unroll
    for (int i = 1; i < Q; i += 2) {
        const int cx = cdir(i, 0), cy = cdir(i, 1), cz = cdir(i, 2);
        const float w = (float)wgt<Q>(i);
        const float cu = cx * M.ux + cy * M.uy + cz * M.uz;
        const float cF = cx * F0 + cy * F1 + cz * F2;
        const float deqp = w * (base + 4.5f * M.rho * cu * cu);
        const float eqm = 3.f * w * M.rho * cu;
        const float Sp = w * (9.f * cu * cF - 3.f * uF);
        const float Sm = 3.f * w * cF;
        const float dp = 0.5f * (d[i] + d[i + 1]);
        const float dm = 0.5f * (d[i] - d[i + 1]);
        const float A = -wp * (dp - deqp) + kp * Sp;
        const float B = -wm * (dm - eqm) + km * Sm;
        const float di = d[i], dj = d[i + 1];
        d[i] = keep ? dj : di + A + B;
        d[i + 1] = keep ? di : dj + A - B;
    }
}

// Multiple-relaxation-time collision on deviations.  Forward transform
// m = M d; every moment relaxes toward its equilibrium moment with the rate
// of its group (viscous: wnu; ghosts: the domain's five rates) and takes the
// Guo source moment with weight (1 - s/2); density is unchanged and the
// momentum moments change by exactly F.  The equilibrium and source moments
// are closed forms in rho, u, F with lattice constants fixed at compile
// time.  Back with M^-1 = M^T diag(1/|row|^2).
template <int Q>
__device__ inline void mrt_collide(const LatticeArgs &a, float (&d)[Q], float drho, const Macro &M, float wnu,
                                   bool keep = false)
{
    const float F[3] = {a.F[0], a.F[1], a.F[2]};
    const float U[3] = {M.ux, M.uy, M.uz};
    const float usq = U[0] * U[0] + U[1] * U[1] + U[2] * U[2];
    const float uF = U[0] * F[0] + U[1] * F[1] + U[2] * F[2];
    const float base = drho - 1.5f * M.rho * usq;
    const float rate[8] = {0.f, 0.f, wnu, a.mrt[0], a.mrt[1], a.mrt[2], a.mrt[3], a.mrt[4]};
    float m[Q];
    for_dirs<0, Q>([&](auto R) {
        constexpr int r = decltype(R)::value;
        float acc = 0.f;
        for_dirs<0, Q>([&](auto I) {
            constexpr int i = decltype(I)::value;
            constexpr int mv = mrt_value<Q>(r, i);
            if constexpr (mv == 1)
                acc += d[i];
            else if constexpr (mv == -1)
                acc -= d[i];
            else if constexpr (mv != 0)
                acc += (float)mv * d[i];
        });
        m[r] = acc;
    });
    for_dirs<0, Q>([&](auto R) {
        constexpr int r = decltype(R)::value;
        constexpr int grp = mrt_group<Q>(r);
        if constexpr (grp == MG_J) {
            m[r] += keep ? 0.f : F[mrt_j_axis<Q>(r)];
        } else if constexpr (grp != MG_RHO) {
            constexpr float A = (float)mrt_A<Q>(r);
            float meq = A * base, ms = -3.f * A * uF;
            for_dirs<0, 3>([&](auto K) {
                constexpr int k = decltype(K)::value;
                constexpr float B = (float)mrt_B<Q>(r, k);
                if constexpr (B != 0.f) {
                    meq += 3.f * M.rho * B * U[k];
                    ms += 3.f * B * F[k];
                }
                for_dirs<0, 3>([&](auto L) {
                    constexpr int l = decltype(L)::value;
                    constexpr float C = (float)mrt_C<Q>(r, k, l);
                    if constexpr (C != 0.f) {
                        meq += 4.5f * M.rho * C * U[k] * U[l];
                        ms += 9.f * C * U[k] * F[l];
                    }
                });
            });
            const float sr = rate[grp];
            const float dmr = -sr * (m[r] - meq) + (1.f - 0.5f * sr) * ms;
            m[r] += keep ? 0.f : dmr;
        }
    });
    for_dirs<0, Q>([&](auto I) {
        constexpr int i = decltype(I)::value;
        float acc = 0.f;
        for_dirs<0, Q>([&](auto R) {
            constexpr int r = decltype(R)::value;
            constexpr int mv = mrt_value<Q>(r, i);
            if constexpr (mv != 0) acc += ((float)mv / (float)mrt_norm<Q>(r)) * m[r];
        });
        d[i] = acc;
    });
}

// ---------------------------------------------------------------------------
// hybrid recursive regularised collision (HRR, D3Q19; the "D3Q19HRR" of the
// LaBS section, after Jacob, Malaspinas & Sagaut 2018)
// ---------------------------------------------------------------------------
// Velocity gradient G[a][b] = d u_a / d x_b of the previous step's velocity
// field U [3][n] at a fluid cell.  Per axis: central differences between two
// domain neighbours (periodic faces wrap); next to a wall half a cell away
// (a no-slip face, a velocity face with its u_bc, or a solid neighbour at
// rest) the derivative of the quadratic through the wall point and the two
// nearest cells, -4/3 u_w + u_0 + u_1/3 (mirrored on the + side); between two
// walls u_w+ - u_w-; a pressure face's ghost takes the cell's own velocity.
template <int Q>
__device__ inline void fd_gradient(const LatticeArgs &a, const HrrArgs &h, const Geom &g, uint32_t m,
                                   float (&G)[3][3])
{
    const float *U = h.uprev;
    const uint64_t n = cells(a);
    float u0[3];
#pragma unroll
    for (int k = 0; k < 3; ++k) u0[k] = U[k * n + cidx(a, g)];
    for_dirs<0, 3>([&](auto B) {
        constexpr int b = decltype(B)::value;
        constexpr int dm = 2 * b + 2, dp = 2 * b + 1;  // directions -e_b and +e_b
        const bool cutm = b == 0 ? g.cxl : (b == 1 ? g.cyl : g.czl);
        const bool cutp = b == 0 ? g.cxh : (b == 1 ? g.cyh : g.czh);
        const int km = cutm ? (a.bc[2 * b] == BC_PRESSURE ? 2 : 1) : (int)((m >> dm) & 1u);
        const int kp = cutp ? (a.bc[2 * b + 1] == BC_PRESSURE ? 2 : 1) : (int)((m >> dp) & 1u);
        const bool velm = cutm && a.bc[2 * b] == BC_VELOCITY, velp = cutp && a.bc[2 * b + 1] == BC_VELOCITY;
        const uint64_t im = km == 0 ? nbr(a, g, -cdir(dp, 0), -cdir(dp, 1), -cdir(dp, 2)) : cidx(a, g);
        const uint64_t ip = kp == 0 ? nbr(a, g, cdir(dp, 0), cdir(dp, 1), cdir(dp, 2)) : cidx(a, g);
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            const float um = U[k * n + im], up = U[k * n + ip];
            const float wm = velm ? a.ubc[2 * b][k] : 0.f, wp = velp ? a.ubc[2 * b + 1][k] : 0.f;
            float dd = 0.5f * (up - um);
            if (km == 1) dd = -(4.f / 3.f) * wm + u0[k] + up * (1.f / 3.f);
            if (kp == 1) dd = (4.f / 3.f) * wp - u0[k] - um * (1.f / 3.f);
            if (km == 1 && kp == 1) dd = wp - wm;
            G[k][b] = dd;
        }
    });
}

// HRR on deviations d_i = f_i - w_i, D3Q19:
//   f*_i = feq_i + (1 - 1/tau) f1_i + S_i / 2,
//   f1_i = w_i [ 9/2 H2_i : Pi + sum_k T_k(c_i) A_k / N_k ],
// Pi = sigma P_c + (1 - sigma)(-1/3 rho tau (G + G^T)) blends the projected
// non-equilibrium flux with the finite-difference one; A_k combine the
// recursive third-order coefficients a3_abg = u_a Pi_bg + u_b Pi_ag +
// u_g Pi_ab; the equilibrium adds the same third-order terms with
// a3 = rho u u u.  (BGK with Guo forcing is feq + (1 - 1/tau)(f - feq + S/2)
// + S/2; the regularisation replaces the middle term by f1.)  keep: leave
// the populations as they are (solid lanes on the even step).
template <int Q>
__device__ inline void hrr_collide(const LatticeArgs &a, float sigma, const float (&G)[3][3], float (&d)[Q],
                                   float drho, const Macro &M, bool keep)
{
    static_assert(Q == 19, "HRR is built for D3Q19");
    if (keep) return;
    float P[6];
    noneq_flux<Q>(a, d, drho, M, P);
    const float fd = -(1.f / 3.f) * M.rho * a.tau, s1 = 1.f - sigma;
    const float pxx = sigma * P[0] + s1 * fd * 2.f * G[0][0];
    const float pyy = sigma * P[1] + s1 * fd * 2.f * G[1][1];
    const float pzz = sigma * P[2] + s1 * fd * 2.f * G[2][2];
    const float pxy = sigma * P[3] + s1 * fd * (G[0][1] + G[1][0]);
    const float pxz = sigma * P[4] + s1 * fd * (G[0][2] + G[2][0]);
    const float pyz = sigma * P[5] + s1 * fd * (G[1][2] + G[2][1]);
    const float ux = M.ux, uy = M.uy, uz = M.uz;
    // recursive third-order coefficients, combined as the lattice carries them
    const float xxy = 2.f * ux * pxy + uy * pxx, yzz = 2.f * uz * pyz + uy * pzz;
    const float xzz = 2.f * uz * pxz + ux * pzz, xyy = 2.f * uy * pxy + ux * pyy;
    const float yyz = 2.f * uy * pyz + uz * pyy, xxz = 2.f * ux * pxz + uz * pxx;
    const float R = M.rho;
    const float e_xxy = R * ux * ux * uy, e_yzz = R * uy * uz * uz, e_xzz = R * ux * uz * uz;
    const float e_xyy = R * ux * uy * uy, e_yyz = R * uy * uy * uz, e_xxz = R * ux * ux * uz;
    const float k1 = 1.f - a.omp;
    // per combination: (1 - 1/tau) A_k / N_k + A^eq_k / N_k
    // (the norms are compile-time constants: 27/2 for the sums, 27/6 for the differences)
    constexpr float iN0 = (float)(1.0 / t3norm(0)), iN1 = (float)(1.0 / t3norm(1)), iN2 = (float)(1.0 / t3norm(2));
    constexpr float iN3 = (float)(1.0 / t3norm(3)), iN4 = (float)(1.0 / t3norm(4)), iN5 = (float)(1.0 / t3norm(5));
    float Bk[6];
    Bk[0] = (k1 * (xxy + yzz) + (e_xxy + e_yzz)) * iN0;
    Bk[1] = (k1 * (xxy - yzz) + (e_xxy - e_yzz)) * iN1;
    Bk[2] = (k1 * (xzz + xyy) + (e_xzz + e_xyy)) * iN2;
    Bk[3] = (k1 * (xzz - xyy) + (e_xzz - e_xyy)) * iN3;
    Bk[4] = (k1 * (yyz + xxz) + (e_yyz + e_xxz)) * iN4;
    Bk[5] = (k1 * (yyz - xxz) + (e_yyz - e_xxz)) * iN5;
    const float F0 = a.F[0], F1 = a.F[1], F2 = a.F[2];
    const float usq = ux * ux + uy * uy + uz * uz;
    const float uF = ux * F0 + uy * F1 + uz * F2;
    const float base = drho - 1.5f * R * usq;
    const float trp = (pxx + pyy + pzz) * (1.f / 3.f);
    // Pairs (i, opposite(i)): the equilibrium's quadratic part, the
    // second-order term and the forcing's -uF and cu cF parts are even in c
    // (E), the linear parts and the third-order term odd (O), so
    // f*_i = E + O and f*_opp(i) = E - O.
    float even_sum = 0.f;
    for_dirs<1, Q>([&](auto I) {
        constexpr int i = decltype(I)::value;
        if constexpr (i & 1) {
            constexpr int cx = cdir(i, 0), cy = cdir(i, 1), cz = cdir(i, 2);
            constexpr float w = (float)wgt<Q>(i);
            const float cu = cx * ux + cy * uy + cz * uz;
            const float cF = cx * F0 + cy * F1 + cz * F2;
            const float h2 = (float)(cx * cx) * pxx + (float)(cy * cy) * pyy + (float)(cz * cz) * pzz +
                             2.f * ((float)(cx * cy) * pxy + (float)(cx * cz) * pxz + (float)(cy * cz) * pyz) - trp;
            float t3 = 0.f;
            for_dirs<0, 6>([&](auto K) {
                constexpr int k = decltype(K)::value;
                constexpr float tv = (float)t3val(i, k);
                if constexpr (tv != 0.f) t3 += tv * Bk[k];
            });
            const float E = w * (base + 4.5f * R * cu * cu + k1 * 4.5f * h2 + 0.5f * (9.f * cu * cF - 3.f * uF));
            const float O = w * (3.f * R * cu + t3 + 1.5f * cF);
            d[i] = E + O;
            d[opp(i)] = E - O;
            even_sum += E;
        }
    });
    // The update keeps the cell's mass exactly (sum f* = rho); the rest
    // population takes what the moving ones leave (their sum is twice the
    // even parts' sum), so FP32 rounding of the moving ones cannot drift the
    // total mass.
    d[0] = drho - 2.f * even_sum;
}

// Canonical read for the state kernels, any scheme.  With sparse addressing
// (fluid cells only, the AA pattern over the fluid index) f_i sits after an
// odd number of steps in slot opposite(i) of the neighbour x - c_i, or in the
// cell's own slot i when that link is cut; solid cells read as zero
// deviations.
template <int Q, int ST>
__device__ inline void load_state(const LatticeArgs &a, const SparseArgs &sp, const Geom &g, uint32_t m, int odd,
                                  float (&d)[Q])
{
    if (!sp.on) {
        load_canonical<Q, ST>(a, g, m, odd, d);
        return;
    }
    using S = Store<ST>;
    const typename S::T *A = (const typename S::T *)a.pdf;
    const int32_t kf = sp.fmap[cidx(a, g)];
    if (kf < 0) {
#pragma unroll
        for (int i = 0; i < Q; ++i) d[i] = 0.f;
        return;
    }
    const uint32_t k = (uint32_t)kf;
    d[0] = S::ld(A + sp_index<Q>(k, 0));
#pragma unroll
    for (int i = 1; i < Q; ++i) {
        const uint32_t t = odd ? sp.nbt[sp_table<Q>(k, opp(i))] : NB_FACE0;
        d[i] = S::ld(A + (t >= NB_FACE0 ? sp_index<Q>(k, i) : sp_index<Q>(t, opp(i))));
    }
}

// Storage index of f_i(x) after zero steps (any scheme; with sparse
// addressing only for fluid cells).
template <int Q>
__device__ inline uint64_t index_t0(const LatticeArgs &a, const SparseArgs &sp, const Geom &g, int i)
{
    if (sp.on) return sp_index<Q>((uint32_t)sp.fmap[cidx(a, g)], i);
    if (a.et) return et_index<Q>(a, g, i, cdir(i, 0) < 0, cdir(i, 1) < 0, cdir(i, 2) < 0);
    return pidx<Q>(a, i, g.row, g.x);
}

// Relaxation rates of a cell: the molecular ones, those of the Smagorinsky
// relaxation time, or those of the learned closure.  The network runs on the
// matrix cores across the whole wavefront, so with CL_MLP every lane of the
// wavefront must call this; `active` marks the lanes that hold a fluid cell,
// and tab is the network's per-lane operand table (in LDS).  A cell whose
// features leave the trusted range, or whose network output is not finite,
// falls back to Smagorinsky and is counted in a.fallbacks.
template <int Q, int CL>
__device__ inline void closure_rates(const LatticeArgs &a, [[maybe_unused]] const uint32_t *tab, const float (&d)[Q],
                                     float drho, const Macro &M, [[maybe_unused]] bool active, float &wp, float &wm)
{
    wp = a.omp;
    wm = a.omm;
    if constexpr (CL == CL_SMAG || CL == CL_MLP) {
        float P[6];
        noneq_flux<Q>(a, d, drho, M, P);
        const float excess = smag_excess(a.tau, a.cs, flux_norm(P), M.rho);
        const float tsm = a.tau + excess;
        float tt = tsm;
        if constexpr (CL == CL_MLP) {
            const float ir = rcp(M.rho);
            float Pn[6], xf[6];
#pragma unroll
            for (int k = 0; k < 6; ++k) Pn[k] = P[k] * ir;
            closure_features(Pn, M.rho, a.tau, excess, xf);
            const int lane = (threadIdx.y * blockDim.x + threadIdx.x) & 63;
            const bool inside = features_in_range(a.mlp, xf);
            float xin[6];
#pragma unroll
            for (int k = 0; k < 6; ++k) xin[k] = inside ? xf[k] : a.mlp[P_MU + k];
            const float dtau = softplus_fast(mlp_forward_table(tab, xin, lane));
            const bool use = inside && isfinite(dtau);
            tt = use ? a.tau + dtau : tsm;
            const uint64_t fb = __ballot(active && !use);
            if (lane == 0 && fb) atomicAdd(a.fallbacks, (unsigned long long)__popcll(fb));
        }
        trt_rates(tt, a.magic, wp, wm);
    }
}

// Stage the network's per-lane operand table in LDS (all threads of the
// workgroup take part; the caller's barrier follows).
__device__ inline void stage_mlp_table(const LatticeArgs &a, uint32_t *tab_lds)
{
    const int tid = threadIdx.y * blockDim.x + threadIdx.x;
    const int nthr = blockDim.x * blockDim.y;
    for (int k = tid; k < TAB_WORDS * 64; k += nthr) tab_lds[k] = a.mlp_tab[k];
}

// Value a cut link returns to its own cell (deviation form).  The face's
// parameters are picked with an unrolled compare chain (uniform values,
// per-lane selects) rather than by indexing the argument block with a
// per-lane face number, which would force the block into scratch memory.
template <int Q>
__device__ inline float wall_value(const LatticeArgs &a, int face, int i, float v, const Macro &M)
{
    if (face < 0) return v;  // solid neighbour: plain bounce-back
    int k = BC_NOSLIP;
    float uw0 = 0.f, uw1 = 0.f, uw2 = 0.f, rw = 1.f;
#pragma unroll
    for (int f = 0; f < 6; ++f) {
        const bool sel = face == f;
        k = sel ? a.bc[f] : k;
        uw0 = sel ? a.ubc[f][0] : uw0;
        uw1 = sel ? a.ubc[f][1] : uw1;
        uw2 = sel ? a.ubc[f][2] : uw2;
        rw = sel ? a.rhobc[f] : rw;
    }
    const float w = (float)wgt<Q>(i);
    const int cx = cdir(i, 0), cy = cdir(i, 1), cz = cdir(i, 2);
    if (k == BC_VELOCITY) return v - 6.f * w * rw * (cx * uw0 + cy * uw1 + cz * uw2);
    if (k == BC_PRESSURE) {
        const float cu = cx * M.ux + cy * M.uy + cz * M.uz;
        const float usq = M.ux * M.ux + M.uy * M.uy + M.uz * M.uz;
        return -v + 2.f * w * (rw - 1.f + rw * (4.5f * cu * cu - 1.5f * usq));
    }
    return v;
}

// One path for every cell: the odd step selects the cell's own slot for
// links cut by a face or a solid neighbour (read side) and sends cut links'
// values to the own slot (write side); velocity and pressure faces modify
// those values in registers.
template <int Q, int ST, bool MASK>
__device__ inline void load_all(const LatticeArgs &a, const Geom &g, uint32_t m, int odd, float (&d)[Q])
{
    using S = Store<ST>;
    const typename S::T *A = (const typename S::T *)a.pdf;
    if (!odd) {
        const typename S::T *R = A + pidx<Q>(a, 0, g.row, g.x);
        for_dirs<0, Q>([&](auto I) {
            constexpr int i = decltype(I)::value;
            d[i] = S::template ld<Hint<i, MASK>::even>(R + (uint64_t)i * (uint32_t)a.sx);
        });
    } else {
        for_dirs<0, Q>([&](auto I) {
            constexpr int i = decltype(I)::value;
            const int dx = cdir(i, 0), dy = cdir(i, 1), dz = cdir(i, 2);
            const bool cut = face_cut(g, -dx, -dy, -dz) || (MASK && ((m >> opp(i)) & 1u));
            const uint64_t k = cut ? pidx<Q>(a, i, g.row, g.x) : pidx_nbr<Q>(a, g, opp(i), -dx, -dy, -dz);
            d[i] = S::template ld<Hint<i, MASK>::odd>(A + k);
        });
    }
}

template <int Q, int ST, bool MASK, bool SWAP>
__device__ inline void store_all(const LatticeArgs &a, const Geom &g, uint32_t m, int odd, const float (&d)[Q],
                                 const Macro &M, bool keep)
{
    using S = Store<ST>;
    typename S::T *A = (typename S::T *)a.pdf;
    if (!odd) {
        typename S::T *R = A + pidx<Q>(a, 0, g.row, g.x);
        for_dirs<0, Q>([&](auto I) {
            constexpr int i = decltype(I)::value;
            const int dx = cdir(i, 0), dy = cdir(i, 1), dz = cdir(i, 2);
            float v = d[i];
            if (a.any_vp && !keep && face_cut(g, dx, dy, dz))
                v = wall_value<Q>(a, deciding_face(a, g, dx, dy, dz), i, v, M);
            // a kept (solid) lane puts every slot's own value back (the TRT
            // collision has already exchanged its pairs)
            if constexpr (MASK && SWAP) v = keep ? d[opp(i)] : v;
            S::template st<Hint<i, MASK>::even>(R + (uint64_t)opp(i) * (uint32_t)a.sx, v);
        });
    } else {
        for_dirs<0, Q>([&](auto I) {
            constexpr int i = decltype(I)::value;
            const int dx = cdir(i, 0), dy = cdir(i, 1), dz = cdir(i, 2);
            const bool fcut = face_cut(g, dx, dy, dz);
            const bool cut = fcut || (MASK && ((m >> i) & 1u));
            float v = d[i];
            if (a.any_vp && fcut) v = wall_value<Q>(a, deciding_face(a, g, dx, dy, dz), i, v, M);
            const uint64_t k = cut ? pidx<Q>(a, opp(i), g.row, g.x) : pidx_nbr<Q>(a, g, i, dx, dy, dz);
            S::template st<Hint<i, MASK>::odd>(A + k, v);
        });
    }
}

// Calls f(integral_constant<Q>, integral_constant<ST>) for the runtime pair.
template <class Fn>
inline hipError_t dispatch(int q, int st, Fn &&f)
{
    using I19 = std::integral_constant<int, 19>;
    using I27 = std::integral_constant<int, 27>;
    using S0 = std::integral_constant<int, ST_F32>;
    using S1 = std::integral_constant<int, ST_F16>;
    using S2 = std::integral_constant<int, ST_BF16>;
    if (q == 19) {
        if (st == ST_F32) return f(I19{}, S0{});
        if (st == ST_F16) return f(I19{}, S1{});
        return f(I19{}, S2{});
    }
    if (st == ST_F32) return f(I27{}, S0{});
    if (st == ST_F16) return f(I27{}, S1{});
    return f(I27{}, S2{});
}

}  // namespace lbm
