// lbm_refine.hip -- the packet exchange of a 2:1 grid refinement between a
// coarse lattice and fine lattices below and/or above it (the paper's 2:1
// block refinement, Section 3, joined by coarse-to-fine and fine-to-coarse
// kernels, Section 5.2; the volumetric, mass-conservative scheme of Rohde,
// Kandhai, Derksen & van den Akker 2006).
//
// The interface is a plane normal to y; x and z are periodic on every level
// and a fine lattice has twice the coarse nx and nz.  Within a lattice the
// interface face is a no-slip face (the step kernels see BC_NOSLIP), so the
// packets that cross it come back into the emitting cell.  Every population
// these kernels touch has its source across the interface: its link is cut,
// and in the AA pattern a cut link's population sits in the cell's own slot
// after any number of steps.  So the kernels read and write own slots of the
// interface rows only, whatever the step parity.
//
// Populations are stored as deviations f_i - w_i; w_i = w_opposite(i), so the
// exchange works on deviations directly (a copy is exact, and an average of
// deviations is the deviation of the average).  Per coarse step:
//   record:      cout[i](X) = f_opp(i)(X) of the coarse interface row, c_iy = dy
//                (the packet coarse cell X sent across toward the fine level);
//   twice:       fine step; add: acc[i](Y) (+)= 1/8 sum of f_opp(i)(x_f) over
//                the four fine interface cells whose target x_f + c_i lies in
//                coarse cell Y, c_iy = -dy; fill fine: f_j(x_f) = cout[j](X)
//                for the coarse cell X containing the source point x_f - c_j,
//                c_jy = dy;
//   fill coarse: f_i(Y) = acc[i](Y) in the coarse interface row, c_iy = -dy.
// dy is +1 for a fine lattice above the coarse one, -1 below.  The plane
// buffers cout and acc are [q][nz_c][nx_c] FP32; only the directions named
// above are used.
//
// Bytes per launch (FP32): record and fill coarse 4 (q_y) n_c * (4 + 4), add
// 4 (q_y) n_c * (4 * 4 + 4), fill fine 4 (q_y) 4 n_c * (4 + 4) (the plane
// buffer is read from cache), with q_y = 5 (D3Q19) or 9 (D3Q27) directions
// and n_c = nx_c nz_c coarse interface cells: a few MB per coarse step at
// the sizes of interest, small beside the levels' own steps.
#include "lattice.h"

namespace lbm {

constexpr int kRefineThreads = 256;

__device__ inline int wrap_int(int v, int n) { return v < 0 ? v + n : (v >= n ? v - n : v); }

// record the packets coarse interface row yc sent across
template <int Q, int ST>
__global__ void __launch_bounds__(kRefineThreads) k_refine_record(LatticeArgs a, int yc, int dy, float *cout)
{
    using S = Store<ST>;
    const typename S::T *A = (const typename S::T *)a.pdf;
    const int x = blockIdx.x * kRefineThreads + threadIdx.x, z = blockIdx.y;
    if (x >= a.nx) return;
    const Geom g = make_geom(a, x, yc, z);
    const size_t plane = (size_t)a.nx * a.nz, k = (size_t)z * a.nx + x;
    for_dirs<1, Q>([&](auto I) {
        constexpr int i = decltype(I)::value;
        if (cdir(i, 1) == dy) cout[i * plane + k] = S::ld(A + pidx<Q>(a, opp(i), g.row, x));
    });
}

// fine packets sent across: a gather per coarse cell (four fine cells per
// direction), so no two threads write one sum
template <int Q, int ST>
__global__ void __launch_bounds__(kRefineThreads)
    k_refine_add(LatticeArgs f, int yf, int dy, int nxc, int nzc, int first, float *acc)
{
    using S = Store<ST>;
    const typename S::T *A = (const typename S::T *)f.pdf;
    const int X = blockIdx.x * kRefineThreads + threadIdx.x, Z = blockIdx.y;
    if (X >= nxc) return;
    const size_t plane = (size_t)nxc * nzc, k = (size_t)Z * nxc + X;
    for_dirs<1, Q>([&](auto I) {
        constexpr int i = decltype(I)::value;
        if (cdir(i, 1) != -dy) return;
        // fine cells x_f with x_f + c_i in {2X, 2X + 1} (and the same in z)
        float s = 0.f;
#pragma unroll
        for (int bz = 0; bz < 2; ++bz) {
            const int zf = wrap_int(2 * Z + bz - cdir(i, 2), f.nz);
            const Geom g = make_geom(f, 0, yf, zf);
#pragma unroll
            for (int bx = 0; bx < 2; ++bx) {
                const int xf = wrap_int(2 * X + bx - cdir(i, 0), f.nx);
                s += S::ld(A + pidx<Q>(f, opp(i), g.row, xf));
            }
        }
        const float v = 0.125f * s;
        acc[i * plane + k] = first ? v : acc[i * plane + k] + v;
    });
}

// the coarse packets enter the fine interface row
template <int Q, int ST>
__global__ void __launch_bounds__(kRefineThreads)
    k_refine_fill_fine(LatticeArgs f, int yf, int dy, int nxc, int nzc, const float *cout)
{
    using S = Store<ST>;
    typename S::T *A = (typename S::T *)f.pdf;
    const int x = blockIdx.x * kRefineThreads + threadIdx.x, z = blockIdx.y;
    if (x >= f.nx) return;
    const Geom g = make_geom(f, x, yf, z);
    const size_t plane = (size_t)nxc * nzc;
    for_dirs<1, Q>([&](auto J) {
        constexpr int j = decltype(J)::value;
        if (cdir(j, 1) != dy) return;
        const int px = wrap_int(x - cdir(j, 0), f.nx) >> 1, pz = wrap_int(z - cdir(j, 2), f.nz) >> 1;
        A[pidx<Q>(f, j, g.row, x)] = S::cvt(cout[j * plane + (size_t)pz * nxc + px]);
    });
}

// the summed fine packets enter the coarse interface row
template <int Q, int ST>
__global__ void __launch_bounds__(kRefineThreads) k_refine_fill_coarse(LatticeArgs a, int yc, int dy, const float *acc)
{
    using S = Store<ST>;
    typename S::T *A = (typename S::T *)a.pdf;
    const int x = blockIdx.x * kRefineThreads + threadIdx.x, z = blockIdx.y;
    if (x >= a.nx) return;
    const Geom g = make_geom(a, x, yc, z);
    const size_t plane = (size_t)a.nx * a.nz, k = (size_t)z * a.nx + x;
    for_dirs<1, Q>([&](auto I) {
        constexpr int i = decltype(I)::value;
        if (cdir(i, 1) == -dy) A[pidx<Q>(a, i, g.row, x)] = S::cvt(acc[i * plane + k]);
    });
}

static dim3 plane_grid(int nx, int nz) { return dim3((unsigned)((nx + kRefineThreads - 1) / kRefineThreads), (unsigned)nz, 1); }

hipError_t launch_refine_record(const LatticeArgs &c, int q, int st, int yc, int dy, float *cout, hipStream_t s)
{
    return dispatch(q, st, [&](auto Q, auto ST) {
        k_refine_record<Q.value, ST.value><<<plane_grid(c.nx, c.nz), kRefineThreads, 0, s>>>(c, yc, dy, cout);
        return hipGetLastError();
    });
}

hipError_t launch_refine_add(const LatticeArgs &f, int q, int st, int yf, int dy, int nxc, int nzc, int first,
                             float *acc, hipStream_t s)
{
    return dispatch(q, st, [&](auto Q, auto ST) {
        k_refine_add<Q.value, ST.value><<<plane_grid(nxc, nzc), kRefineThreads, 0, s>>>(f, yf, dy, nxc, nzc, first, acc);
        return hipGetLastError();
    });
}

hipError_t launch_refine_fill_fine(const LatticeArgs &f, int q, int st, int yf, int dy, int nxc, int nzc,
                                   const float *cout, hipStream_t s)
{
    return dispatch(q, st, [&](auto Q, auto ST) {
        k_refine_fill_fine<Q.value, ST.value><<<plane_grid(f.nx, f.nz), kRefineThreads, 0, s>>>(f, yf, dy, nxc, nzc, cout);
        return hipGetLastError();
    });
}

hipError_t launch_refine_fill_coarse(const LatticeArgs &c, int q, int st, int yc, int dy, const float *acc, hipStream_t s)
{
    return dispatch(q, st, [&](auto Q, auto ST) {
        k_refine_fill_coarse<Q.value, ST.value><<<plane_grid(c.nx, c.nz), kRefineThreads, 0, s>>>(c, yc, dy, acc);
        return hipGetLastError();
    });
}

}  // namespace lbm
