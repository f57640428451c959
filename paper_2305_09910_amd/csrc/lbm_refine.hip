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
// deviations is the deviation of the average).  dy is +1 for a fine lattice
// above the coarse one, -1 below.  For each crossing direction i toward the
// coarse level (c_iy = -dy) and j = opp(i), per coarse step:
//   - the packet coarse interface cell X sent toward the fine level along j
//     is f*_j(X), which the coarse step left in X's own slot i; it stays
//     there until the coarse interface row is filled at the end;
//   - after each of the two fine steps: the fine interface cells x_f with
//     x_f + c_i in X (four of them) sent f*_i(x_f), now in their own slot j;
//     1/8 of their sum is added to acc_i(X), and slot j of the same cells
//     takes X's packet f*_j(X) (the source point x_f - c_j = x_f + c_i of
//     its link lies in X);
//   - after the second fine step, slot i of X takes acc_i(X).
// So one thread per coarse interface cell does all of it with no other
// thread touching its cells' slots, and the exchange is two launches per
// coarse step and fine level: k_refine_exchange after the first fine step
// (first: acc = sum) and after the second (last: X's slot i = acc + sum).
// acc is [q][nz_c][nx_c] FP32; only the directions i with c_iy = -dy are used.
//
// Bytes per launch (FP32 storage): per coarse interface cell and crossing
// direction (5 of D3Q19, 9 of D3Q27) 4 fine slots read and written (32 B),
// the coarse slot read (4 B), and acc written (first, 4 B) or read with the
// coarse slot written (last, 8 B).
#include "lattice.h"

namespace lbm {

constexpr int kRefineThreads = 256;

__device__ inline int wrap_int(int v, int n) { return v < 0 ? v + n : (v >= n ? v - n : v); }

// the exchange after a fine step (see above): one thread per coarse interface cell (X, Z)
template <int Q, int SC, int SF>
__global__ void __launch_bounds__(kRefineThreads)
    k_refine_exchange(LatticeArgs c, int yc, LatticeArgs f, int yf, int dy, int last, float *acc)
{
    using C = Store<SC>;
    using F = Store<SF>;
    typename C::T *Ac = (typename C::T *)c.pdf;
    typename F::T *Af = (typename F::T *)f.pdf;
    const int X = blockIdx.x * kRefineThreads + threadIdx.x, Z = blockIdx.y;
    if (X >= c.nx) return;
    const Geom gc = make_geom(c, X, yc, Z);
    const size_t plane = (size_t)c.nx * c.nz, k = (size_t)Z * c.nx + X;
    for_dirs<1, Q>([&](auto I) {
        constexpr int i = decltype(I)::value, j = opp(i);
        if (cdir(i, 1) != -dy) return;
        const uint64_t ci = pidx<Q>(c, i, gc.row, X);
        const auto packet = F::cvt(C::ld(Ac + ci));
        float s = 0.f;
#pragma unroll
        for (int bz = 0; bz < 2; ++bz) {
            const int zf = wrap_int(2 * Z + bz - cdir(i, 2), f.nz);
            const Geom g = make_geom(f, 0, yf, zf);
#pragma unroll
            for (int bx = 0; bx < 2; ++bx) {
                const int xf = wrap_int(2 * X + bx - cdir(i, 0), f.nx);
                typename F::T *p = Af + pidx<Q>(f, j, g.row, xf);
                s += F::ld(p);
                *p = packet;
            }
        }
        const float v = 0.125f * s;
        if (last)
            Ac[ci] = C::cvt(acc[i * plane + k] + v);
        else
            acc[i * plane + k] = v;
    });
}

hipError_t launch_refine_exchange(const LatticeArgs &c, int sc, int yc, const LatticeArgs &f, int q, int sf, int yf,
                                  int dy, int last, float *acc, hipStream_t s)
{
    const dim3 grid((unsigned)((c.nx + kRefineThreads - 1) / kRefineThreads), (unsigned)c.nz, 1);
    return dispatch(q, sf, [&](auto Q, auto SF) {
        auto go = [&](auto SC) {
            k_refine_exchange<Q.value, SC.value, SF.value><<<grid, kRefineThreads, 0, s>>>(c, yc, f, yf, dy, last, acc);
            return hipGetLastError();
        };
        if (sc == ST_F32) return go(std::integral_constant<int, ST_F32>{});
        if (sc == ST_F16) return go(std::integral_constant<int, ST_F16>{});
        return go(std::integral_constant<int, ST_BF16>{});
    });
}

}  // namespace lbm
