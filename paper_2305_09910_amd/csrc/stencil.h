// stencil.h -- D3Q19 / D3Q27 velocity sets for the device kernels.
//
// Directions come in opposite pairs (2k-1, 2k); direction 0 is the rest
// population.  Order: rest; the six axis neighbours; the twelve edge
// neighbours; for D3Q27 the eight corner neighbours.  Weights follow from
// |c|^2: D3Q19 {1/3, 1/18, 1/36}, D3Q27 {8/27, 2/27, 1/54, 1/216}; both sets
// have c_s^2 = 1/3.  Everything is constexpr so that unrolled loops over the
// directions fold the components into immediates.
#pragma once

namespace lbm {

__host__ __device__ constexpr int cdir(int i, int axis)
{
    constexpr int E[27][3] = {
        {0, 0, 0},
        {1, 0, 0},   {-1, 0, 0},   {0, 1, 0},   {0, -1, 0},  {0, 0, 1},  {0, 0, -1},
        {1, 1, 0},   {-1, -1, 0},  {1, -1, 0},  {-1, 1, 0},
        {1, 0, 1},   {-1, 0, -1},  {1, 0, -1},  {-1, 0, 1},
        {0, 1, 1},   {0, -1, -1},  {0, 1, -1},  {0, -1, 1},
        {1, 1, 1},   {-1, -1, -1}, {1, 1, -1},  {-1, -1, 1},
        {1, -1, 1},  {-1, 1, -1},  {-1, 1, 1},  {1, -1, -1},
    };
    return E[i][axis];
}

__host__ __device__ constexpr int opp(int i) { return i == 0 ? 0 : ((i & 1) ? i + 1 : i - 1); }

__host__ __device__ constexpr int norm1(int i)
{
    return (cdir(i, 0) != 0) + (cdir(i, 1) != 0) + (cdir(i, 2) != 0);
}

template <int Q>
__host__ __device__ constexpr double wgt(int i)
{
    if (Q == 19) {
        const int k = norm1(i);
        return k == 0 ? 1.0 / 3.0 : (k == 1 ? 1.0 / 18.0 : 1.0 / 36.0);
    }
    const int k = norm1(i);
    return k == 0 ? 8.0 / 27.0 : (k == 1 ? 2.0 / 27.0 : (k == 2 ? 1.0 / 54.0 : 1.0 / 216.0));
}

}  // namespace lbm
