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

namespace lbm {

// ---------------------------------------------------------------------------
// Moment bases of the multiple-relaxation-time collision.
// D3Q19: nineteen mutually orthogonal polynomials of c (density, energy,
// energy square, momentum, heat flux, the five traceless second-order
// moments, two fourth-order moments, three third-order anti-symmetric ones).
// D3Q27: the products T_a(c_x) T_b(c_y) T_c(c_z) with T_0 = 1, T_1 = c,
// T_2 = 3c^2 - 2 (row index a + 3b + 9c).
// Rate groups: density, momentum, viscous, energy, energy square, heat
// flux, fourth-order, third-order anti-symmetric.
// ---------------------------------------------------------------------------
enum { MG_RHO = 0, MG_J = 1, MG_NU = 2, MG_E = 3, MG_EPS = 4, MG_Q = 5, MG_PI = 6, MG_M = 7 };

__host__ __device__ constexpr int mrt19_group(int a)
{
    constexpr int G[19] = {MG_RHO, MG_E,  MG_EPS, MG_J,  MG_Q,  MG_J,  MG_Q,  MG_J,  MG_Q, MG_NU,
                           MG_PI,  MG_NU, MG_PI,  MG_NU, MG_NU, MG_NU, MG_M,  MG_M,  MG_M};
    return G[a];
}

__host__ __device__ constexpr int mrt19_value(int a, int i)
{
    const int x = cdir(i, 0), y = cdir(i, 1), z = cdir(i, 2);
    const int c2 = x * x + y * y + z * z;
    switch (a) {
    case 0: return 1;
    case 1: return 19 * c2 - 30;
    case 2: return (21 * c2 * c2 - 53 * c2 + 24) / 2;
    case 3: return x;
    case 4: return (5 * c2 - 9) * x;
    case 5: return y;
    case 6: return (5 * c2 - 9) * y;
    case 7: return z;
    case 8: return (5 * c2 - 9) * z;
    case 9: return 3 * x * x - c2;
    case 10: return (3 * c2 - 5) * (3 * x * x - c2);
    case 11: return y * y - z * z;
    case 12: return (3 * c2 - 5) * (y * y - z * z);
    case 13: return x * y;
    case 14: return y * z;
    case 15: return x * z;
    case 16: return (y * y - z * z) * x;
    case 17: return (z * z - x * x) * y;
    default: return (x * x - y * y) * z;
    }
}

__host__ __device__ constexpr int cheb3(int k, int c) { return k == 0 ? 1 : (k == 1 ? c : 3 * c * c - 2); }

__host__ __device__ constexpr int mrt27_value(int a, int i)
{
    return cheb3(a % 3, cdir(i, 0)) * cheb3((a / 3) % 3, cdir(i, 1)) * cheb3(a / 9, cdir(i, 2));
}

__host__ __device__ constexpr int mrt27_group(int a)
{
    const int kx = a % 3, ky = (a / 3) % 3, kz = a / 9;
    const int ones = (kx == 1) + (ky == 1) + (kz == 1), twos = (kx == 2) + (ky == 2) + (kz == 2);
    const int order = ones + 2 * twos;
    return order == 0 ? MG_RHO
         : order == 1 ? MG_J
         : order == 2 ? MG_NU
         : order == 3 ? MG_Q
         : order == 4 ? (ones == 0 ? MG_E : MG_PI)
         : order == 5 ? MG_M
                      : MG_EPS;
}

template <int Q>
__host__ __device__ constexpr int mrt_value(int a, int i)
{
    return Q == 19 ? mrt19_value(a, i) : mrt27_value(a, i);
}

template <int Q>
__host__ __device__ constexpr int mrt_group(int a)
{
    return Q == 19 ? mrt19_group(a) : mrt27_group(a);
}

// squared norm of row a (the rows are orthogonal, so M^-1 = M^T diag(1/norm))
template <int Q>
__host__ __device__ constexpr int mrt_norm(int a)
{
    int s = 0;
    for (int i = 0; i < Q; ++i) s += mrt_value<Q>(a, i) * mrt_value<Q>(a, i);
    return s;
}

// exact zero for sums that vanish up to the rounding of the weights
__host__ __device__ constexpr double snap0(double v) { return (v < 1e-12 && v > -1e-12) ? 0.0 : v; }

// Lattice constants of row a: A = sum_i w_i M_ai, B_k = sum_i w_i M_ai c_ik,
// C_kl = sum_i w_i M_ai c_ik c_il.  They give the moments of f^eq and of
// the Guo source in closed form.
template <int Q>
__host__ __device__ constexpr double mrt_A(int a)
{
    double s = 0.0;
    for (int i = 0; i < Q; ++i) s += wgt<Q>(i) * mrt_value<Q>(a, i);
    return snap0(s);
}

template <int Q>
__host__ __device__ constexpr double mrt_B(int a, int k)
{
    double s = 0.0;
    for (int i = 0; i < Q; ++i) s += wgt<Q>(i) * mrt_value<Q>(a, i) * cdir(i, k);
    return snap0(s);
}

template <int Q>
__host__ __device__ constexpr double mrt_C(int a, int k, int l)
{
    double s = 0.0;
    for (int i = 0; i < Q; ++i) s += wgt<Q>(i) * mrt_value<Q>(a, i) * cdir(i, k) * cdir(i, l);
    return snap0(s);
}

// axis of a momentum row (-1 for other rows)
template <int Q>
__host__ __device__ constexpr int mrt_j_axis(int a)
{
    if (mrt_group<Q>(a) != MG_J) return -1;
    for (int k = 0; k < 3; ++k) {
        bool same = true;
        for (int i = 0; i < Q; ++i) same = same && mrt_value<Q>(a, i) == cdir(i, k);
        if (same) return k;
    }
    return -1;
}

}  // namespace lbm

namespace lbm {

// ---------------------------------------------------------------------------
// Hermite polynomials of the hybrid recursive regularised collision (D3Q19).
// Second order: H_ab = c_a c_b - c_s^2 delta_ab.  Third order: D3Q19 carries
// the mixed polynomials H_aab only as the six sums and differences
// T_0,1 = H_xxy +- H_yzz, T_2,3 = H_xzz +- H_xyy, T_4,5 = H_yyz +- H_xxz,
// which are orthogonal with the lattice weights (norms 2/27 and 6/27).
// ---------------------------------------------------------------------------
__host__ __device__ constexpr double herm3(int i, int a, int b, int g)
{
    return (double)(cdir(i, a) * cdir(i, b) * cdir(i, g)) -
           (cdir(i, a) * (b == g) + cdir(i, b) * (a == g) + cdir(i, g) * (a == b)) / 3.0;
}

__host__ __device__ constexpr double t3val(int i, int k)
{
    constexpr int A[6][2][3] = {{{0, 0, 1}, {1, 2, 2}}, {{0, 0, 1}, {1, 2, 2}}, {{0, 2, 2}, {0, 1, 1}},
                                {{0, 2, 2}, {0, 1, 1}}, {{1, 1, 2}, {0, 0, 2}}, {{1, 1, 2}, {0, 0, 2}}};
    const double s = (k & 1) ? -1.0 : 1.0;
    return herm3(i, A[k][0][0], A[k][0][1], A[k][0][2]) + s * herm3(i, A[k][1][0], A[k][1][1], A[k][1][2]);
}

__host__ __device__ constexpr double t3norm(int k)
{
    double s = 0.0;
    for (int i = 0; i < 19; ++i) s += wgt<19>(i) * t3val(i, k) * t3val(i, k);
    return s;
}

}  // namespace lbm
