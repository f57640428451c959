// lbm_closure.hip -- training data and training kernels of the learned
// LES closure: a 4^3 box filter of fine-grid fields, the per-cell dataset
// (six flux invariants -> target relaxation-time correction), and the MLP
// forward, backward (bfloat16 matrix cores, FP32 accumulation,
// deterministic reductions) and Adam update.
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

#include <algorithm>
#include <mutex>

#include "internal.h"
#include "mlp_wave.h"

namespace lbm {

// ---------------------------------------------------------------------------
// box filter over 4x4x4 blocks (one thread per coarse cell, FP64 sums)
// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(256) k_box_filter4(int nx, int ny, int nz, const float *__restrict__ rho,
                                                     const float *__restrict__ u, float *__restrict__ out)
{
    const int cx = nx / 4, cy = ny / 4, cz = nz / 4;
    const uint32_t nc = (uint32_t)cx * cy * cz;
    const uint32_t c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= nc) return;
    const int X = c % cx, Y = (c / cx) % cy, Z = c / ((uint32_t)cx * cy);
    const uint64_t nf = (uint64_t)nx * ny * nz;
    double s[10] = {0, 0, 0, 0, 0, 0, 0, 0, 0, 0};
    for (int dz = 0; dz < 4; ++dz)
        for (int dy = 0; dy < 4; ++dy) {
            const uint64_t row = ((uint64_t)(4 * Z + dz) * ny + (4 * Y + dy)) * nx + 4 * X;
#pragma unroll
            for (int dx = 0; dx < 4; ++dx) {
                const uint64_t f = row + dx;
                const double ux = u[f], uy = u[nf + f], uz = u[2 * nf + f];
                s[0] += rho[f];
                s[1] += ux;
                s[2] += uy;
                s[3] += uz;
                s[4] += ux * ux;
                s[5] += uy * uy;
                s[6] += uz * uz;
                s[7] += ux * uy;
                s[8] += ux * uz;
                s[9] += uy * uz;
            }
        }
#pragma unroll
    for (int k = 0; k < 10; ++k) out[(uint64_t)k * nc + c] = (float)(s[k] * (1.0 / 64.0));
}

hipError_t launch_box_filter4(int nx, int ny, int nz, const float *rho, const float *u, float *out, hipStream_t s)
{
    const uint32_t nc = (uint32_t)(nx / 4) * (ny / 4) * (nz / 4);
    k_box_filter4<<<(nc + 255) / 256, 256, 0, s>>>(nx, ny, nz, rho, u, out);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// closure dataset (one thread per coarse cell)
// ---------------------------------------------------------------------------
// derivative along an axis of a cell-centred field: central inside, wrapped
// on periodic axes, and next to a wall (value zero half a cell outside) the
// slope of the quadratic through the wall point and the two nearest cells
__device__ inline double deriv_axis(const float *g, int64_t stride, int i, int n, int periodic)
{
    if (periodic) {
        const int im = i == 0 ? n - 1 : i - 1, ip = i == n - 1 ? 0 : i + 1;
        return 0.5 * ((double)g[(int64_t)(ip - i) * stride] - (double)g[(int64_t)(im - i) * stride]);
    }
    if (n == 1) return 0.0;
    if (i == 0) return (double)g[0] + (double)g[stride] / 3.0;
    if (i == n - 1) return -((double)g[0] + (double)g[-stride] / 3.0);
    return 0.5 * ((double)g[stride] - (double)g[-stride]);
}

__global__ void __launch_bounds__(256) k_closure_dataset(int cx, int cy, int cz, int px, int py, int pz,
                                                         const float *__restrict__ filt, float tau, float cs,
                                                         float *__restrict__ xo, float *__restrict__ to)
{
    const uint32_t nc = (uint32_t)cx * cy * cz;
    const uint32_t c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= nc) return;
    const int pos[3] = {(int)(c % cx), (int)((c / cx) % cy), (int)(c / ((uint32_t)cx * cy))};
    const int ext[3] = {cx, cy, cz};
    const int per[3] = {px, py, pz};
    const int64_t strd[3] = {1, cx, (int64_t)cx * cy};
    double G[3][3];  // G[a][b] = d u_a / d x_b
#pragma unroll
    for (int a = 0; a < 3; ++a)
#pragma unroll
        for (int b = 0; b < 3; ++b)
            G[a][b] = deriv_axis(filt + (uint64_t)(1 + a) * nc + c, strd[b], pos[b], ext[b], per[b]);
    const double S[6] = {G[0][0], G[1][1], G[2][2], 0.5 * (G[0][1] + G[1][0]), 0.5 * (G[0][2] + G[2][0]),
                         0.5 * (G[1][2] + G[2][1])};
    const int A[6] = {0, 1, 2, 0, 0, 1}, B[6] = {0, 1, 2, 1, 2, 2};
    double ts[6];
#pragma unroll
    for (int m = 0; m < 6; ++m)
        ts[m] = (double)filt[(uint64_t)(4 + m) * nc + c] -
                (double)filt[(uint64_t)(1 + A[m]) * nc + c] * (double)filt[(uint64_t)(1 + B[m]) * nc + c];
    const double trt = (ts[0] + ts[1] + ts[2]) / 3.0;
    double dd = 0.0, ss = 0.0;
#pragma unroll
    for (int m = 0; m < 6; ++m) {
        const double mult = m < 3 ? 1.0 : 2.0;
        const double tdev = m < 3 ? ts[m] - trt : ts[m];
        dd += mult * tdev * S[m];
        ss += mult * S[m] * S[m];
    }
    double nut = -dd / (2.0 * ss + 1e-30);
    nut = nut < 0.0 ? 0.0 : nut;
    const double dtau = 3.0 * nut;
    double P[6];
#pragma unroll
    for (int m = 0; m < 6; ++m) P[m] = -(2.0 / 3.0) * ((double)tau + dtau) * S[m];
    // features (FP64 here, stored FP32)
    const double tr = P[0] + P[1] + P[2];
    const double d0 = P[0] - tr / 3.0, d1 = P[1] - tr / 3.0, d2 = P[2] - tr / 3.0;
    const double xy = P[3], xz = P[4], yz = P[5];
    const double nd = sqrt(d0 * d0 + d1 * d1 + d2 * d2 + 2.0 * (xy * xy + xz * xz + yz * yz));
    const double det = d0 * (d1 * d2 - yz * yz) - xy * (xy * d2 - yz * xz) + xz * (xy * yz - d1 * xz);
    const double np = sqrt(P[0] * P[0] + P[1] * P[1] + P[2] * P[2] + 2.0 * (xy * xy + xz * xz + yz * yz));
    const double rho = filt[c];
    const double t = (double)tau;
    const double asm_ = 18.0 * sqrt(2.0) * (double)cs * cs * (rho * np) / rho;
    const double excess = 0.5 * asm_ / (sqrt(t * t + asm_) + t);  // tau_smag - tau without cancellation
    float *x = xo + (uint64_t)c * 6;
    x[0] = (float)tr;
    x[1] = (float)nd;
    x[2] = (float)cbrt(det);
    x[3] = (float)(rho - 1.0);
    x[4] = (float)excess;
    x[5] = tau;
    to[c] = (float)dtau;
}

hipError_t launch_closure_dataset(int cx, int cy, int cz, const int *per, const float *filt, float tau, float cs,
                                  float *x, float *t, hipStream_t s)
{
    const uint32_t nc = (uint32_t)cx * cy * cz;
    k_closure_dataset<<<(nc + 255) / 256, 256, 0, s>>>(cx, cy, cz, per[0], per[1], per[2], filt, tau, cs, x, t);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// batched forward: one wavefront per 64 samples
// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(256) k_mlp_forward(const float *__restrict__ P, const float *__restrict__ X,
                                                     int64_t n, float *__restrict__ Y)
{
    const int lane = threadIdx.x & 63;
    const int64_t waves = (int64_t)gridDim.x * (blockDim.x >> 6);
    const int64_t w0 = (int64_t)blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6);
    const int64_t tiles = (n + 63) / 64;
    for (int64_t tile = w0; tile < tiles; tile += waves) {  // wave-uniform trip count
        const int64_t r = tile * 64 + lane;
        const bool act = r < n;
        float x[6];
#pragma unroll
        for (int k = 0; k < 6; ++k) x[k] = act ? X[r * 6 + k] : P[P_MU + k];
        const float o = mlp_forward_wave(P, x, lane);
        if (act) Y[r] = softplus_f(o);
    }
}

hipError_t launch_mlp_forward(const float *params, const float *x, int64_t n, float *y, hipStream_t s)
{
    if (n <= 0) return hipSuccess;
    const int64_t tiles = (n + 63) / 64;
    const int blocks = (int)std::min<int64_t>((tiles + 3) / 4, 8192);
    k_mlp_forward<<<blocks, 256, 0, s>>>(params, x, n, y);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// loss and gradient: forward + backward per 64-sample tile on the matrix
// cores; every block owns a fixed set of tiles and writes one partial
// gradient; a second kernel sums the partials in block order.
// ---------------------------------------------------------------------------
constexpr int GRAD_BLOCKS = 512;
constexpr int GRAD_WORDS = MLP_NPARAM + 1;  // gradients then the loss sum

size_t mlp_work_bytes(int64_t) { return (size_t)GRAD_BLOCKS * GRAD_WORDS * sizeof(float); }

// LDS tile [rows][64 samples] of bfloat16 bits
struct WaveTiles {
    uint16_t h1[32][64];  // layer-1 activations (rows: hidden unit)
    uint16_t d2[32][64];  // layer-2 deltas
    uint16_t d1[32][64];  // layer-1 deltas
    uint16_t z[8][64];    // standardised inputs (rows 6, 7 zero)
};

__device__ inline void wave_lds_sync()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
}

// operand of a K=8 slice (samples 8kb .. 8kb+7) read from a tile row
__device__ inline bf16x4 tile_operand(const uint16_t (*T)[64], int row, int kb, int lane)
{
    const int c0 = 8 * kb + 4 * ((lane >> 5) & 1);
    bf16x4 r;
    r.x = (short)T[row][c0];
    r.y = (short)T[row][c0 + 1];
    r.z = (short)T[row][c0 + 2];
    r.w = (short)T[row][c0 + 3];
    return r;
}

__device__ inline float sum32(float v)  // sum over lanes with equal l/32
{
#pragma unroll
    for (int o = 1; o < 32; o <<= 1) v += __shfl_xor(v, o, 64);
    return v;
}

__global__ void __launch_bounds__(256) k_mlp_loss_grad(const float *__restrict__ P, const float *__restrict__ X,
                                                       const float *__restrict__ T, int64_t n,
                                                       float *__restrict__ work)
{
    // per-wave tiles; after its loop each wave reuses its own tile region
    // for its partial gradient (GRAD_WORDS floats fit in one tile region)
    __shared__ WaveTiles tiles_lds[4];
    static_assert(sizeof(WaveTiles) >= GRAD_WORDS * sizeof(float), "partial does not fit");
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    WaveTiles &L = tiles_lds[wave];
    const bool hi = lane >= 32;
    const int col = lane & 31;
    const float inv_n = 1.f / (float)n;

    f32x16 gW2 = {}, gW1 = {};
    float gb1[16], gb2[16], gW3[16];
#pragma unroll
    for (int r = 0; r < 16; ++r) gb1[r] = gb2[r] = gW3[r] = 0.f;
    float gb3 = 0.f, loss = 0.f;

    const int64_t ntiles = (n + 63) / 64;
    const int64_t per_block = (ntiles + gridDim.x - 1) / gridDim.x;
    const int64_t t_lo = (int64_t)blockIdx.x * per_block;
    const int64_t t_hi = std::min<int64_t>(ntiles, t_lo + per_block);
    for (int64_t tile = t_lo + wave; tile < t_hi; tile += 4) {  // wave-uniform trip count
        const int64_t r = tile * 64 + lane;
        const bool act = r < n;
        float x[6], z[6];
#pragma unroll
        for (int k = 0; k < 6; ++k) x[k] = act ? X[r * 6 + k] : P[P_MU + k];
        f32x16 h1_0, h1_1, h2_0, h2_1;
        const float o = mlp_forward_wave(P, x, lane, z, h1_0, h1_1, h2_0, h2_1);
        const float y = softplus_f(o);
        const float e = act ? y - T[r] : 0.f;
        loss += e * e;
        const float dout = 2.f * e * inv_n * sigmoid_f(o);  // own sample
        gb3 += dout;
        const float dpart = __shfl_xor(dout, 32, 64);
        const float dout0 = hi ? dpart : dout;  // sample col (block 0)
        const float dout1 = hi ? dout : dpart;  // sample col + 32 (block 1)

        // layer 3 and the delta of layer 2 (accumulator layout)
        f32x16 d2_0, d2_1;
#pragma unroll
        for (int rr = 0; rr < 16; ++rr) {
            const float w3 = P[P_W3 + drow(rr, lane)];
            gW3[rr] += dout0 * h2_0[rr] + dout1 * h2_1[rr];
            d2_0[rr] = dout0 * w3 * (1.f - h2_0[rr] * h2_0[rr]);
            d2_1[rr] = dout1 * w3 * (1.f - h2_1[rr] * h2_1[rr]);
            gb2[rr] += d2_0[rr] + d2_1[rr];
            const int row = drow(rr, lane);
            L.h1[row][col] = bf16_rne_bits(h1_0[rr]);
            L.h1[row][col + 32] = bf16_rne_bits(h1_1[rr]);
            L.d2[row][col] = bf16_rne_bits(d2_0[rr]);
            L.d2[row][col + 32] = bf16_rne_bits(d2_1[rr]);
        }
        // z tile: lane writes its own sample's inputs
#pragma unroll
        for (int k = 0; k < 6; ++k) L.z[k][lane] = bf16_rne_bits(z[k]);
        L.z[6][lane] = 0;
        L.z[7][lane] = 0;

        // delta of layer 1: D[k][s] = sum_m W2[m][k] d2[m][s], chained from d2's layout
        f32x16 d1_0 = {}, d1_1 = {};
#pragma unroll
        for (int kb = 0; kb < 4; ++kb) {
            const int m0 = 8 * kb + 4 * ((lane >> 5) & 1);
            const bf16x4 a = pack4(P[P_W2 + (m0 + 0) * 32 + col], P[P_W2 + (m0 + 1) * 32 + col],
                                   P[P_W2 + (m0 + 2) * 32 + col], P[P_W2 + (m0 + 3) * 32 + col]);
            d1_0 = mfma32(a, pack4(d2_0[4 * kb], d2_0[4 * kb + 1], d2_0[4 * kb + 2], d2_0[4 * kb + 3]), d1_0);
            d1_1 = mfma32(a, pack4(d2_1[4 * kb], d2_1[4 * kb + 1], d2_1[4 * kb + 2], d2_1[4 * kb + 3]), d1_1);
        }
#pragma unroll
        for (int rr = 0; rr < 16; ++rr) {
            d1_0[rr] *= 1.f - h1_0[rr] * h1_0[rr];
            d1_1[rr] *= 1.f - h1_1[rr] * h1_1[rr];
            gb1[rr] += d1_0[rr] + d1_1[rr];
            const int row = drow(rr, lane);
            L.d1[row][col] = bf16_rne_bits(d1_0[rr]);
            L.d1[row][col + 32] = bf16_rne_bits(d1_1[rr]);
        }
        wave_lds_sync();
        // weight gradients: contractions over the 64 samples (8 slices of 8)
#pragma unroll
        for (int kb = 0; kb < 8; ++kb) {
            gW2 = mfma32(tile_operand(L.d2, col, kb, lane), tile_operand(L.h1, col, kb, lane), gW2);
            const bf16x4 bz = col < 8 ? tile_operand(L.z, col, kb, lane) : bf16x4{0, 0, 0, 0};
            gW1 = mfma32(tile_operand(L.d1, col, kb, lane), bz, gW1);
        }
        wave_lds_sync();
    }

    // reduce each wave's partial into its own tile region (fixed order)
    float *R = reinterpret_cast<float *>(&tiles_lds[wave]);
#pragma unroll
    for (int rr = 0; rr < 16; ++rr) {
        const int row = drow(rr, lane);
        R[P_W2 + row * 32 + col] = gW2[rr];
        if (col < 6) R[P_W1 + row * 6 + col] = gW1[rr];
        const float a = sum32(gb1[rr]), b = sum32(gb2[rr]), c = sum32(gW3[rr]);
        if (col == 0) {
            R[P_B1 + row] = a;
            R[P_B2 + row] = b;
            R[P_W3 + row] = c;
        }
    }
    float g3 = gb3, ls = loss;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        g3 += __shfl_xor(g3, o, 64);
        ls += __shfl_xor(ls, o, 64);
    }
    if (lane == 0) {
        R[P_B3] = g3;
        R[MLP_NPARAM] = ls;
    }
    __syncthreads();
    const float *R0 = reinterpret_cast<const float *>(&tiles_lds[0]);
    const float *R1 = reinterpret_cast<const float *>(&tiles_lds[1]);
    const float *R2 = reinterpret_cast<const float *>(&tiles_lds[2]);
    const float *R3 = reinterpret_cast<const float *>(&tiles_lds[3]);
    for (int k = threadIdx.x; k < GRAD_WORDS; k += blockDim.x)
        work[(size_t)blockIdx.x * GRAD_WORDS + k] = ((R0[k] + R1[k]) + R2[k]) + R3[k];
}

__global__ void __launch_bounds__(256) k_mlp_grad_final(const float *__restrict__ work, int nblocks, int64_t n,
                                                        float *__restrict__ grad, float *__restrict__ loss)
{
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= GRAD_WORDS) return;
    double s = 0.0;
    for (int b = 0; b < nblocks; ++b) s += work[(size_t)b * GRAD_WORDS + k];
    if (k < MLP_NPARAM)
        grad[k] = (float)s;
    else
        loss[0] = (float)(s / (double)n);
}

hipError_t launch_mlp_loss_grad(const float *params, const float *x, const float *t, int64_t n, float *grad,
                                float *loss, void *work, hipStream_t s)
{
    k_mlp_loss_grad<<<GRAD_BLOCKS, 256, 0, s>>>(params, x, t, n, (float *)work);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    k_mlp_grad_final<<<(GRAD_WORDS + 255) / 256, 256, 0, s>>>((const float *)work, GRAD_BLOCKS, n, grad, loss);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Loss and gradient for callers that cannot allocate device memory (code
// under graph capture, serving loops): the per-block partial gradients go to
// a file-scope device array instead of a caller workspace.  Each device the
// library runs on holds its own copy until the process ends.  Every call on a
// device shares that copy, so calls that overlap on one device race.  Every
// call writes each partial in full (blocks without samples write zeros), so
// nothing needs clearing between calls.
// ---------------------------------------------------------------------------
constexpr size_t NOALLOC_SCRATCH_FLOATS = (size_t)GRAD_BLOCKS * GRAD_WORDS;
static __device__ __align__(256) float scratch[NOALLOC_SCRATCH_FLOATS];

size_t mlp_noalloc_scratch_bytes() { return NOALLOC_SCRATCH_FLOATS * sizeof(float); }

constexpr int SCRATCH_MAX_DEVICES = 64;
static std::mutex scratch_mu;
static void *scratch_ptr[SCRATCH_MAX_DEVICES];

// Device address of the current device's copy of `scratch`, looked up once
// per device with that device current.  In host code the array's name is
// only a stand-in for the symbol, never a device address.
static hipError_t scratch_address(void **out)
{
    int dev = -1;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    if (dev < 0 || dev >= SCRATCH_MAX_DEVICES) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(scratch_mu);
    if (!scratch_ptr[dev]) {
        void *p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        if (!p) return hipErrorInvalidSymbol;
        scratch_ptr[dev] = p;
    }
    *out = scratch_ptr[dev];
    return hipSuccess;
}

hipError_t launch_mlp_loss_grad_noalloc(const float *params, const float *x, const float *t, int64_t n,
                                        float *grad, float *loss, hipStream_t s)
{
    if (mlp_work_bytes(n) > mlp_noalloc_scratch_bytes()) return hipErrorInvalidValue;
    void *w = nullptr;
    const hipError_t e = scratch_address(&w);
    if (e != hipSuccess) return e;
    return launch_mlp_loss_grad(params, x, t, n, grad, loss, w, s);
}

// ---------------------------------------------------------------------------
// Adam (Kingma & Ba) on the 1313 network parameters
// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(256) k_mlp_adam(float *p, const float *g, float *m, float *v, float c1, float c2,
                                                  float lr, float b1, float b2, float eps)
{
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= MLP_NPARAM) return;
    const float gk = g[k];
    const float mk = b1 * m[k] + (1.f - b1) * gk;
    const float vk = b2 * v[k] + (1.f - b2) * gk * gk;
    m[k] = mk;
    v[k] = vk;
    p[k] -= lr * (mk / c1) / (sqrtf(vk / c2) + eps);
}

hipError_t launch_mlp_adam(float *p, const float *g, float *m, float *v, int64_t step, float lr, float b1, float b2,
                           float eps, hipStream_t s)
{
    const float c1 = (float)(1.0 - pow((double)b1, (double)step));
    const float c2 = (float)(1.0 - pow((double)b2, (double)step));
    k_mlp_adam<<<(MLP_NPARAM + 255) / 256, 256, 0, s>>>(p, g, m, v, c1, c2, lr, b1, b2, eps);
    return hipGetLastError();
}

}  // namespace lbm
