// mlp_wave.h -- wavefront-level MLP 6 -> 32 -> 32 -> 1 on the bfloat16 matrix
// cores of gfx950 (v_mfma_f32_32x32x8_bf16, FP32 accumulation).
//
// One wavefront evaluates the network for its 64 lanes at once: lane l owns
// sample (cell) l.  The hidden layers are computed transposed, H^T = W X^T,
// as two 32x32 blocks (samples 0-31 and 32-63).  The accumulator layout of
// a 32x32x8 product -- lane l, register r holds row 8(r/4) + 4(l/32) + r%4
// and column l%32 -- is exactly the B-operand layout of the next 32x32x8
// product for K-block r/4, so layer 1 feeds layer 2 without any data
// movement.  The third layer (32 -> 1) is a 16-term dot product per lane
// plus one exchange between lanes l and l^32.
//
// Operand precision: inputs and weights of every layer are rounded to
// bfloat16 (round to nearest even); accumulation, biases and activations
// are FP32.  Output: o (pre-softplus); the correction is softplus(o) >= 0.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace lbm {

typedef short bf16x4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf16x2 __attribute__((ext_vector_type(2)));
typedef float f32x2 __attribute__((ext_vector_type(2)));
typedef float f32x16 __attribute__((ext_vector_type(16)));

// parameter block (FP32): W1[32][6], b1[32], W2[32][32], b2[32], W3[32], b3,
// then mu[6], sigma[6], lo[6], hi[6]
constexpr int P_W1 = 0, P_B1 = 192, P_W2 = 224, P_B2 = 1248, P_W3 = 1280, P_B3 = 1312;
constexpr int P_MU = 1313, P_SG = 1319, P_LO = 1325, P_HI = 1331;

// FP32 -> bfloat16, round to nearest even (gfx950 converts in hardware)
__device__ inline uint16_t bf16_rne_bits(float v) { return __builtin_bit_cast(uint16_t, (__bf16)v); }

__device__ inline float bf16_round(float v) { return __uint_as_float((uint32_t)bf16_rne_bits(v) << 16); }

// two values to bfloat16 (round to nearest even) in one v_cvt_pk_bf16_f32
__device__ inline bf16x2 pack2(float a, float b)
{
    const f32x2 v = {a, b};
    return __builtin_convertvector(v, bf16x2);
}

__device__ inline uint32_t pack2_bits(float a, float b) { return __builtin_bit_cast(uint32_t, pack2(a, b)); }

__device__ inline bf16x4 pack4(float a, float b, float c, float d)
{
    const uint64_t lo = pack2_bits(a, b), hi = pack2_bits(c, d);
    return __builtin_bit_cast(bf16x4, lo | (hi << 32));
}

// row of the 32x32 result held by accumulator register r of lane l
__device__ inline int drow(int r, int lane) { return 8 * (r >> 2) + 4 * ((lane >> 5) & 1) + (r & 3); }

__device__ inline f32x16 mfma32(bf16x4 a, bf16x4 b, f32x16 c)
{
    return __builtin_amdgcn_mfma_f32_32x32x8bf16_1k(a, b, c, 0, 0, 0);
}

// tanh in FP32: odd Taylor polynomial below |x| = 0.1 (truncation < 1e-10),
// (1 - e^{-2|x|}) / (1 + e^{-2|x|}) above.
__device__ inline float tanh_f(float x)
{
    const float ax = fabsf(x);
    const float x2 = x * x;
    const float p = x * (1.f + x2 * (-1.f / 3.f + x2 * (2.f / 15.f + x2 * (-17.f / 315.f))));
    const float e = __expf(-2.f * ax);
    const float t = copysignf((1.f - e) / (1.f + e), x);
    return ax < 0.1f ? p : t;
}

// tanh(x) = 1 - 2 / (1 + e^{2x}) with the hardware exp2 and reciprocal:
// five instructions, absolute error ~1e-7 (below the bfloat16 rounding the
// activations meet next); saturates correctly for large |x|.
__device__ inline float tanh_fast(float x)
{
    const float e = __builtin_amdgcn_exp2f(x * 2.8853900817779268f);  // 2 log2(e)
    return fmaf(-2.f, __builtin_amdgcn_rcpf(1.f + e), 1.f);
}

__device__ inline float softplus_f(float o) { return o > 20.f ? o : log1pf(__expf(o)); }

__device__ inline float sigmoid_f(float o) { return 1.f / (1.f + __expf(-o)); }

// softplus(o) = max(o, 0) + log1p(e) with e = exp(-|o|) <= 1, from the
// hardware exp2, log2 and reciprocal.  log1p(e) is taken as
// log(1 + e) * e / ((1 + e) - 1): the quotient cancels the rounding error of
// 1 + e, so the result stays within a few ulp for every e (Goldberg 1991,
// Theorem 4).  NaN in, NaN out; +inf in, +inf out.
__device__ inline float softplus_fast(float o)
{
    const float e = __builtin_amdgcn_exp2f(-fabsf(o) * 1.4426950408889634f);
    const float u = 1.f + e;
    const float l = u == 1.f ? e : __builtin_amdgcn_logf(u) * 0.6931471805599453f * e * __builtin_amdgcn_rcpf(u - 1.f);
    return fmaxf(o, 0.f) + l;
}

// Standardised inputs of this lane and the B operands of layer 1 for the
// two sample blocks: block b holds samples 32b .. 32b+31 as columns; lane l
// supplies inputs 4(l/32) .. 4(l/32)+3 (inputs 6 and 7 are zero padding).
__device__ inline void layer1_operands(const float *__restrict__ P, const float (&x)[6], int lane, float (&z)[6],
                                       bf16x4 &b0, bf16x4 &b1)
{
#pragma unroll
    for (int k = 0; k < 6; ++k) z[k] = (x[k] - P[P_MU + k]) / P[P_SG + k];
    float zp[6];
#pragma unroll
    for (int k = 0; k < 6; ++k) zp[k] = __shfl_xor(z[k], 32, 64);
    const bool hi = lane >= 32;
    b0 = hi ? pack4(zp[4], zp[5], 0.f, 0.f) : pack4(z[0], z[1], z[2], z[3]);
    b1 = hi ? pack4(z[4], z[5], 0.f, 0.f) : pack4(zp[0], zp[1], zp[2], zp[3]);
}

// A operand of layer 1: W1[l%32][4(l/32)+t], zero for the padded inputs.
__device__ inline bf16x4 layer1_weights(const float *__restrict__ P, int lane)
{
    const int row = lane & 31, k0 = 4 * ((lane >> 5) & 1);
    float w[4];
#pragma unroll
    for (int t = 0; t < 4; ++t) w[t] = (k0 + t < 6) ? P[P_W1 + row * 6 + k0 + t] : 0.f;
    return pack4(w[0], w[1], w[2], w[3]);
}

// A operand of layer 2 for K-block kb: W2[l%32][8kb + 4(l/32) + t].
__device__ inline bf16x4 layer2_weights(const float *__restrict__ P, int lane, int kb)
{
    const int row = lane & 31, k0 = 8 * kb + 4 * ((lane >> 5) & 1);
    const float *w = P + P_W2 + row * 32 + k0;
    return pack4(w[0], w[1], w[2], w[3]);
}

__device__ inline f32x16 bias16(const float *__restrict__ P, int off, int lane)
{
    f32x16 c;
#pragma unroll
    for (int r = 0; r < 16; ++r) c[r] = P[off + drow(r, lane)];
    return c;
}

// Per-lane operand table of a parameter block, built once per weight set
// (lbm_set_closure_weights) and staged in LDS by the fused kernel: entry k of
// lane l sits at T[k * 64 + l] (one coalesced 256-byte row per entry).
//   k 0-1    A operand of layer 1 (4 bfloat16)
//   k 2-9    A operands of layer 2, K-blocks 0-3 (4 bfloat16 each)
//   k 10-25  b1 of the 16 accumulator rows of this lane
//   k 26-41  b2 of the 16 accumulator rows
//   k 42-49  W3 of accumulator rows 2j and 2j+1 in entry 42 + j, as a
//            bfloat16 pair (operand of v_dot2_f32_bf16)
//   k 50-55  mu, k 56-61 1/sigma, k 62 b3 (lane-uniform, replicated)
constexpr int TAB_W3 = 42, TAB_MU = 50, TAB_ISG = 56, TAB_B3 = 62;
constexpr int TAB_WORDS = 63;

__device__ inline void build_table_lane(const float *__restrict__ P, int lane, uint32_t *__restrict__ T)
{
    auto put4 = [&](int k, bf16x4 v) {
        T[k * 64 + lane] = (uint32_t)(uint16_t)v.x | ((uint32_t)(uint16_t)v.y << 16);
        T[(k + 1) * 64 + lane] = (uint32_t)(uint16_t)v.z | ((uint32_t)(uint16_t)v.w << 16);
    };
    const int row = lane & 31, k0 = 4 * ((lane >> 5) & 1);
    float w[4];
    for (int t = 0; t < 4; ++t) w[t] = (k0 + t < 6) ? P[P_W1 + row * 6 + k0 + t] : 0.f;
    put4(0, pack4(w[0], w[1], w[2], w[3]));
    for (int kb = 0; kb < 4; ++kb) {
        const float *q = P + P_W2 + row * 32 + 8 * kb + k0;
        put4(2 + 2 * kb, pack4(q[0], q[1], q[2], q[3]));
    }
    for (int r = 0; r < 16; ++r) {
        T[(10 + r) * 64 + lane] = __float_as_uint(P[P_B1 + drow(r, lane)]);
        T[(26 + r) * 64 + lane] = __float_as_uint(P[P_B2 + drow(r, lane)]);
    }
    for (int j = 0; j < 8; ++j)
        T[(TAB_W3 + j) * 64 + lane] = pack2_bits(P[P_W3 + drow(2 * j, lane)], P[P_W3 + drow(2 * j + 1, lane)]);
    for (int k = 0; k < 6; ++k) {
        T[(TAB_MU + k) * 64 + lane] = __float_as_uint(P[P_MU + k]);
        T[(TAB_ISG + k) * 64 + lane] = __float_as_uint(1.f / P[P_SG + k]);
    }
    T[TAB_B3 * 64 + lane] = __float_as_uint(P[P_B3]);
}

__device__ inline bf16x4 tab4(const uint32_t *T, int k, int lane)
{
    const uint32_t lo = T[k * 64 + lane], hi = T[(k + 1) * 64 + lane];
    bf16x4 r;
    r.x = (short)(lo & 0xffffu);
    r.y = (short)(lo >> 16);
    r.z = (short)(hi & 0xffffu);
    r.w = (short)(hi >> 16);
    return r;
}

__device__ inline float tabf(const uint32_t *T, int k, int lane) { return __uint_as_float(T[k * 64 + lane]); }

// Forward pass from the operand table (fused inference).  Returns o of this
// lane's own sample.
__device__ inline float mlp_forward_table(const uint32_t *T, const float (&x)[6], int lane)
{
    float z[6], zp[6];
#pragma unroll
    for (int k = 0; k < 6; ++k) z[k] = (x[k] - tabf(T, TAB_MU + k, lane)) * tabf(T, TAB_ISG + k, lane);
#pragma unroll
    for (int k = 0; k < 6; ++k) zp[k] = __shfl_xor(z[k], 32, 64);
    const bool hi = lane >= 32;
    const bf16x4 b0 = hi ? pack4(zp[4], zp[5], 0.f, 0.f) : pack4(z[0], z[1], z[2], z[3]);
    const bf16x4 b1 = hi ? pack4(z[4], z[5], 0.f, 0.f) : pack4(zp[0], zp[1], zp[2], zp[3]);
    const bf16x4 a1 = tab4(T, 0, lane);
    f32x16 c1;
#pragma unroll
    for (int r = 0; r < 16; ++r) c1[r] = tabf(T, 10 + r, lane);
    f32x16 h0 = mfma32(a1, b0, c1);
    f32x16 h1 = mfma32(a1, b1, c1);
#pragma unroll
    for (int r = 0; r < 16; ++r) {
        h0[r] = tanh_fast(h0[r]);
        h1[r] = tanh_fast(h1[r]);
    }
    f32x16 g0, g1;
#pragma unroll
    for (int r = 0; r < 16; ++r) g0[r] = g1[r] = tabf(T, 26 + r, lane);
#pragma unroll
    for (int kb = 0; kb < 4; ++kb) {
        const bf16x4 a2 = tab4(T, 2 + 2 * kb, lane);
        g0 = mfma32(a2, pack4(h0[4 * kb], h0[4 * kb + 1], h0[4 * kb + 2], h0[4 * kb + 3]), g0);
        g1 = mfma32(a2, pack4(h1[4 * kb], h1[4 * kb + 1], h1[4 * kb + 2], h1[4 * kb + 3]), g1);
    }
    // third layer: bfloat16 activation pairs against bfloat16 weight pairs,
    // products exact, FP32 sums (v_dot2_f32_bf16)
    float s0 = 0.f, s1 = 0.f;
#pragma unroll
    for (int j = 0; j < 8; ++j) {
        const bf16x2 w = __builtin_bit_cast(bf16x2, T[(TAB_W3 + j) * 64 + lane]);
        s0 = __builtin_amdgcn_fdot2_f32_bf16(pack2(tanh_fast(g0[2 * j]), tanh_fast(g0[2 * j + 1])), w, s0, false);
        s1 = __builtin_amdgcn_fdot2_f32_bf16(pack2(tanh_fast(g1[2 * j]), tanh_fast(g1[2 * j + 1])), w, s1, false);
    }
    s0 += __shfl_xor(s0, 32, 64);
    s1 += __shfl_xor(s1, 32, 64);
    return (hi ? s1 : s0) + tabf(T, TAB_B3, lane);
}

// Forward pass.  h1_* and h2_* receive the FP32 activations of both blocks
// (accumulator layout); the return value is o for this lane's own sample.
__device__ inline float mlp_forward_wave(const float *__restrict__ P, const float (&x)[6], int lane, float (&z)[6],
                                         f32x16 &h1_0, f32x16 &h1_1, f32x16 &h2_0, f32x16 &h2_1)
{
    bf16x4 b0, b1;
    layer1_operands(P, x, lane, z, b0, b1);
    const bf16x4 a1 = layer1_weights(P, lane);
    const f32x16 c1 = bias16(P, P_B1, lane);
    h1_0 = mfma32(a1, b0, c1);
    h1_1 = mfma32(a1, b1, c1);
#pragma unroll
    for (int r = 0; r < 16; ++r) {
        h1_0[r] = tanh_f(h1_0[r]);
        h1_1[r] = tanh_f(h1_1[r]);
    }
    const f32x16 c2 = bias16(P, P_B2, lane);
    h2_0 = c2;
    h2_1 = c2;
#pragma unroll
    for (int kb = 0; kb < 4; ++kb) {
        const bf16x4 a2 = layer2_weights(P, lane, kb);
        const bf16x4 g0 = pack4(h1_0[4 * kb], h1_0[4 * kb + 1], h1_0[4 * kb + 2], h1_0[4 * kb + 3]);
        const bf16x4 g1 = pack4(h1_1[4 * kb], h1_1[4 * kb + 1], h1_1[4 * kb + 2], h1_1[4 * kb + 3]);
        h2_0 = mfma32(a2, g0, h2_0);
        h2_1 = mfma32(a2, g1, h2_1);
    }
    float s0 = 0.f, s1 = 0.f;
#pragma unroll
    for (int r = 0; r < 16; ++r) {
        h2_0[r] = tanh_f(h2_0[r]);
        h2_1[r] = tanh_f(h2_1[r]);
        const float w = bf16_round(P[P_W3 + drow(r, lane)]);
        s0 += w * bf16_round(h2_0[r]);
        s1 += w * bf16_round(h2_1[r]);
    }
    s0 += __shfl_xor(s0, 32, 64);
    s1 += __shfl_xor(s1, 32, 64);
    return (lane >= 32 ? s1 : s0) + P[P_B3];
}

__device__ inline float mlp_forward_wave(const float *__restrict__ P, const float (&x)[6], int lane)
{
    float z[6];
    f32x16 a, b, c, d;
    return mlp_forward_wave(P, x, lane, z, a, b, c, d);
}

// The six closure features of a cell from its non-equilibrium flux per
// unit density P (xx, yy, zz, xy, xz, yz): tr P, |dev P|, cbrt det dev P,
// rho - 1, tau_smag - tau (passed in as smag_excess), tau.
__device__ inline void closure_features(const float (&Pn)[6], float rho, float tau, float smag_excess,
                                        float (&x)[6])
{
    const float tr = Pn[0] + Pn[1] + Pn[2];
    const float d0 = Pn[0] - tr * (1.f / 3.f), d1 = Pn[1] - tr * (1.f / 3.f), d2 = Pn[2] - tr * (1.f / 3.f);
    const float xy = Pn[3], xz = Pn[4], yz = Pn[5];
    const float nd = __builtin_amdgcn_sqrtf(d0 * d0 + d1 * d1 + d2 * d2 + 2.f * (xy * xy + xz * xz + yz * yz));
    const float det = d0 * (d1 * d2 - yz * yz) - xy * (xy * d2 - yz * xz) + xz * (xy * yz - d1 * xz);
    x[0] = tr;
    x[1] = nd;
    // cube root as sign * 2^(log2|det| / 3) (hardware log2 and exp2; 0 -> 0)
    x[2] = copysignf(__builtin_amdgcn_exp2f(__builtin_amdgcn_logf(fabsf(det)) * (1.f / 3.f)), det);
    x[3] = rho - 1.f;
    x[4] = smag_excess;
    x[5] = tau;
}

__device__ inline bool features_in_range(const float *__restrict__ P, const float (&x)[6])
{
    bool ok = true;
#pragma unroll
    for (int k = 0; k < 6; ++k) ok &= (x[k] >= P[P_LO + k]) & (x[k] <= P[P_HI + k]);
    return ok;
}

}  // namespace lbm
