// Learned initial guess for the inversion: a 5 -> 64 -> 64 -> 64 -> 2 SiLU
// network.  Training runs in FP32 (layer-wise kernels, gradients reduced over
// the batch in a fixed order, Adam); deployment runs in BF16 on the matrix
// cores (v_mfma_f32_16x16x16_bf16, FP32 accumulation), one wavefront per 64
// cells, and writes mu0 = exp(-y1) for the Newton solve.  Included once, by
// grmhd.hip.
#pragma once
#include "dev.h"

namespace grmhd {

constexpr int MLP_IN = 5, MLP_H = 64, MLP_OUT = 2;
// FP32 parameter layout: W1[64][5] b1[64] W2[64][64] b2[64] W3[64][64] b3[64] W4[2][64] b4[2]
constexpr int MLP_OFF_W1 = 0, MLP_OFF_B1 = MLP_OFF_W1 + MLP_H * MLP_IN;
constexpr int MLP_OFF_W2 = MLP_OFF_B1 + MLP_H, MLP_OFF_B2 = MLP_OFF_W2 + MLP_H * MLP_H;
constexpr int MLP_OFF_W3 = MLP_OFF_B2 + MLP_H, MLP_OFF_B3 = MLP_OFF_W3 + MLP_H * MLP_H;
constexpr int MLP_OFF_W4 = MLP_OFF_B3 + MLP_H, MLP_OFF_B4 = MLP_OFF_W4 + MLP_OUT * MLP_H;
constexpr int MLP_NPARAM = MLP_OFF_B4 + MLP_OUT;   // 8834

__device__ __forceinline__ float silu_f(float z) { return z / (1.0f + expf(-z)); }
__device__ __forceinline__ float dsilu_f(float z)
{
  const float s = 1.0f / (1.0f + expf(-z));
  return s * (1.0f + z * (1.0f - s));
}

// ------------------------------------------------------------- training (FP32)

// Z[s][o] = b[o] + sum_i H[s][i] W[o][i];  Hout = act ? silu(Z) : Z
__global__ __launch_bounds__(256) void k_dense_fwd(const float *__restrict__ H, int nin,
                                                   const float *__restrict__ W,
                                                   const float *__restrict__ b, int nout,
                                                   float *__restrict__ Z, float *__restrict__ Hout,
                                                   int batch, int act)
{
  const int e = blockIdx.x * 256 + threadIdx.x;
  if (e >= batch * nout) return;
  const int s = e / nout, o = e % nout;
  float z = b[o];
  for (int i = 0; i < nin; ++i) z = fmaf(H[s * nin + i], W[o * nin + i], z);
  Z[e] = z;
  Hout[e] = act ? silu_f(z) : z;
}

// delta = 2 (out - Y) / batch ; per-block partial sums of the squared error
__global__ __launch_bounds__(256) void k_mse(const float *__restrict__ out,
                                             const float *__restrict__ Y, int batch,
                                             float *__restrict__ delta, float *__restrict__ part)
{
  __shared__ float sh[256];
  const int s = blockIdx.x * 256 + threadIdx.x;
  float acc = 0.0f;
  if (s < batch) {
    for (int k = 0; k < MLP_OUT; ++k) {
      const float d = out[s * MLP_OUT + k] - Y[s * MLP_OUT + k];
      delta[s * MLP_OUT + k] = 2.0f * d / (float)batch;
      acc += d * d / (float)batch;
    }
  }
  sh[threadIdx.x] = acc;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (threadIdx.x < w) sh[threadIdx.x] += sh[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) part[blockIdx.x] = sh[0];
}

// dprev[s][i] = (sum_o delta[s][o] W[o][i]) * silu'(Zprev[s][i])
__global__ __launch_bounds__(256) void k_dense_bwd_data(const float *__restrict__ delta, int nout,
                                                        const float *__restrict__ W, int nin,
                                                        const float *__restrict__ Zprev,
                                                        float *__restrict__ dprev, int batch)
{
  const int e = blockIdx.x * 256 + threadIdx.x;
  if (e >= batch * nin) return;
  const int s = e / nin, i = e % nin;
  float g = 0.0f;
  for (int o = 0; o < nout; ++o) g = fmaf(delta[s * nout + o], W[o * nin + i], g);
  dprev[e] = g * dsilu_f(Zprev[e]);
}

// gW[o][i] = sum_s delta[s][o] H[s][i], gb[o] = sum_s delta[s][o]; the batch
// sum runs in a fixed order (deterministic)
__global__ __launch_bounds__(256) void k_dense_bwd_weight(const float *__restrict__ delta,
                                                          int nout, const float *__restrict__ H,
                                                          int nin, int batch,
                                                          float *__restrict__ gW,
                                                          float *__restrict__ gb)
{
  const int e = blockIdx.x * 256 + threadIdx.x;
  if (e >= nout * (nin + 1)) return;
  const int o = e / (nin + 1), i = e % (nin + 1);
  float acc = 0.0f;
  if (i < nin) {
    for (int s = 0; s < batch; ++s) acc = fmaf(delta[s * nout + o], H[s * nin + i], acc);
    gW[o * nin + i] = acc;
  } else {
    for (int s = 0; s < batch; ++s) acc += delta[s * nout + o];
    gb[o] = acc;
  }
}

__global__ __launch_bounds__(256) void k_sum(const float *__restrict__ part, int n, float *out)
{
  __shared__ float sh[256];
  float a = 0.0f;
  for (int k = threadIdx.x; k < n; k += 256) a += part[k];
  sh[threadIdx.x] = a;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (threadIdx.x < w) sh[threadIdx.x] += sh[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) *out = sh[0];
}

// Adam (Kingma & Ba), bias-corrected step t >= 1
__global__ __launch_bounds__(256) void k_adam(float *__restrict__ p, const float *__restrict__ g,
                                              float *__restrict__ m, float *__restrict__ v, int n,
                                              float lr, float b1, float b2, float eps, int t)
{
  const int e = blockIdx.x * 256 + threadIdx.x;
  if (e >= n) return;
  const float gg = g[e];
  const float mm = b1 * m[e] + (1.0f - b1) * gg;
  const float vv = b2 * v[e] + (1.0f - b2) * gg * gg;
  m[e] = mm;
  v[e] = vv;
  const float mh = mm / (1.0f - powf(b1, (float)t));
  const float vh = vv / (1.0f - powf(b2, (float)t));
  p[e] -= lr * mh / (sqrtf(vh) + eps);
}

// ------------------------------------------------------ deployment (BF16 MFMA)

typedef short bf16x4 __attribute__((ext_vector_type(4)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ unsigned short f2bf(float f)
{
  // round to nearest even
  unsigned int u = __float_as_uint(f);
  u += 0x7FFFu + ((u >> 16) & 1u);
  return (unsigned short)(u >> 16);
}

// BF16 weights in the workspace: W1p[64][16] (inputs zero-padded to 16),
// W2[64][64], W3[64][64], W4p[16][64] (outputs zero-padded to 16); FP32 biases
// b1[64] b2[64] b3[64] b4[2]; feature mean[5], 1/std[5].
constexpr int MLPB_W1 = 0, MLPB_W2 = MLPB_W1 + 64 * 16, MLPB_W3 = MLPB_W2 + 64 * 64,
              MLPB_W4 = MLPB_W3 + 64 * 64, MLPB_N = MLPB_W4 + 16 * 64;   // bf16 count
constexpr int MLPF_B1 = 0, MLPF_B2 = 64, MLPF_B3 = 128, MLPF_B4 = 192, MLPF_MEAN = 196,
              MLPF_ISTD = 201, MLPF_N = 208;                             // fp32 count

struct MlpDev {
  const unsigned short *w;   // MLPB_N bf16
  const float *f;            // MLPF_N fp32
};

// One 16x16x16 MFMA: D(16x16) += A(16 rows x 16 k) B(16 k x 16 cols).
// Operand lane layout (wave64): A: row = lane % 16, k = 4 (lane / 16) .. +3;
// B: col = lane % 16, k = 4 (lane / 16) .. +3; D: col = lane % 16,
// rows 4 (lane / 16) .. +3.
__device__ __forceinline__ f32x4 mfma16(bf16x4 a, bf16x4 b, f32x4 c)
{
  return __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, b, c, 0, 0, 0);
}

// SiLU for inference, z / (1 + e^-z) with the hardware exp2 and reciprocal:
// the activations are rounded to BF16 right after, far above their error.
__device__ __forceinline__ float silu_hw(float z)
{
  return z * __builtin_amdgcn_rcpf(1.0f + __builtin_amdgcn_exp2f(-1.4426950408889634f * z));
}

// Four floats to BF16 (round to nearest even) with gfx950's packed convert,
// two values per instruction.
typedef __bf16 bf16v2 __attribute__((ext_vector_type(2)));
typedef float f32v2 __attribute__((ext_vector_type(2)));
struct Bf16Pair { bf16v2 lo, hi; };
__device__ __forceinline__ bf16x4 pack_bf16(float a, float b, float c, float d)
{
  const Bf16Pair p = {__builtin_convertvector(f32v2{a, b}, bf16v2),
                      __builtin_convertvector(f32v2{c, d}, bf16v2)};
  return __builtin_bit_cast(bf16x4, p);
}

// One dense layer over the 64 rows (cells) of a wavefront, computed
// transposed, O^T = W H^T, so that the MFMA result tile is already the next
// layer's B operand: with r = lane % 16 and q = lane / 16,
//   H[kt][mt] (lane) = H(row 16 mt + r, columns 16 kt + 4 q .. + 3)   (B operand)
//   A operand = W(row 16 nt + r, columns 16 kt + 4 q .. + 3)           (8-byte load)
//   D[mt] of tile nt (lane) = O(row 16 mt + r, columns 16 nt + 4 q .. + 3)
// W [N][K] bf16 row-major (global, L2-resident).  Hidden layers (ACT): the
// bias enters as the accumulator's initial value and SiLU + BF16 rounding
// are applied tile by tile (16 output columns at a time, so only 16
// accumulators are live) into Hout[nt][mt].  Output layer: the raw tiles in
// Dout[nt][mt], bias left to the caller.
template <int K, int N, bool ACT>
__device__ __forceinline__ void dense_t(const bf16x4 (&H)[K / 16][4], const unsigned short *W,
                                        const float *bias, bf16x4 (&Hout)[N / 16][4],
                                        f32x4 (&Dout)[N / 16][4], int lane)
{
  const int r = lane % 16, q = lane / 16;
#pragma unroll
  for (int nt = 0; nt < N / 16; ++nt) {
    f32x4 init = {0.0f, 0.0f, 0.0f, 0.0f};
    if constexpr (ACT)
      init = f32x4{bias[16 * nt + 4 * q], bias[16 * nt + 4 * q + 1], bias[16 * nt + 4 * q + 2],
                   bias[16 * nt + 4 * q + 3]};
    f32x4 D[4] = {init, init, init, init};
#pragma unroll
    for (int kt = 0; kt < K / 16; ++kt) {
      const bf16x4 a = *(const bf16x4 *)(W + (16 * nt + r) * K + 16 * kt + 4 * q);
#pragma unroll
      for (int mt = 0; mt < 4; ++mt) D[mt] = mfma16(a, H[kt][mt], D[mt]);
    }
#pragma unroll
    for (int mt = 0; mt < 4; ++mt) {
      if constexpr (ACT)
        Hout[nt][mt] = pack_bf16(silu_hw(D[mt][0]), silu_hw(D[mt][1]), silu_hw(D[mt][2]),
                                 silu_hw(D[mt][3]));
      else
        Dout[nt][mt] = D[mt];
    }
  }
}

// Features of one cell (undensitized conserved state on the cell's metric):
// log10 D, log(1 + S^2/D^2), log(1 + tau/D), log(1 + B^2/D), log(1 + (S.B)^2/D^3),
// standardised with the training set's mean and standard deviation.  The
// ratios are formed in FP64 and the logarithms taken in FP32 with the
// hardware log2: the features are rounded to BF16 next.
__device__ __forceinline__ void mlp_features(double D, double S2, double tau, double BB, double SB,
                                             const float *mean, const float *istd, float x[5])
{
  const double iD = 1.0 / D;
  auto ratio = [](double v) { return (float)fmin(fmax(v, 0.0), 1e30); };
  constexpr float ln2 = 0.69314718055994531f, lg2 = 0.30102999566398120f;
  const float raw[5] = {__builtin_amdgcn_logf((float)fmax(D, 1e-37)) * lg2,
                        __builtin_amdgcn_logf(1.0f + ratio(S2 * iD * iD)) * ln2,
                        __builtin_amdgcn_logf(1.0f + ratio(tau * iD)) * ln2,
                        __builtin_amdgcn_logf(1.0f + ratio(BB * iD)) * ln2,
                        __builtin_amdgcn_logf(1.0f + ratio(SB * SB * iD * iD * iD)) * ln2};
#pragma unroll
  for (int k = 0; k < 5; ++k) x[k] = (raw[k] - mean[k]) * istd[k];
}

// Wavefront-level inference for 64 feature rows already in LDS (X [64][16]
// bf16, written by the 64 lanes before a barrier).  The activations stay in
// registers; the two outputs of every row go to outf [64][2] (LDS), visible
// to the whole wavefront when this returns.
__device__ __forceinline__ void mlp_wave(const MlpDev &m, const unsigned short *X, float *outf,
                                         int lane)
{
  const int r = lane % 16, q = lane / 16;
  bf16x4 h0[1][4], h1[4][4], h2[4][4], unused[1][4];
  f32x4 none[4][4], o[1][4];
#pragma unroll
  for (int mt = 0; mt < 4; ++mt) h0[0][mt] = *(const bf16x4 *)(X + (16 * mt + r) * 16 + 4 * q);
  dense_t<16, 64, true>(h0, m.w + MLPB_W1, m.f + MLPF_B1, h1, none, lane);
  dense_t<64, 64, true>(h1, m.w + MLPB_W2, m.f + MLPF_B2, h2, none, lane);
  dense_t<64, 64, true>(h2, m.w + MLPB_W3, m.f + MLPF_B3, h1, none, lane);
  dense_t<64, 16, false>(h1, m.w + MLPB_W4, nullptr, unused, o, lane);   // W4 padded to 16 rows
  if (q == 0) {          // lanes 0..15 hold outputs 0..3 of rows 16 mt + r
#pragma unroll
    for (int mt = 0; mt < 4; ++mt) {
      outf[(16 * mt + r) * MLP_OUT + 0] = o[0][mt][0] + m.f[MLPF_B4];
      outf[(16 * mt + r) * MLP_OUT + 1] = o[0][mt][1] + m.f[MLPF_B4 + 1];
    }
  }
  __syncthreads();
}

// Inference on a plain feature array (tests): X [n][5] raw features -> Y [n][2]
__global__ __launch_bounds__(64) void k_mlp_infer(MlpDev m, const float *__restrict__ Xin,
                                                  float *__restrict__ Y, int n)
{
  __shared__ __align__(16) unsigned short X[64 * 16];
  __shared__ float out[64 * MLP_OUT];
  const int lane = threadIdx.x;
  const int s = blockIdx.x * 64 + lane;
#pragma unroll
  for (int k = 0; k < 16; ++k) {
    float v = 0.0f;
    if (k < 5 && s < n) v = (Xin[s * 5 + k] - m.f[MLPF_MEAN + k]) * m.f[MLPF_ISTD + k];
    X[lane * 16 + k] = f2bf(v);
  }
  __syncthreads();
  mlp_wave(m, X, out, lane);
  if (s < n) {
    Y[s * 2 + 0] = out[lane * 2 + 0];
    Y[s * 2 + 1] = out[lane * 2 + 1];
  }
}

// FP32 parameters -> padded BF16 weights + FP32 biases and feature scaling
__global__ __launch_bounds__(256) void k_mlp_pack(const float *__restrict__ p,
                                                  const float *__restrict__ mean,
                                                  const float *__restrict__ stdv,
                                                  unsigned short *__restrict__ w,
                                                  float *__restrict__ f)
{
  const int e = blockIdx.x * 256 + threadIdx.x;
  if (e < 64 * 16) {
    const int o = e / 16, i = e % 16;
    w[MLPB_W1 + e] = i < MLP_IN ? f2bf(p[MLP_OFF_W1 + o * MLP_IN + i]) : 0;
  }
  if (e < 64 * 64) {
    w[MLPB_W2 + e] = f2bf(p[MLP_OFF_W2 + e]);
    w[MLPB_W3 + e] = f2bf(p[MLP_OFF_W3 + e]);
  }
  if (e < 16 * 64) {
    const int o = e / 64;
    w[MLPB_W4 + e] = o < MLP_OUT ? f2bf(p[MLP_OFF_W4 + e]) : 0;
  }
  if (e < 64) {
    f[MLPF_B1 + e] = p[MLP_OFF_B1 + e];
    f[MLPF_B2 + e] = p[MLP_OFF_B2 + e];
    f[MLPF_B3 + e] = p[MLP_OFF_B3 + e];
  }
  if (e < MLP_OUT) f[MLPF_B4 + e] = p[MLP_OFF_B4 + e];
  if (e < MLP_IN) {
    f[MLPF_MEAN + e] = mean[e];
    f[MLPF_ISTD + e] = 1.0f / stdv[e];
  }
}

}  // namespace grmhd
