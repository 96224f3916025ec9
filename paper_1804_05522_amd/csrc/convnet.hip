// Learned warm start for the 2D per-step Sylvester solve (not part of the
// paper): a four-layer convolutional network predicts u_{k+1} from u_k,
//   pred = u + net(u),  net = conv4 o relu o conv3 o relu o conv2 o relu o conv1,
// every conv 3x3 with zero padding (zero = the absorbing boundary of the
// fractional problem), channels 1 -> 32 -> 32 -> 32 -> 1.  Loss: mean squared
// error over the interior of the image (a margin of `margin` pixels is left
// out, so crops of a larger field are not judged where their zero padding is
// artificial).  Optimiser: Adam with FP32 master weights.
//
// Layout: images are row-major n x H x W (FP32); hidden activations are
// pixel-major with the 32 channels contiguous (NHWC), stored in FP32 (test
// mode) or BF16 (production).  Weights w[o][c][tap], tap = 3 (dp + 1) + (dq + 1)
// for the neighbour (i + dp, j + dq).
//
// Kernels:
//   k_net_conv1         1 -> 32, ReLU (one thread per pixel)
//   k_net_conv32_mfma   32 -> 32, ReLU, BF16 MFMA 32x32x8 with FP32
//                       accumulation: one wave computes 32 pixels x 32 outputs
//                       as an implicit GEMM over K = 9 taps x 32 channels
//   k_net_conv32        32 -> 32 on FMAs (FP32 activations, and the
//                       transposed convolution of the backward pass)
//   k_net_conv4         32 -> 1 plus the residual connection
//   k_net_loss          loss partials and dL/dpred
//   k_net_bwd4          dL/da3 from dL/dpred (ReLU mask applied)
//   k_net_wgrad32/4/1   weight and bias gradient partials per pixel chunk
//   k_net_reduce        deterministic sum of the partials (FP64)
//   k_net_adam          Adam step
#include "internal.hpp"

namespace hfde {

constexpr int kNetC = 32;
constexpr int kNW1 = 0, kNB1 = kNW1 + kNetC * 9, kNW2 = kNB1 + kNetC, kNB2 = kNW2 + kNetC * kNetC * 9;
constexpr int kNW3 = kNB2 + kNetC, kNB3 = kNW3 + kNetC * kNetC * 9, kNW4 = kNB3 + kNetC, kNB4 = kNW4 + kNetC * 9;
constexpr int kNetParams = kNB4 + 1;       // 19105
constexpr int kNetChunk = 1024;            // pixels per weight-gradient partial

__device__ inline float to_f(float v) { return v; }
__device__ inline float to_f(bf16 v) { return __uint_as_float(uint32_t(v.v) << 16); }
template <typename T>
__device__ inline T from_f(float f);
template <>
__device__ inline float from_f<float>(float f) { return f; }
template <>
__device__ inline bf16 from_f<bf16>(float f) {
  uint32_t u = __float_as_uint(f);
  uint32_t rounding = 0x7FFFu + ((u >> 16) & 1u);       // round to nearest even
  if ((u & 0x7F800000u) == 0x7F800000u) rounding = 0;   // keep inf / nan
  bf16 b;
  b.v = uint16_t((u + rounding) >> 16);
  return b;
}

struct NetImg {
  int n, H, W;
  __host__ __device__ inline int64_t pixels() const { return int64_t(n) * H * W; }
  // neighbour of pixel p at offset (s*dp, s*dq), or -1 outside the image
  __device__ inline int64_t nb(int64_t p, int dp, int dq) const {
    const int64_t img = p / (int64_t(H) * W);
    const int rem = int(p - img * H * W);
    const int i = rem / W + dp, j = rem % W + dq;
    if (i < 0 || i >= H || j < 0 || j >= W) return -1;
    return (img * H + i) * W + j;
  }
};

// ---------------------------------------------------------------- forward
template <typename TA>
__global__ void __launch_bounds__(256) k_net_conv1(NetImg g, const float* u, const float* par, TA* a1) {
  __shared__ float w[kNetC * 9], bb[kNetC];
  for (int e = threadIdx.x; e < kNetC * 9; e += 256) w[e] = par[kNW1 + e];
  if (threadIdx.x < kNetC) bb[threadIdx.x] = par[kNB1 + threadIdx.x];
  __syncthreads();
  const int64_t p = int64_t(blockIdx.x) * 256 + threadIdx.x;
  if (p >= g.pixels()) return;
  float x[9];
#pragma unroll
  for (int tap = 0; tap < 9; ++tap) {
    const int64_t q = g.nb(p, tap / 3 - 1, tap % 3 - 1);
    x[tap] = q >= 0 ? u[q] : 0.0f;
  }
#pragma unroll
  for (int o = 0; o < kNetC; ++o) {
    float z = bb[o];
#pragma unroll
    for (int tap = 0; tap < 9; ++tap) z += w[o * 9 + tap] * x[tap];
    a1[p * kNetC + o] = from_f<TA>(fmaxf(z, 0.0f));
  }
}

// out[p][j] = bias[j] + sum_tap sum_i Wt[tap][i][j] in[nb(p, s*off(tap))][i]
// forward (s = +1): Wt[tap][i][j] = w[j][i][tap], ReLU, output TO = activation type;
// backward (s = -1): Wt[tap][i][j] = w[i][j][tap] (transposed), no bias, output
// multiplied by (mask[p][j] > 0) (the ReLU derivative of the layer below).
template <typename TI, typename TO, typename TM, bool BACKWARD>
__global__ void __launch_bounds__(256) k_net_conv32(NetImg g, const TI* in, const float* par, int woff, int boff,
                                                     const TM* mask, TO* out) {
  __shared__ float wt[9 * kNetC * kNetC];
  __shared__ float bb[kNetC];
  for (int e = threadIdx.x; e < 9 * kNetC * kNetC; e += 256) {
    const int tap = e / (kNetC * kNetC), r = e % (kNetC * kNetC), i = r / kNetC, j = r % kNetC;
    wt[e] = BACKWARD ? par[woff + (i * kNetC + j) * 9 + tap] : par[woff + (j * kNetC + i) * 9 + tap];
  }
  if (threadIdx.x < kNetC) bb[threadIdx.x] = BACKWARD ? 0.0f : par[boff + threadIdx.x];
  __syncthreads();
  const int64_t p = int64_t(blockIdx.x) * 256 + threadIdx.x;
  if (p >= g.pixels()) return;
  float acc[kNetC];
#pragma unroll
  for (int j = 0; j < kNetC; ++j) acc[j] = bb[j];
  for (int tap = 0; tap < 9; ++tap) {
    const int sgn = BACKWARD ? -1 : 1;
    const int64_t q = g.nb(p, sgn * (tap / 3 - 1), sgn * (tap % 3 - 1));
    if (q < 0) continue;
    const TI* src = in + q * kNetC;
    float x[kNetC];
#pragma unroll
    for (int i = 0; i < kNetC; ++i) x[i] = to_f(src[i]);
    const float* wk = wt + tap * kNetC * kNetC;
#pragma unroll 4
    for (int i = 0; i < kNetC; ++i) {
#pragma unroll
      for (int j = 0; j < kNetC; ++j) acc[j] += wk[i * kNetC + j] * x[i];
    }
  }
#pragma unroll
  for (int j = 0; j < kNetC; ++j) {
    float v = acc[j];
    if (BACKWARD) v = to_f(mask[p * kNetC + j]) > 0.0f ? v : 0.0f;
    else v = fmaxf(v, 0.0f);
    out[p * kNetC + j] = from_f<TO>(v);
  }
}

// 32 -> 32 with ReLU on BF16 matrix cores: per wave a tile of 32 consecutive
// pixels x 32 output channels, C = A B with A[p][k] = act(nb(p, tap))[c] and
// B[k][o] = w[o][c][tap], k = 32 tap + c, in 36 steps of K = 8.  Operand
// layout of v_mfma_f32_32x32x8bf16_1k: lane l holds A[l % 32][4 (l / 32) + 0..3]
// and B[4 (l / 32) + 0..3][l % 32]; the result element (row, col) sits in lane
// col + 32 ((row / 4) % 2), register (row % 4) + 4 (row / 8).
typedef short net_v4s __attribute__((ext_vector_type(4)));
typedef float net_v16f __attribute__((ext_vector_type(16)));

__global__ void __launch_bounds__(256) k_net_conv32_mfma(NetImg g, const bf16* in, const float* par, int woff, int boff,
                                                          bf16* out) {
  __shared__ bf16 wb[kNetC * 9 * kNetC];   // [o][k], k = 32 tap + c
  __shared__ float bb[kNetC];
  for (int e = threadIdx.x; e < kNetC * 9 * kNetC; e += 256) {
    const int o = e / (9 * kNetC), k = e % (9 * kNetC), tap = k / kNetC, c = k % kNetC;
    wb[e] = from_f<bf16>(par[woff + (o * kNetC + c) * 9 + tap]);
  }
  if (threadIdx.x < kNetC) bb[threadIdx.x] = par[boff + threadIdx.x];
  __syncthreads();
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int64_t p0 = (int64_t(blockIdx.x) * 4 + wave) * 32;
  const int64_t P = g.pixels();
  if (p0 >= P) return;
  const int64_t prow = p0 + (lane & 31);
  const int kh = (lane >> 5) * 4;
  net_v16f acc;
#pragma unroll
  for (int r = 0; r < 16; ++r) acc[r] = 0.0f;
  for (int tap = 0; tap < 9; ++tap) {
    const int64_t q = prow < P ? g.nb(prow, tap / 3 - 1, tap % 3 - 1) : -1;
#pragma unroll
    for (int cb = 0; cb < 4; ++cb) {
      const int c0 = cb * 8 + kh;
      net_v4s a, b;
      if (q >= 0) {
        const uint64_t v = *reinterpret_cast<const uint64_t*>(in + q * kNetC + c0);
        a[0] = short(v & 0xFFFF);
        a[1] = short((v >> 16) & 0xFFFF);
        a[2] = short((v >> 32) & 0xFFFF);
        a[3] = short((v >> 48) & 0xFFFF);
      } else {
        a[0] = a[1] = a[2] = a[3] = 0;
      }
      const bf16* wrow = wb + (lane & 31) * (9 * kNetC) + tap * kNetC + c0;
#pragma unroll
      for (int e = 0; e < 4; ++e) b[e] = short(wrow[e].v);
      acc = __builtin_amdgcn_mfma_f32_32x32x8bf16_1k(a, b, acc, 0, 0, 0);
    }
  }
  const int col = lane & 31;
#pragma unroll
  for (int r = 0; r < 16; ++r) {
    const int row = (r / 4) * 8 + (lane >> 5) * 4 + (r % 4);
    const int64_t p = p0 + row;
    if (p < P) out[p * kNetC + col] = from_f<bf16>(fmaxf(acc[r] + bb[col], 0.0f));
  }
}

template <typename TA>
__global__ void __launch_bounds__(256) k_net_conv4(NetImg g, const TA* a3, const float* u, const float* par,
                                                   float* pred) {
  __shared__ float w[kNetC * 9];
  for (int e = threadIdx.x; e < kNetC * 9; e += 256) w[e] = par[kNW4 + e];
  __syncthreads();
  const int64_t p = int64_t(blockIdx.x) * 256 + threadIdx.x;
  if (p >= g.pixels()) return;
  float z = par[kNB4];
  for (int tap = 0; tap < 9; ++tap) {
    const int64_t q = g.nb(p, tap / 3 - 1, tap % 3 - 1);
    if (q < 0) continue;
#pragma unroll
    for (int c = 0; c < kNetC; ++c) z += w[c * 9 + tap] * to_f(a3[q * kNetC + c]);
  }
  pred[p] = u[p] + z;
}

// ---------------------------------------------------------------- backward
// dL/dpred over the interior (margin excluded), and per-block loss partials.
__global__ void __launch_bounds__(256) k_net_loss(NetImg g, const float* pred, const float* target, int margin,
                                                  double inv_count, float* gpred, double* lpart) {
  __shared__ double red[256];
  const int64_t p = int64_t(blockIdx.x) * 256 + threadIdx.x;
  double l = 0.0;
  if (p < g.pixels()) {
    const int rem = int(p % (int64_t(g.H) * g.W));
    const int i = rem / g.W, j = rem % g.W;
    const bool in = i >= margin && i < g.H - margin && j >= margin && j < g.W - margin;
    const double d = double(pred[p]) - double(target[p]);
    gpred[p] = in ? float(2.0 * d * inv_count) : 0.0f;
    l = in ? d * d * inv_count : 0.0;
  }
  red[threadIdx.x] = l;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if (threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
    __syncthreads();
  }
  if (threadIdx.x == 0) lpart[blockIdx.x] = red[0];
}

// dL/da3[q][c] = (a3[q][c] > 0) sum_tap w4[c][tap] gpred[nb(q, -off(tap))]
template <typename TA>
__global__ void __launch_bounds__(256) k_net_bwd4(NetImg g, const float* gpred, const TA* a3, const float* par,
                                                  float* g3) {
  __shared__ float w[kNetC * 9];
  for (int e = threadIdx.x; e < kNetC * 9; e += 256) w[e] = par[kNW4 + e];
  __syncthreads();
  const int64_t q = int64_t(blockIdx.x) * 256 + threadIdx.x;
  if (q >= g.pixels()) return;
  float gv[9];
#pragma unroll
  for (int tap = 0; tap < 9; ++tap) {
    const int64_t p = g.nb(q, -(tap / 3 - 1), -(tap % 3 - 1));
    gv[tap] = p >= 0 ? gpred[p] : 0.0f;
  }
#pragma unroll
  for (int c = 0; c < kNetC; ++c) {
    float s = 0.0f;
#pragma unroll
    for (int tap = 0; tap < 9; ++tap) s += w[c * 9 + tap] * gv[tap];
    g3[q * kNetC + c] = to_f(a3[q * kNetC + c]) > 0.0f ? s : 0.0f;
  }
}

// Weight / bias gradient partials of a 32 -> 32 layer over one chunk of
// pixels: part[chunk][(o * 32 + c) * 9 + tap] = sum_p gout[p][o] in[nb(p, off(tap))][c],
// part[chunk][9216 + o] = sum_p gout[p][o].  Thread t owns output channel
// o = t % 32 and input channels 4 (t / 32) .. +3, all nine taps.
template <typename TI>
__global__ void __launch_bounds__(256) k_net_wgrad32(NetImg g, const float* gout, const TI* in, float* part) {
  constexpr int kT = 32;                       // pixels staged per tile
  __shared__ float gs[kT * kNetC];
  __shared__ float xs[kT * 9 * kNetC];
  const int t = threadIdx.x, o = t % kNetC, cg = (t / kNetC) * 4;
  float acc[36];
  float bacc = 0.0f;
#pragma unroll
  for (int k = 0; k < 36; ++k) acc[k] = 0.0f;
  const int64_t P = g.pixels();
  const int64_t c0 = int64_t(blockIdx.x) * kNetChunk;
  for (int64_t t0 = c0; t0 < min<int64_t>(P, c0 + kNetChunk); t0 += kT) {
    __syncthreads();
    for (int e = t; e < kT * kNetC; e += 256) {
      const int64_t p = t0 + e / kNetC;
      gs[e] = p < P ? gout[p * kNetC + e % kNetC] : 0.0f;
    }
    for (int e = t; e < kT * 9 * kNetC; e += 256) {
      const int pl = e / (9 * kNetC), r = e % (9 * kNetC), tap = r / kNetC, c = r % kNetC;
      const int64_t p = t0 + pl;
      const int64_t q = p < P ? g.nb(p, tap / 3 - 1, tap % 3 - 1) : -1;
      xs[e] = q >= 0 ? to_f(in[q * kNetC + c]) : 0.0f;
    }
    __syncthreads();
    for (int pl = 0; pl < kT; ++pl) {
      const float gv = gs[pl * kNetC + o];
      bacc += gv;
#pragma unroll
      for (int tap = 0; tap < 9; ++tap)
#pragma unroll
        for (int k = 0; k < 4; ++k) acc[tap * 4 + k] += gv * xs[pl * 9 * kNetC + tap * kNetC + cg + k];
    }
  }
  float* out = part + int64_t(blockIdx.x) * (kNetC * kNetC * 9 + kNetC);
#pragma unroll
  for (int tap = 0; tap < 9; ++tap)
#pragma unroll
    for (int k = 0; k < 4; ++k) out[(o * kNetC + cg + k) * 9 + tap] = acc[tap * 4 + k];
  if (t < kNetC) out[kNetC * kNetC * 9 + o] = bacc;
}

// Layer 4 (32 -> 1) and layer 1 (1 -> 32) weight partials: 288 + bias values.
// layer 4: part[c * 9 + tap] = sum_p gpred[p] a3[nb(p, off)][c], part[288] = sum gpred
// layer 1: part[o * 9 + tap] = sum_p g1[p][o] u[nb(p, off)],     part[288 + o] = sum g1[.][o]
template <typename TA, bool FIRST>
__global__ void __launch_bounds__(288) k_net_wgrad_edge(NetImg g, const float* gout, const TA* a3, const float* u,
                                                        float* part) {
  const int t = threadIdx.x;                   // t = 9 * ch + tap
  const int ch = t / 9, tap = t % 9;
  const int64_t P = g.pixels();
  const int64_t c0 = int64_t(blockIdx.x) * kNetChunk;
  float acc = 0.0f, bacc = 0.0f;
  for (int64_t p = c0; p < min<int64_t>(P, c0 + kNetChunk); ++p) {
    const int64_t q = g.nb(p, tap / 3 - 1, tap % 3 - 1);
    if (FIRST) {
      const float gv = gout[p * kNetC + ch];
      acc += q >= 0 ? gv * u[q] : 0.0f;
      bacc += gv;
    } else {
      const float gv = gout[p];
      acc += q >= 0 ? gv * to_f(a3[q * kNetC + ch]) : 0.0f;
      bacc += gv;
    }
  }
  const int stride = FIRST ? (kNetC * 9 + kNetC) : (kNetC * 9 + 1);
  float* out = part + int64_t(blockIdx.x) * stride;
  out[t] = acc;
  if (FIRST) {
    if (tap == 0) out[kNetC * 9 + ch] = bacc;
  } else if (t == 0) {
    out[kNetC * 9] = bacc;
  }
}

// grad[dst + e] = sum over chunks of part[chunk * stride + e], in chunk order.
__global__ void k_net_reduce(const float* part, int chunks, int stride, float* grad, int dst) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= stride) return;
  double s = 0.0;
  for (int k = 0; k < chunks; ++k) s += double(part[int64_t(k) * stride + e]);
  grad[dst + e] = float(s);
}

__global__ void k_net_adam(float* par, const float* grad, float* m, float* v, int count, float lr, float b1, float b2,
                           float eps, float c1, float c2) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= count) return;
  const float gv = grad[e];
  const float mm = b1 * m[e] + (1.0f - b1) * gv;
  const float vv = b2 * v[e] + (1.0f - b2) * gv * gv;
  m[e] = mm;
  v[e] = vv;
  par[e] -= lr * (mm / c1) / (sqrtf(vv / c2) + eps);
}

// Dense field out[i + j nx] = sum_r Z[i][r] W[j][r] (FP32) from X = Z W^T.
__global__ void k_lr_to_dense(int64_t nx, int64_t ny, int r, const double* Z, int64_t ldz, const double* Wf,
                              int64_t ldw, float* out) {
  const int64_t e = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (e >= nx * ny) return;
  const int64_t i = e % nx, j = e / nx;
  double s = 0.0;
  for (int k = 0; k < r; ++k) s += Z[i + k * ldz] * Wf[j + k * ldw];
  out[e] = float(s);
}

}  // namespace hfde
