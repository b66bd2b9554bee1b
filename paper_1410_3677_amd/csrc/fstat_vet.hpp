// Kernels of the candidate-vetting network (forward, backward, Adam) and of the
// patch capture that follows the F-statistic kernel.
//
// Network: u = log(1 + 2F) - log 5 over a 256-bin patch; three "same" convolutions
// of width 7 (1 -> 32 -> 32 -> 32 channels, ReLU); flatten position-major
// (x[p*32 + c]); dense 8192 -> 128 -> 128 -> 1 (ReLU, ReLU, logit).  Activations
// are stored position-major [n][256][32].  Convolutions 2 and 3, the dense layers
// and all their gradients are products of BF16 matrices with FP32 accumulation on
// the matrix cores (v_mfma_f32_16x16x16_bf16); the first convolution (one input
// channel) and the last dense layer are plain FP32 loops.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace fstat {
namespace vet {

constexpr int L = 256;        // patch length
constexpr int C = 32;         // channels
constexpr int KW = 7;         // kernel width
constexpr int KC = KW * C;    // im2col width (224)
constexpr int H = 128;        // hidden units
constexpr int X = L * C;      // flattened conv output (8192)

// flat parameter vector offsets (order w1 b1 w2 b2 w3 b3 w4 b4 w5 b5 w6 b6)
constexpr long O_W1 = 0, O_B1 = O_W1 + C * KW, O_W2 = O_B1 + C, O_B2 = O_W2 + C * C * KW, O_W3 = O_B2 + C,
               O_B3 = O_W3 + C * C * KW, O_W4 = O_B3 + C, O_B4 = O_W4 + (long)H * X, O_W5 = O_B4 + H,
               O_B5 = O_W5 + H * H, O_W6 = O_B5 + H, O_B6 = O_W6 + H, N_PARAMS = O_B6 + 1;

typedef short v4s __attribute__((ext_vector_type(4)));
typedef short v8s __attribute__((ext_vector_type(8)));
typedef __bf16 v8bf __attribute__((ext_vector_type(8)));
typedef float v4f __attribute__((ext_vector_type(4)));

// 16 x 16 x 32 BF16 matrix-core step (gfx950): lane l (q = l / 16) holds A[l % 16][8q + j]
// and B[8q + j][l % 16], j = 0..7, and receives D[4q + i][l % 16], i = 0..3.
__device__ __forceinline__ v4f mfma32(v8s a, v8s b, v4f c) {
  return __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(v8bf, a), __builtin_bit_cast(v8bf, b), c, 0,
                                                 0, 0);
}
// eight BF16 from an 8-byte aligned LDS address
__device__ __forceinline__ v8s lds8(const uint16_t* p) {
  const v4s lo = *reinterpret_cast<const v4s*>(p), hi = *reinterpret_cast<const v4s*>(p + 4);
  return v8s{lo[0], lo[1], lo[2], lo[3], hi[0], hi[1], hi[2], hi[3]};
}

// FP32 -> BF16, round to nearest even (the hardware conversion of gfx950)
__device__ __forceinline__ uint16_t f2bf(float f) { return __builtin_bit_cast(uint16_t, (__bf16)f); }
__device__ __forceinline__ float bf2f(uint16_t h) { return __uint_as_float(((uint32_t)h) << 16); }

// C[m][n] = sum_k A(m, k) B(k, n) over k in this workgroup's K range
// A(m, k) = A[m*sam + k*sak], B(k, n) = B[k*sbk + n*sbn] (BF16), C row-major with ldc (FP32).
// Workgroup: 4 wavefronts, a 64 x 64 tile of C; each wavefront a 32 x 32 block made of
// 2 x 2 matrix-core tiles of 16 x 16, stepping K by 16.  Out-of-range elements are zero.
// Matrix-core operand layout (16x16x16): lane l holds A[l%16][4(l/16)+i], B[4(l/16)+i][l%16]
// and receives D[4(l/16)+i][l%16], i = 0..3.  With gridDim.z > 1 the K range is split and
// each split writes its partial tile to C + z * split_stride (summed by k_vet_sum_splits).
// Operands contiguous along K (stride 1) are read four elements per 8-byte load.
__device__ __forceinline__ v4s load4(const uint16_t* __restrict__ p, long base, long stride, int k, int K, bool vec) {
  v4s r;
  if (vec && k + 3 < K && (reinterpret_cast<uintptr_t>(p + base + k) & 7) == 0) {
    const ushort4 q = *reinterpret_cast<const ushort4*>(p + base + k);
    r[0] = (short)q.x;
    r[1] = (short)q.y;
    r[2] = (short)q.z;
    r[3] = (short)q.w;
  } else {
#pragma unroll
    for (int i = 0; i < 4; ++i) r[i] = (k + i < K) ? (short)p[base + (long)(k + i) * stride] : (short)0;
  }
  return r;
}

__global__ void __launch_bounds__(256) k_gemm_bf16(int M, int N, int K, const uint16_t* __restrict__ A, long sam,
                                                   long sak, const uint16_t* __restrict__ B, long sbk, long sbn,
                                                   float* __restrict__ Cm, long ldc, long split_stride, int kchunk) {
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int m0 = blockIdx.y * 64 + (w >> 1) * 32;
  const int n0 = blockIdx.x * 64 + (w & 1) * 32;
  const int r16 = lane & 15, kq = (lane >> 4) * 4;
  const int kbeg = blockIdx.z * kchunk;
  const int kend = min(K, kbeg + kchunk);
  const bool va = (sak == 1), vb = (sbk == 1);
  v4f acc[2][2];
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b) acc[a][b] = v4f{0.f, 0.f, 0.f, 0.f};
  for (int k0 = kbeg; k0 < kend; k0 += 16) {
    v4s fa[2], fb[2];
#pragma unroll
    for (int t = 0; t < 2; ++t) {
      const int m = m0 + t * 16 + r16;
      const int n = n0 + t * 16 + r16;
      fa[t] = m < M ? load4(A, (long)m * sam, sak, k0 + kq, kend, va) : v4s{0, 0, 0, 0};
      fb[t] = n < N ? load4(B, (long)n * sbn, sbk, k0 + kq, kend, vb) : v4s{0, 0, 0, 0};
    }
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
      for (int b = 0; b < 2; ++b) acc[a][b] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(fa[a], fb[b], acc[a][b], 0, 0, 0);
  }
  float* Cz = Cm + (long)blockIdx.z * split_stride;
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b)
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const int m = m0 + a * 16 + kq + i;
        const int n = n0 + b * 16 + r16;
        if (m < M && n < N) Cz[(long)m * ldc + n] = acc[a][b][i];
      }
}

// out[m][n] = sum over splits z (in order) of part[z][m][n]
__global__ void k_vet_sum_splits(const float* __restrict__ part, int splits, long count, int N, long ldc,
                                 float* __restrict__ out) {
  const long idx = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= count) return;
  const long m = idx / N, n = idx % N;
  float acc = 0.f;
  for (int z = 0; z < splits; ++z) acc += part[(long)z * count + idx];
  out[m * ldc + n] = acc;
}

// Column sums in two fixed-order stages: block (j, chunk) sums its rows of column j.
__global__ void __launch_bounds__(256) k_vet_colsum_part(const float* __restrict__ m, long rows, int cols,
                                                         long rows_per_chunk, float* __restrict__ part) {
  const int j = blockIdx.x, chunk = blockIdx.y;
  const long r0 = (long)chunk * rows_per_chunk;
  const long r1 = min(rows, r0 + rows_per_chunk);
  float acc = 0.f;
  for (long r = r0 + threadIdx.x; r < r1; r += 256) acc += m[r * cols + j];
  __shared__ float red[256];
  red[threadIdx.x] = acc;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if (threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
    __syncthreads();
  }
  if (threadIdx.x == 0) part[(long)chunk * cols + j] = red[0];
}

// u = log(1 + 2F) - log 5 per patch bin (n * L threads)
// Network input u = log(1 + 2F) - log 5, with the hardware logarithm (absolute error
// about 1e-7, far below the BF16 rounding of the layers that follow).
__device__ __forceinline__ float vet_u(float v) { return __logf(1.f + v) - 1.6094379124341003f; }

__global__ void k_vet_input(const float* __restrict__ patches, long count, float* __restrict__ u) {
  const long idx = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx < count) u[idx] = vet_u(patches[idx]);
}

// conv1 (one input channel): z1[n][p][c] = b1[c] + sum_t w1[c][t] u[n][p+t-3]; a1 = relu(z1)
// as BF16 (n * L * C threads).
__global__ void k_vet_conv1(const float* __restrict__ u, int n, const float* __restrict__ theta,
                            float* __restrict__ z1, uint16_t* __restrict__ a1b) {
  const long idx = (long)blockIdx.x * blockDim.x + threadIdx.x;  // over n * L * C
  if (idx >= (long)n * L * C) return;
  const int c = idx % C;
  const int p = (idx / C) % L;
  const long s = idx / (C * L);
  const float* us = u + s * L;
  float z = theta[O_B1 + c];
#pragma unroll
  for (int t = 0; t < KW; ++t) {
    const int q = p + t - 3;
    if (q >= 0 && q < L) z += theta[O_W1 + c * KW + t] * us[q];
  }
  z1[idx] = z;
  a1b[idx] = f2bf(z > 0.f ? z : 0.f);
}

// im2col of a position-major BF16 activation [n][L][C]:
//   col[(s*L + p)][t*C + c] = act[s][p + dir*(t-3)][c]   (zero outside [0, L))
// dir = +1 for a convolution, -1 for the transposed convolution of its input gradient.
__global__ void k_vet_im2col(const uint16_t* __restrict__ act, int n, int dir, uint16_t* __restrict__ col) {
  const long idx = (long)blockIdx.x * blockDim.x + threadIdx.x;  // over n * L * KC
  if (idx >= (long)n * L * KC) return;
  const int kk = idx % KC;
  const long row = idx / KC;
  const int p = row % L;
  const long s = row / L;
  const int t = kk / C, c = kk % C;
  const int q = p + dir * (t - 3);
  col[idx] = (q >= 0 && q < L) ? act[(s * L + q) * C + c] : (uint16_t)0;
}

// z[r][j] += bias[j]; optional relu output as BF16; z kept for the backward masks.
__global__ void k_vet_bias_relu(float* __restrict__ z, long rows, int cols, const float* __restrict__ bias,
                                uint16_t* __restrict__ outb, float* __restrict__ outf) {
  const long idx = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= rows * cols) return;
  const float v = z[idx] + bias[idx % cols];
  z[idx] = v;
  const float a = v > 0.f ? v : 0.f;
  if (outb) outb[idx] = f2bf(a);
  if (outf) outf[idx] = a;
}

// logit[s] = b6 + sum_j w6[j] a5[s][j]   (a5 = relu(z5), FP32)
__global__ void k_vet_fc3(const float* __restrict__ a5, int n, const float* __restrict__ theta,
                          float* __restrict__ logit) {
  const int s = blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= n) return;
  float v = theta[O_B6];
  for (int j = 0; j < H; ++j) v += theta[O_W6 + j] * a5[(long)s * H + j];
  logit[s] = v;
}

// Loss and the first backward step: dlogit = (sigmoid(logit) - y) / n; loss = mean BCE.
// dz5[s][j] = dlogit[s] w6[j] (z5 > 0); also dW6, db6 partial sums per block.
// Head backward over n * H threads: dlogit = (sigmoid(logit) - y) / n, its loss term, and
// dz5[s][j] = dlogit w6[j] [z5 > 0] (FP32 and BF16).
__global__ void k_vet_head_backward(const float* __restrict__ logit, const float* __restrict__ y, int n,
                                    const float* __restrict__ theta, const float* __restrict__ z5,
                                    float* __restrict__ dz5, uint16_t* __restrict__ dz5b,
                                    float* __restrict__ dlogit, float* __restrict__ loss_terms) {
  const long idx = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= (long)n * H) return;
  const int s = (int)(idx / H), j = (int)(idx % H);
  const float l = logit[s];
  const float sig = 1.f / (1.f + expf(-l));
  const float d = (sig - y[s]) / (float)n;
  if (j == 0) {
    dlogit[s] = d;
    loss_terms[s] = fmaxf(l, 0.f) - l * y[s] + log1pf(expf(-fabsf(l)));
  }
  const float g = z5[idx] > 0.f ? d * theta[O_W6 + j] : 0.f;
  dz5[idx] = g;
  dz5b[idx] = f2bf(g);
}

// dz = dh * (z > 0) in place, BF16 copy.
__global__ void k_vet_relu_mask(float* __restrict__ dh, const float* __restrict__ z, long count,
                                uint16_t* __restrict__ outb) {
  const long idx = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= count) return;
  const float g = z[idx] > 0.f ? dh[idx] : 0.f;
  dh[idx] = g;
  outb[idx] = f2bf(g);
}

// out[j] = sum over chunks (in order) of part[chunk][j]
__global__ void k_vet_colsum_final(const float* __restrict__ part, int chunks, int cols, float* __restrict__ out) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= cols) return;
  float acc = 0.f;
  for (int c = 0; c < chunks; ++c) acc += part[(long)c * cols + j];
  out[j] = acc;
}

// dW6[j] = sum_s dlogit[s] a5[s][j], db6 = sum_s dlogit[s], loss = mean of the loss terms:
// 1024 threads, eight interleaved partial sums per column added in a fixed order.
__global__ void __launch_bounds__(1024) k_vet_head_reduce(const float* __restrict__ dlogit,
                                                          const float* __restrict__ a5,
                                                          const float* __restrict__ loss_terms, int n,
                                                          float* __restrict__ grad, float* __restrict__ loss) {
  constexpr int PARTS = 1024 / H;
  __shared__ float red[PARTS][H + 2];
  const int j = threadIdx.x % H, part = threadIdx.x / H;
  float acc = 0.f, accd = 0.f, accl = 0.f;
  for (int s = part; s < n; s += PARTS) {
    const float d = dlogit[s];
    acc += d * a5[(long)s * H + j];
    if (j == 0) {
      accd += d;
      accl += loss_terms[s];
    }
  }
  red[part][j] = acc;
  if (j == 0) {
    red[part][H] = accd;
    red[part][H + 1] = accl;
  }
  __syncthreads();
  const int t = threadIdx.x;
  if (t < H + 2) {
    float sum = 0.f;
    for (int q = 0; q < PARTS; ++q) sum += red[q][t];
    if (t < H) grad[O_W6 + t] = sum;
    else if (t == H) grad[O_B6] = sum;
    else if (loss) *loss = sum / (float)n;
  }
}

// conv1 weight and bias gradients: dW1[c][t] = sum_{s,p} dz1[s][p][c] u[s][p+t-3]; db1[c].
// Block b sums rows [b rows_per_chunk, ...) with thread (c = t % 32, k = t / 32): tap k < KW
// or the bias (k = KW), writing part[b][c (KW + 1) + k]; k_vet_colsum_final adds the chunks
// in order.
__global__ void __launch_bounds__(256) k_vet_conv1_backward_part(const float* __restrict__ dz1,
                                                                 const float* __restrict__ u, long rows,
                                                                 long rows_per_chunk, float* __restrict__ part) {
  const int c = threadIdx.x % C, k = threadIdx.x / C;
  const long r0 = (long)blockIdx.x * rows_per_chunk;
  const long r1 = min(rows, r0 + rows_per_chunk);
  float acc = 0.f;
  for (long r = r0; r < r1; ++r) {
    const float g = dz1[r * C + c];
    if (k == KW) {
      acc += g;
    } else {
      const int p = r % L;
      const int q = p + k - 3;
      if (q >= 0 && q < L) acc += g * u[(r - p) + q];
    }
  }
  part[(long)blockIdx.x * (C * (KW + 1)) + c * (KW + 1) + k] = acc;
}

// Move the conv1 sums (c * (KW + 1) + t order) into the flat gradient (weights c * KW + t, biases c).
__global__ void k_vet_conv1_scatter(const float* __restrict__ sums, float* __restrict__ grad) {
  const int ct = threadIdx.x;
  if (ct >= C * (KW + 1)) return;
  const int c = ct / (KW + 1), t = ct % (KW + 1);
  if (t == KW) grad[O_B1 + c] = sums[ct];
  else grad[O_W1 + c * KW + t] = sums[ct];
}

// BF16 weight layouts for the matrix products, from the FP32 master vector:
//   wf[l][t*C + ci][co] = w_l[co][ci][t]   (forward convolution, [KC][C])
//   wt[l][t*C + co][ci] = w_l[co][ci][t]   (input-gradient convolution, [KC][C])
//   w4b[j][k] = w4[j][k], w5b[j][k] = w5[j][k]
__global__ void k_vet_prepare(const float* __restrict__ theta, uint16_t* __restrict__ wf2,
                              uint16_t* __restrict__ wt2, uint16_t* __restrict__ wf3, uint16_t* __restrict__ wt3,
                              uint16_t* __restrict__ w4b, uint16_t* __restrict__ w5b) {
  const long idx = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx < (long)H * X) w4b[idx] = f2bf(theta[O_W4 + idx]);
  if (idx < H * H) w5b[idx] = f2bf(theta[O_W5 + idx]);
  if (idx < C * C * KW) {
    const int co = idx / (C * KW), ci = (idx / KW) % C, t = idx % KW;
    wf2[(t * C + ci) * C + co] = f2bf(theta[O_W2 + idx]);
    wt2[(t * C + co) * C + ci] = f2bf(theta[O_W2 + idx]);
    wf3[(t * C + ci) * C + co] = f2bf(theta[O_W3 + idx]);
    wt3[(t * C + co) * C + ci] = f2bf(theta[O_W3 + idx]);
  }
}

// Gradient of a convolution weight from its matrix-product form dWm[t*C + ci][co]
// back to the flat layout w[co][ci][t].
__global__ void k_vet_scatter_conv_grad(const float* __restrict__ dwm, float* __restrict__ gw) {
  const int idx = blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= C * C * KW) return;
  const int co = idx / (C * KW), ci = (idx / KW) % C, t = idx % KW;
  gw[idx] = dwm[(t * C + ci) * C + co];
}

// Adam on the FP32 master vector (bias-corrected step size precomputed on the host).
__global__ void k_vet_adam(float* __restrict__ theta, const float* __restrict__ g, float* __restrict__ m1,
                           float* __restrict__ m2, long count, float step, float b1, float b2, float eps) {
  const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= count) return;
  const float gi = g[i];
  const float a = b1 * m1[i] + (1.f - b1) * gi;
  const float b = b2 * m2[i] + (1.f - b2) * gi * gi;
  m1[i] = a;
  m2[i] = b;
  theta[i] -= step * a / (sqrtf(b) + eps);
}

// Patch capture after the F kernel: for candidate slots [first, last) of the current
// launch, copy the 256-bin 2F window centred on the candidate's bin from the launch's
// spectrum buffer (template-major, bins [k_min, k_max)); bins outside that range read 0.
struct PatchArgs {
  const unsigned long long* count;   // candidates found so far (after this launch)
  const unsigned long long* first;   // value of the count before this launch
  long long capacity;                // candidate buffer entries (= patch store rows)
  int k_min, k_max;
  int t0, nfdot, sky0;               // launch: templates t0.., sky index base
};

// ------------------------------------------------------------------ inference
// Inference convolutions.  A work item is one 64-position segment of one patch, owned by
// one wavefront from input to output, so that no workgroup barrier orders its layers: the
// wavefront recomputes the three-position halos its neighbours also compute (the second
// convolution over 80 positions, the first over 80 positions, for 64 outputs), holds the
// item's activations in LDS rows of its own (position-major, 32 BF16 channels padded to
// CV_LD so that the sixteen rows one matrix-core operand spans hit distinct banks), and
// writes the third convolution's outputs straight from the accumulators to HBM.
// Workgroups of CV_WAVES wavefronts (one per compute unit: the LDS holds one) stage the
// second and third convolutions' weight fragments once and walk the items with a
// stride of the grid, prefetching the next item's input during the current one.
//
// All three convolutions run on the matrix cores.  The second and third use the training
// forward's BF16 operands and K order (D[co][p] = sum over taps t and input channels of
// W[co][k] X[p][k], K step t = tap t over all 32 channels; a lane's B operand is eight
// channels of one LDS row and its result four consecutive channels of one position).  The
// first has one input channel: its input u and weights w are split into BF16 pairs
// u = uh + ul, w = wh + wl (each to 2^-17 relative), and one 16 x 16 x 32 step covers all
// seven taps (padded to eight) times the four products wh uh, wl uh, wh ul, wl ul, which
// the accumulator sums in FP32: the FP32 convolution to about 2^-16 relative before the
// BF16 rounding of its output.
constexpr int CV_SEG = 64;              // third-convolution outputs of one item
constexpr int CV_ITEMS = L / CV_SEG;    // items per patch
constexpr int CV_WAVES = 16;            // wavefronts per workgroup
constexpr int CV_NT = CV_WAVES * 64;
constexpr int CV_ROWS = 86;             // LDS rows of an item: positions s0 - 11 .. s0 + 74
constexpr int CV_LD = 36;               // BF16 per LDS row
constexpr int CV_U = 88;                // split input entries: positions s0 - 11 .. s0 + 76
constexpr int KS = KC / 32;             // matrix-core K steps of a convolution (7: one tap each)

// Convolution weights in matrix-core fragment order: [step s][column block nb][lane][8],
// element j of lane l = w[co = 16 nb + l % 16][ci = 8 (l / 16) + j][t = s].
constexpr int WQ_ELEMS = KS * 2 * 64 * 8;

__global__ void k_vet_prepare_frag(const float* __restrict__ theta, uint16_t* __restrict__ wq2,
                                   uint16_t* __restrict__ wq3) {
  const int idx = blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= WQ_ELEMS) return;
  const int j = idx & 7, l = (idx >> 3) & 63, nb = (idx >> 9) & 1, t = idx >> 10;
  const int ci = 8 * (l >> 4) + j, co = 16 * nb + (l & 15);
  wq2[idx] = f2bf(theta[O_W2 + (co * C + ci) * KW + t]);
  wq3[idx] = f2bf(theta[O_W3 + (co * C + ci) * KW + t]);
}

typedef __bf16 v2bf __attribute__((ext_vector_type(2)));
typedef float v2f __attribute__((ext_vector_type(2)));
// two FP32 values to BF16 (round to nearest even), packed low then high
__device__ __forceinline__ uint32_t bf16_pair(float a, float b) {
  return __builtin_bit_cast(uint32_t, __builtin_convertvector((v2f){a, b}, v2bf));
}
// ReLU then BF16: as integers, negative floats (and -0) are below zero
__device__ __forceinline__ uint32_t relu_bf16_pair(float a, float b) {
  return bf16_pair(__int_as_float(max(__float_as_int(a), 0)), __int_as_float(max(__float_as_int(b), 0)));
}
__device__ __forceinline__ uint2 relu_bf16_tile(v4f d) {
  return make_uint2(relu_bf16_pair(d[0], d[1]), relu_bf16_pair(d[2], d[3]));
}
// (hi | hi << 16, lo | lo << 16) of u = hi + lo, the first convolution's B operand entry
__device__ __forceinline__ uint2 split_bf16(float u) {
  const float hi = (float)(__bf16)u;
  const uint32_t p = bf16_pair(hi, u - hi);
  return make_uint2((p & 0xffffu) * 0x10001u, (p >> 16) * 0x10001u);
}
// LDS ordering between the steps of one wavefront's item: a wavefront's LDS operations
// complete in order, so only compiler reordering must be prevented
__device__ __forceinline__ void item_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}
// zero eight LDS rows from row0 (positions outside the patch)
__device__ __forceinline__ void zero_rows8(uint16_t* buf, int row0, int lane) {
  *reinterpret_cast<uint2*>(buf + (row0 + (lane >> 3)) * CV_LD + 4 * (lane & 7)) = make_uint2(0u, 0u);
}

// u -> conv1 -> conv2 -> conv3 for items [0, 4n) (item i: patch i / 4, positions 64 (i % 4)
// .. + 63); x[s][p*32 + c] (BF16).  Every wavefront reaches the single workgroup barrier
// (after the weight staging) before its item loop.
__global__ void __launch_bounds__(CV_NT) k_vet_conv_infer(const float* __restrict__ patches, int n,
                                                        const float* __restrict__ theta,
                                                        const uint16_t* __restrict__ wq2,
                                                        const uint16_t* __restrict__ wq3, uint16_t* __restrict__ x) {
  __shared__ __align__(16) uint16_t swq[2 * WQ_ELEMS];                  // conv2 and conv3 fragments
  __shared__ __align__(16) uint16_t sbuf[CV_WAVES][CV_ROWS * CV_LD];   // activations of each wavefront's item
  __shared__ __align__(16) uint2 ssplit[CV_WAVES][CV_U];               // split input of each item
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  for (int i = tid; i < 2 * WQ_ELEMS / 8; i += CV_NT) {
    const uint4* src = reinterpret_cast<const uint4*>(i < WQ_ELEMS / 8 ? wq2 : wq3);
    reinterpret_cast<uint4*>(swq)[i] = src[i < WQ_ELEMS / 8 ? i : i - WQ_ELEMS / 8];
  }
  uint16_t* buf = sbuf[w];
  uint2* su = ssplit[w];
  // rows 0-2 and 83-85 are never written again: the zero padding below and above the
  // second convolution's 80 positions
  for (int i = lane; i < CV_ROWS * CV_LD / 4; i += 64) reinterpret_cast<uint2*>(buf)[i] = make_uint2(0u, 0u);
  __syncthreads();
  const long items = (long)n * CV_ITEMS;
  const long stride = (long)gridDim.x * CV_WAVES;
  const int r16 = lane & 15, q = lane >> 4, cb = 4 * q, ci0 = 8 * q;
  auto bias4 = [&](long o) { return v4f{theta[o + cb], theta[o + cb + 1], theta[o + cb + 2], theta[o + cb + 3]}; };
  const v4f b10 = bias4(O_B1), b11 = bias4(O_B1 + 16), b20 = bias4(O_B2), b21 = bias4(O_B2 + 16),
            b30 = bias4(O_B3), b31 = bias4(O_B3 + 16);
  // first-convolution weights as the A operand: element j of lane l is product term j % 4
  // (wh, wl, wh, wl) of tap 2 q + j / 4 (zero for the eighth tap) of channel 16 nb + l % 16
  v8s w1f[2];
#pragma unroll
  for (int nb = 0; nb < 2; ++nb) {
    uint32_t d[4];
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      const int t = 2 * q + h;
      const float wv = t < KW ? theta[O_W1 + (16 * nb + r16) * KW + t] : 0.f;
      const float whi = (float)(__bf16)wv;
      d[2 * h] = d[2 * h + 1] = bf16_pair(whi, wv - whi);
    }
    w1f[nb] = __builtin_bit_cast(v8s, make_uint4(d[0], d[1], d[2], d[3]));
  }
  const v8s* wqv = reinterpret_cast<const v8s*>(swq);
  // an item's input: lane holds positions s0 - 11 + lane and (lanes < 23) s0 + 53 + lane
  auto load_raw = [&](long it, float& a, float& b) {
    a = 0.f;
    b = 0.f;
    if (it < items) {
      const long s = it / CV_ITEMS;
      const int s0 = (int)(it % CV_ITEMS) * CV_SEG;
      const int q0 = s0 - 11 + lane, q1 = s0 + 53 + lane;
      if (q0 >= 0 && q0 < L) a = patches[s * L + q0];
      if (lane < 23 && q1 < L) b = patches[s * L + q1];
    }
  };
  long item = (long)blockIdx.x * CV_WAVES + w;
  float ra, rb;
  load_raw(item, ra, rb);
  for (; item < items; item += stride) {
    const long s = item / CV_ITEMS;
    const int s0 = (int)(item % CV_ITEMS) * CV_SEG;
    {
      const int q0 = s0 - 11 + lane, q1 = s0 + 53 + lane;
      su[lane] = split_bf16((q0 >= 0 && q0 < L) ? vet_u(ra) : 0.f);
      if (lane < CV_U - 64) su[64 + lane] = split_bf16((lane < 23 && q1 < L) ? vet_u(rb) : 0.f);
    }
    load_raw(item + stride, ra, rb);
    item_sync();
    // conv1: output rows 3 + 16 m + r16 (position s0 - 8 + 16 m + r16); the B operand of
    // lane l is input entries 16 m + r16 + 2 q and + 1 (taps 2 q, 2 q + 1)
#pragma unroll
    for (int m = 0; m < 5; ++m) {
      const uint2* e = su + 16 * m + r16 + 2 * q;
      const uint2 e0 = e[0], e1 = e[1];
      const v8s bop = __builtin_bit_cast(v8s, make_uint4(e0.x, e0.y, e1.x, e1.y));
      uint16_t* row = buf + (3 + 16 * m + r16) * CV_LD + cb;
      *reinterpret_cast<uint2*>(row) = relu_bf16_tile(mfma32(w1f[0], bop, b10));
      *reinterpret_cast<uint2*>(row + 16) = relu_bf16_tile(mfma32(w1f[1], bop, b11));
    }
    if (s0 == 0) zero_rows8(buf, 3, lane);               // positions -8 .. -1
    if (s0 + CV_SEG == L) zero_rows8(buf, 75, lane);     // positions 256 .. 263
    item_sync();
    // conv2: output rows 3 + 16 m + r16, input rows 16 m + r16 + t; written in place once
    // every input row has been read
    {
      v4f acc[5][2];
#pragma unroll
      for (int m = 0; m < 5; ++m) {
        acc[m][0] = b20;
        acc[m][1] = b21;
      }
#pragma unroll
      for (int t = 0; t < KS; ++t) {
        const v8s w0 = wqv[(t * 2 + 0) * 64 + lane];
        const v8s w1 = wqv[(t * 2 + 1) * 64 + lane];
#pragma unroll
        for (int m = 0; m < 5; ++m) {
          const v8s a = lds8(buf + (16 * m + r16 + t) * CV_LD + ci0);
          acc[m][0] = mfma32(w0, a, acc[m][0]);
          acc[m][1] = mfma32(w1, a, acc[m][1]);
        }
      }
      item_sync();
#pragma unroll
      for (int m = 0; m < 5; ++m) {
        uint16_t* row = buf + (3 + 16 * m + r16) * CV_LD + cb;
        *reinterpret_cast<uint2*>(row) = relu_bf16_tile(acc[m][0]);
        *reinterpret_cast<uint2*>(row + 16) = relu_bf16_tile(acc[m][1]);
      }
      if (s0 == 0) zero_rows8(buf, 3, lane);
      if (s0 + CV_SEG == L) zero_rows8(buf, 75, lane);
    }
    item_sync();
    // conv3: output position s0 + 16 m + r16 (row 11 + 16 m + r16), input rows
    // 8 + 16 m + r16 + t; four channels (8 bytes) per lane and tile to x
    {
      v4f acc[4][2];
#pragma unroll
      for (int m = 0; m < 4; ++m) {
        acc[m][0] = b30;
        acc[m][1] = b31;
      }
#pragma unroll
      for (int t = 0; t < KS; ++t) {
        const v8s w0 = wqv[((KS + t) * 2 + 0) * 64 + lane];
        const v8s w1 = wqv[((KS + t) * 2 + 1) * 64 + lane];
#pragma unroll
        for (int m = 0; m < 4; ++m) {
          const v8s a = lds8(buf + (8 + 16 * m + r16 + t) * CV_LD + ci0);
          acc[m][0] = mfma32(w0, a, acc[m][0]);
          acc[m][1] = mfma32(w1, a, acc[m][1]);
        }
      }
      uint16_t* xs = x + s * X + (s0 + r16) * C + cb;
#pragma unroll
      for (int m = 0; m < 4; ++m) {
        *reinterpret_cast<uint2*>(xs + 16 * m * C) = relu_bf16_tile(acc[m][0]);
        *reinterpret_cast<uint2*>(xs + 16 * m * C + 16) = relu_bf16_tile(acc[m][1]);
      }
    }
    item_sync();   // the next item's writes follow this item's reads
  }
}

// C[m][n] (split z of K) = sum_k A[m][k] B[n][k] for row-major BF16 A [M][K] and B [N][K]
// (both contiguous along K), M a multiple of 64, N a multiple of 64 and K of 64 * splits.
// Workgroup tile 64 x 64, four wavefronts of 32 x 32; K in stages of 64 through LDS
// (rows padded to 72 BF16: 16-byte aligned, and the sixteen rows of an operand fall on
// distinct banks), the next stage loaded into registers while the current one
// is multiplied.  Partial tiles of split z go to C + z * M * N (ldc = N).
constexpr int GT = 64, GK = 64, GLD = GK + 8;
__global__ void __launch_bounds__(256) k_gemm_nt_lds(int M, int N, int K, const uint16_t* __restrict__ A,
                                                     const uint16_t* __restrict__ B, float* __restrict__ Cm,
                                                     int kchunk) {
  __shared__ __align__(16) uint16_t sA[GT * GLD];
  __shared__ __align__(16) uint16_t sB[GT * GLD];
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const int m0 = blockIdx.y * GT, n0 = blockIdx.x * GT;
  const int kbeg = blockIdx.z * kchunk, kend = kbeg + kchunk;
  // each thread moves 2 x 16 bytes of A and of B per stage: row r = tid / 4, 16-element group (tid % 4) * 16
  const int lr = tid >> 2, lc = (tid & 3) * 16;
  const uint16_t* ga = A + (long)(m0 + lr) * K + lc;
  const uint16_t* gb = B + (long)(n0 + lr) * K + lc;
  uint4 ra0, ra1, rb0, rb1;
  auto gload = [&](int k0) {
    ra0 = *reinterpret_cast<const uint4*>(ga + k0);
    ra1 = *reinterpret_cast<const uint4*>(ga + k0 + 8);
    rb0 = *reinterpret_cast<const uint4*>(gb + k0);
    rb1 = *reinterpret_cast<const uint4*>(gb + k0 + 8);
  };
  auto sstore = [&]() {
    uint4* pa = reinterpret_cast<uint4*>(sA + lr * GLD + lc);
    uint4* pb = reinterpret_cast<uint4*>(sB + lr * GLD + lc);
    pa[0] = ra0;
    pa[1] = ra1;
    pb[0] = rb0;
    pb[1] = rb1;
  };
  v4f acc[2][2];
#pragma unroll
  for (int a = 0; a < 2; ++a) acc[a][0] = acc[a][1] = v4f{0.f, 0.f, 0.f, 0.f};
  const int wm = (w >> 1) * 32, wn = (w & 1) * 32;
  const int r16 = lane & 15, kq = 4 * (lane >> 4), k8 = 8 * (lane >> 4);
  gload(kbeg);
  for (int k0 = kbeg; k0 < kend; k0 += GK) {
    __syncthreads();  // the previous stage has been read
    sstore();
    __syncthreads();
    if (k0 + GK < kend) gload(k0 + GK);
#pragma unroll
    for (int kk = 0; kk < GK; kk += 32) {
      v8s fa[2], fb[2];
#pragma unroll
      for (int t = 0; t < 2; ++t) {
        fa[t] = *reinterpret_cast<const v8s*>(sA + (wm + 16 * t + r16) * GLD + kk + k8);
        fb[t] = *reinterpret_cast<const v8s*>(sB + (wn + 16 * t + r16) * GLD + kk + k8);
      }
#pragma unroll
      for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b) acc[a][b] = mfma32(fa[a], fb[b], acc[a][b]);
    }
  }
  float* Cz = Cm + (long)blockIdx.z * M * N;
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b)
#pragma unroll
      for (int i = 0; i < 4; ++i)
        Cz[(long)(m0 + wm + 16 * a + kq + i) * N + n0 + wn + 16 * b + r16] = acc[a][b][i];
}

// The scoring call's 8192 -> 128 product: C[m][n] (split z of K) = sum_k A[m][k] B[n][k] for
// row-major BF16 A [M][K] and B [128][K], M a multiple of 128, K of GW_K * splits.  A
// workgroup covers 128 rows and all 128 columns, so that each row of A is read once and B
// once per 128 rows; eight wavefronts of 32 x 64 (2 x 4 matrix-core tiles each; four
// wavefronts of 64 x 64 took 9% longer, fewer loads being in flight per compute unit), K
// in stages of GW_K through LDS (rows padded by 8 BF16), the next stage loaded into
// registers while the current one is multiplied (arrays of native vector types: the
// compiler had put an array of HIP's uint4 structs in scratch memory).  Partial tiles of
// split z go to C + z * M * 128.
constexpr int GW_M = 128, GW_K = 64, GW_LD = GW_K + 8, GW_NT = 512;
__global__ void __launch_bounds__(GW_NT) k_gemm_nt_wide(int M, int K, const uint16_t* __restrict__ A,
                                                        const uint16_t* __restrict__ B, float* __restrict__ Cm,
                                                        int kchunk) {
  typedef unsigned int u4v __attribute__((ext_vector_type(4)));
  constexpr int PER = GW_M * GW_K / 8 / GW_NT;   // 16-byte loads per thread per operand and stage (2)
  constexpr int TPR = GW_K / 8;                  // threads per row
  constexpr int RPP = GW_NT / TPR;               // rows per pass
  constexpr int TA = 2, TB = 4;                  // a wavefront's 16 x 16 tiles: 32 rows x 64 columns
  __shared__ __align__(16) uint16_t sA[GW_M * GW_LD];
  __shared__ __align__(16) uint16_t sB[H * GW_LD];
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const int m0 = blockIdx.y * GW_M;
  const int kbeg = blockIdx.z * kchunk, kend = kbeg + kchunk;
  const int lr = tid / TPR, lc = (tid % TPR) * 8;
  u4v ra[PER], rb[PER];
  auto gload = [&](int k0) {
#pragma unroll
    for (int i = 0; i < PER; ++i) {
      ra[i] = *reinterpret_cast<const u4v*>(A + (long)(m0 + lr + RPP * i) * K + k0 + lc);
      rb[i] = *reinterpret_cast<const u4v*>(B + (long)(lr + RPP * i) * K + k0 + lc);
    }
  };
  v4f acc[TA][TB];
#pragma unroll
  for (int a = 0; a < TA; ++a)
#pragma unroll
    for (int c = 0; c < TB; ++c) acc[a][c] = v4f{0.f, 0.f, 0.f, 0.f};
  const int wm = (w >> 1) * 16 * TA, wn = (w & 1) * 16 * TB;
  const int r16 = lane & 15, kq = 4 * (lane >> 4), k8 = 8 * (lane >> 4);
  gload(kbeg);
  for (int k0 = kbeg; k0 < kend; k0 += GW_K) {
    __syncthreads();  // the previous stage has been read
#pragma unroll
    for (int i = 0; i < PER; ++i) {
      *reinterpret_cast<u4v*>(sA + (lr + RPP * i) * GW_LD + lc) = ra[i];
      *reinterpret_cast<u4v*>(sB + (lr + RPP * i) * GW_LD + lc) = rb[i];
    }
    __syncthreads();
    if (k0 + GW_K < kend) gload(k0 + GW_K);
#pragma unroll
    for (int kk = 0; kk < GW_K; kk += 32) {
      v8s fa[TA], fb[TB];
#pragma unroll
      for (int t = 0; t < TA; ++t) fa[t] = *reinterpret_cast<const v8s*>(sA + (wm + 16 * t + r16) * GW_LD + kk + k8);
#pragma unroll
      for (int t = 0; t < TB; ++t) fb[t] = *reinterpret_cast<const v8s*>(sB + (wn + 16 * t + r16) * GW_LD + kk + k8);
#pragma unroll
      for (int a = 0; a < TA; ++a)
#pragma unroll
        for (int c = 0; c < TB; ++c) acc[a][c] = mfma32(fa[a], fb[c], acc[a][c]);
    }
  }
  float* Cz = Cm + (long)blockIdx.z * M * H;
#pragma unroll
  for (int a = 0; a < TA; ++a)
#pragma unroll
    for (int c = 0; c < TB; ++c)
#pragma unroll
      for (int i = 0; i < 4; ++i) Cz[(long)(m0 + wm + 16 * a + kq + i) * H + wn + 16 * c + r16] = acc[a][c][i];
}

// The dense layers after the 8192 -> 128 product, for HD_NP patches per workgroup: the
// split-K partial sums added in split order, bias, ReLU and BF16 rounding (a4), the
// 128 -> 128 layer on the matrix cores (BF16 a4 and w5, FP32 accumulation), bias and ReLU
// (a5), and the 128 -> 1 head (logit).  With `cand`, the score sigmoid(logit) of patch i is
// also stored in entry i (the patch store is indexed by candidate slot).  One launch
// instead of five.  Wavefront w forms the output columns 32 w .. 32 w + 31 of both
// sixteen-patch row blocks: lane l's A operand is eight consecutive a4 of one patch (an
// LDS row, padded to HD_LD so that the sixteen rows fall on distinct banks), its B operand
// eight consecutive weights of one output's w5 row (16 bytes from global memory).
constexpr int HD_NP = 32, HD_LD = H + 8;
template <int SPLITS>
__global__ void __launch_bounds__(256) k_vet_head_infer(const float* __restrict__ part, long count, int n,
                                                        const float* __restrict__ theta,
                                                        const uint16_t* __restrict__ w5b, float* __restrict__ logit,
                                                        CandEntry* __restrict__ cand) {
  __shared__ __align__(16) uint16_t sa4[HD_NP * HD_LD];   // a4 of the workgroup's patches (BF16)
  __shared__ float sp[HD_NP][H + 1];                       // w6[o] a5[p][o]
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const int r0 = blockIdx.x * HD_NP;
  const float* b4 = theta + O_B4;
  // the partial sums of rows r0 .. r0 + HD_NP - 1 (all within the product's padded rows),
  // every load of a thread issued before the sums
#pragma unroll
  for (int q = 0; q < HD_NP * H / 256; ++q) {
    const int i = tid + 256 * q, pp = i / H, k = i % H, row = r0 + pp;
    float acc = 0.f;
#pragma unroll
    for (int z = 0; z < SPLITS; ++z) acc += part[(long)z * count + (long)row * H + k];
    const float a = acc + b4[k];
    sa4[pp * HD_LD + k] = row < n ? f2bf(a > 0.f ? a : 0.f) : (uint16_t)0;
  }
  __syncthreads();
  v4f acc[2][2];
#pragma unroll
  for (int a = 0; a < 2; ++a) acc[a][0] = acc[a][1] = v4f{0.f, 0.f, 0.f, 0.f};
  const int r16 = lane & 15, k8 = 8 * (lane >> 4);
#pragma unroll
  for (int k0 = 0; k0 < H; k0 += 32) {
    v8s fa[2], fb[2];
#pragma unroll
    for (int t = 0; t < 2; ++t) {
      fa[t] = *reinterpret_cast<const v8s*>(sa4 + (16 * t + r16) * HD_LD + k0 + k8);
      fb[t] = *reinterpret_cast<const v8s*>(w5b + (long)(32 * w + 16 * t + r16) * H + k0 + k8);
    }
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
      for (int b = 0; b < 2; ++b) acc[a][b] = mfma32(fa[a], fb[b], acc[a][b]);
  }
#pragma unroll
  for (int b = 0; b < 2; ++b) {
    const int o = 32 * w + 16 * b + r16;
    const float b5 = theta[O_B5 + o], w6 = theta[O_W6 + o];
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const float z = acc[a][b][i] + b5;
        sp[16 * a + 4 * (lane >> 4) + i][o] = w6 * (z > 0.f ? z : 0.f);
      }
  }
  __syncthreads();
  if (tid < HD_NP && r0 + tid < n) {
    float v = theta[O_B6];
    for (int j = 0; j < H; ++j) v += sp[tid][j];
    logit[r0 + tid] = v;
    if (cand) cand[r0 + tid].pad = __float_as_int(1.f / (1.f + expf(-v)));
  }
}

}  // namespace vet
}  // namespace fstat
