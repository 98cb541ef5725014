// Learned warm start: per-orbital network (forward on FP16 MFMA with FP32
// accumulation), its loss head, backward pass and Adam, the feature build and
// the predicted moment correction.
//
// Layout. FP32 master parameters in the ABI's flat order; FP16 copies of the
// weights transposed to [out][in] (rows padded to a multiple of 32 inputs and
// 32 outputs with zeros) so that each MFMA lane loads its eight k-consecutive
// operands as one 16-byte vector. Activations of the last forward pass are
// kept per network: X16 [rows][32] (features rounded to half, zero padded),
// Z1, Z2 [rows][256] float32 (pre-activations) and A1, A2 [rows][256] half.
//
// Forward: one workgroup = 4 waves x 16 rows, 64 output columns; lane l of a
// wave supplies In[row0 + l % 16][k0 + 8 (l / 16) + t] and
// Wt[col + l % 16][k0 + 8 (l / 16) + t] to v_mfma_f32_16x16x32_f16, whose
// accumulator register r holds D[4 (l / 16) + r][l % 16].
// Backward: float32 GEMMs tiled 64 x 64 through LDS, split over the
// reduction dimension into fixed-order partial sums (no atomics), the GELU
// derivative fused into the epilogue of the activation gradients.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <memory>
#include <vector>

#include "agf2_internal.h"

namespace {

typedef _Float16 h16;
typedef h16 h16x8 __attribute__((ext_vector_type(8)));
typedef float f4 __attribute__((ext_vector_type(4)));

constexpr int NF = AGF2_MLP_FEATURES, NFP = 32, NH = AGF2_MLP_HIDDEN, NO = AGF2_MLP_OUTPUTS,
              NOP = 32, NMOM = 4;
constexpr long OW1 = 0, OB1 = OW1 + (long)NF * NH, OW2 = OB1 + NH, OB2 = OW2 + (long)NH * NH,
               OW3 = OB2 + NH, OB3 = OW3 + (long)NH * NO, NPARAM = OB3 + NO;
static_assert(NPARAM == AGF2_MLP_NPARAM, "parameter count");
// FP16 transposed weights: W1t [NH][NFP], W2t [NH][NH], W3t [NOP][NH]
constexpr long H1 = 0, H2 = H1 + (long)NH * NFP, H3 = H2 + (long)NH * NH,
               NHALF = H3 + (long)NOP * NH;

__device__ __forceinline__ float gelu(float z) {
  return 0.5f * z * (1.0f + erff(z * 0.70710678118654752f));
}
__device__ __forceinline__ float gelu_grad(float z) {
  return 0.5f * (1.0f + erff(z * 0.70710678118654752f)) +
         z * expf(-0.5f * z * z) * 0.39894228040143268f;
}

// X [rows][12] float -> X16 [rows][32] half (columns 12..31 zero)
__global__ void pack_features(int rows, const float* __restrict__ X, h16* __restrict__ X16) {
  const long n = (long)rows * NFP;
  for (long i = blockIdx.x * (long)blockDim.x + threadIdx.x; i < n;
       i += (long)gridDim.x * blockDim.x) {
    const long r = i / NFP;
    const int c = (int)(i % NFP);
    X16[i] = c < NF ? (h16)X[r * NF + c] : (h16)0.0f;
  }
}

// Z = In . W + b (and A = half(gelu(Z)) for hidden layers); K % 32 == 0.
template <bool ACT>
__global__ __launch_bounds__(256) void linear_fwd(const h16* __restrict__ in, int ldi, int rows,
                                                  int K, const h16* __restrict__ wt,
                                                  const float* __restrict__ bias, int nout,
                                                  float* __restrict__ Z, int ldz,
                                                  h16* __restrict__ A, int lda) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int row0 = blockIdx.x * 64 + wave * 16;
  const int col0 = blockIdx.y * 64;
  const int fr = lane & 15, fk = (lane >> 4) * 8;
  f4 acc[4];
#pragma unroll
  for (int j = 0; j < 4; ++j) acc[j] = f4{0.f, 0.f, 0.f, 0.f};
  const int arow = row0 + fr;
  const bool rin = arow < rows;
  for (int k0 = 0; k0 < K; k0 += 32) {
    h16x8 a;
    if (rin) a = *reinterpret_cast<const h16x8*>(in + (long)arow * ldi + k0 + fk);
    else a = h16x8{0, 0, 0, 0, 0, 0, 0, 0};
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      if (col0 + 16 * j >= nout) break;   // uniform over the wave
      const h16x8 b = *reinterpret_cast<const h16x8*>(wt + (long)(col0 + 16 * j + fr) * K + k0 + fk);
      acc[j] = __builtin_amdgcn_mfma_f32_16x16x32_f16(a, b, acc[j], 0, 0, 0);
    }
  }
#pragma unroll
  for (int j = 0; j < 4; ++j)
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int row = row0 + 4 * (lane >> 4) + r;
      const int col = col0 + 16 * j + fr;
      if (row >= rows || col >= nout) continue;
      const float z = acc[j][r] + bias[col];
      Z[(long)row * ldz + col] = z;
      if (ACT) A[(long)row * lda + col] = (h16)gelu(z);
    }
}

template <class T> __device__ __forceinline__ float ld(const T* p) { return (float)*p; }

// Part_s[m][n] = sum_{k in split s} A(m, k) B(k, n), A(m, k) = A[m sAm + k sAk],
// B(k, n) = B[k sBk + n sBn]; with G, the result is multiplied by gelu'(G[m][n])
// (single split only).
template <class TA, class TB>
__global__ __launch_bounds__(256) void gemm_f32(int M, int N, int K, int kchunk,
                                                const TA* __restrict__ A, long sAm, long sAk,
                                                const TB* __restrict__ B, long sBk, long sBn,
                                                float* __restrict__ C, long ldc, long sCs,
                                                const float* __restrict__ G, long ldg) {
  __shared__ float As[16][65], Bs[16][65];
  const int tid = threadIdx.x, tx = tid & 15, ty = tid >> 4;
  const int m0 = blockIdx.x * 64, n0 = blockIdx.y * 64, s = blockIdx.z;
  const int k0 = s * kchunk, k1 = min(K, k0 + kchunk);
  float acc[4][4] = {};
  for (int kb = k0; kb < k1; kb += 16) {
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int idx = tid + 256 * q;
      const int mm = idx & 63, kk = idx >> 6;
      const int m = m0 + mm, k = kb + kk;
      As[kk][mm] = (m < M && k < k1) ? ld(A + (long)m * sAm + (long)k * sAk) : 0.f;
      const int n = n0 + mm;
      Bs[kk][mm] = (n < N && k < k1) ? ld(B + (long)k * sBk + (long)n * sBn) : 0.f;
    }
    __syncthreads();
#pragma unroll
    for (int kk = 0; kk < 16; ++kk) {
      float a[4], b[4];
#pragma unroll
      for (int i = 0; i < 4; ++i) a[i] = As[kk][ty * 4 + i];
#pragma unroll
      for (int j = 0; j < 4; ++j) b[j] = Bs[kk][tx * 4 + j];
#pragma unroll
      for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) acc[i][j] = fmaf(a[i], b[j], acc[i][j]);
    }
    __syncthreads();
  }
  float* Cs = C + (long)s * sCs;
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int m = m0 + ty * 4 + i, n = n0 + tx * 4 + j;
      if (m >= M || n >= N) continue;
      float v = acc[i][j];
      if (G) v *= gelu_grad(G[(long)m * ldg + n]);
      Cs[(long)m * ldc + n] = v;
    }
}

// out[i] = sum_s part[s][i] (fixed order)
__global__ void sum_parts(const float* __restrict__ part, long stride, int nsplit, long n,
                          float* __restrict__ out) {
  for (long i = blockIdx.x * (long)blockDim.x + threadIdx.x; i < n;
       i += (long)gridDim.x * blockDim.x) {
    float acc = 0.f;
    for (int s = 0; s < nsplit; ++s) acc += part[s * stride + i];
    out[i] = acc;
  }
}

// out[n] = sum_m D[m][n] (fixed order)
__global__ void col_sums(int M, int N, const float* __restrict__ D, float* __restrict__ out) {
  const int n = blockIdx.x * blockDim.x + threadIdx.x;
  if (n >= N) return;
  float acc = 0.f;
  for (int m = 0; m < M; ++m) acc += D[(long)m * N + n];
  out[n] = acc;
}

// One workgroup per (orbital x, moment n): row x of the residual
// R = diag(r_n) + sum_m (c_nm(x) + c_nm(y)) U_m / s_m - (mconv - m0)_n / s_n,
// its squared norm, and the gradient dY[x][5n .. 5n+4].
__global__ __launch_bounds__(256) void head_loss(int N, const float* __restrict__ Y,
                                                 const double* __restrict__ m0,
                                                 const double* __restrict__ mc,
                                                 const double* __restrict__ scale,
                                                 float* __restrict__ dY,
                                                 double* __restrict__ lpart) {
  const int x = blockIdx.x, n = blockIdx.y, tid = threadIdx.x;
  const long nn = (long)N * N;
  double cx[NMOM], inv_s[NMOM];
#pragma unroll
  for (int m = 0; m < NMOM; ++m) {
    cx[m] = Y[(long)x * NO + 5 * n + 1 + m];
    inv_s[m] = 1.0 / scale[m];
  }
  const double rx = Y[(long)x * NO + 5 * n];
  double l = 0.0, g[NMOM] = {0.0, 0.0, 0.0, 0.0};
  __shared__ double red[1 + NMOM][256];
  __shared__ double dpxx;
  for (int y = tid; y < N; y += 256) {
    const long xy = (long)x * N + y;
    double p = (x == y) ? rx : 0.0, ut[NMOM];
#pragma unroll
    for (int m = 0; m < NMOM; ++m) {
      ut[m] = m0[m * nn + xy] * inv_s[m];
      p += (cx[m] + (double)Y[(long)y * NO + 5 * n + 1 + m]) * ut[m];
    }
    const double t = (mc[n * nn + xy] - m0[n * nn + xy]) * inv_s[n];
    const double r = p - t;
    l += r * r;
    const double dp = 2.0 * r / N;
    if (x == y) dpxx = dp;
#pragma unroll
    for (int m = 0; m < NMOM; ++m) g[m] += dp * ut[m];
  }
  red[0][tid] = l;
#pragma unroll
  for (int m = 0; m < NMOM; ++m) red[1 + m][tid] = g[m];
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (tid < w)
#pragma unroll
      for (int q = 0; q < 1 + NMOM; ++q) red[q][tid] += red[q][tid + w];
    __syncthreads();
  }
  if (tid == 0) {
    lpart[(long)n * N + x] = red[0][0] / N;
    dY[(long)x * NO + 5 * n] = (float)dpxx;
#pragma unroll
    for (int m = 0; m < NMOM; ++m) dY[(long)x * NO + 5 * n + 1 + m] = (float)(2.0 * red[1 + m][0]);
  }
}

__global__ void add_sum(long n, const double* __restrict__ part, double* __restrict__ acc) {
  if (blockIdx.x != 0 || threadIdx.x != 0) return;
  double s = 0.0;
  for (long i = 0; i < n; ++i) s += part[i];
  *acc += s;
}

// Features and scales of one system (one workgroup).
__global__ __launch_bounds__(256) void features_kernel(int N, int nocc, const double* __restrict__ e,
                                                       const double* __restrict__ m0,
                                                       float* __restrict__ X,
                                                       double* __restrict__ scale) {
  __shared__ double red[NMOM][256];
  __shared__ double s[NMOM];
  const int tid = threadIdx.x;
  double part[NMOM] = {0.0, 0.0, 0.0, 0.0};
  for (int x = tid; x < N; x += 256)
#pragma unroll
    for (int n = 0; n < NMOM; ++n) part[n] += fabs(m0[((long)n * N + x) * N + x]);
#pragma unroll
  for (int n = 0; n < NMOM; ++n) red[n][tid] = part[n];
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (tid < w)
#pragma unroll
      for (int n = 0; n < NMOM; ++n) red[n][tid] += red[n][tid + w];
    __syncthreads();
  }
  if (tid < NMOM) {
    s[tid] = fmax(red[tid][0] / N, 1e-30);
    scale[tid] = s[tid];
  }
  __syncthreads();
  const double homo = e[nocc - 1], lumo = e[nocc];
  const double mu0 = 0.5 * (homo + lumo), gap = lumo - homo;
  for (int x = tid; x < N; x += 256) {
    float* f = X + (long)x * NF;
    f[0] = (float)e[x];
    f[1] = (float)(e[x] - mu0);
    f[2] = (float)gap;
    f[3] = x < nocc ? 1.0f : -1.0f;
#pragma unroll
    for (int n = 0; n < NMOM; ++n) f[4 + n] = (float)(m0[((long)n * N + x) * N + x] / s[n]);
    f[8] = (float)log(s[1] / s[0]);
    f[9] = (float)log(s[2] / s[0]);
    f[10] = (float)log(s[3] / s[2]);
    f[11] = (float)((e[x] - mu0) / gap);
  }
}

// dm[n][x][y] = s_n (delta_xy r_n(x) + sum_m (c_nm(x) + c_nm(y)) m0[m][x][y] / s_m), with
// m0[m][x][y] taken as the mean of the (x, y) and (y, x) entries so that dm is
// exactly symmetric
__global__ void correction_kernel(int N, const float* __restrict__ Y,
                                  const double* __restrict__ m0,
                                  const double* __restrict__ scale, double* __restrict__ dm) {
  const long nn = (long)N * N, total = NMOM * nn;
  for (long i = blockIdx.x * (long)blockDim.x + threadIdx.x; i < total;
       i += (long)gridDim.x * blockDim.x) {
    const int n = (int)(i / nn);
    const long r = i % nn;
    const int x = (int)(r / N), y = (int)(r % N);
    const float* yx = Y + (long)x * NO + 5 * n;
    const float* yy = Y + (long)y * NO + 5 * n;
    double p = (x == y) ? (double)yx[0] : 0.0;
#pragma unroll
    for (int m = 0; m < NMOM; ++m) {
      const double u = 0.5 * (m0[m * nn + r] + m0[m * nn + (long)y * N + x]);
      p += ((double)yx[1 + m] + (double)yy[1 + m]) * u / scale[m];
    }
    dm[i] = scale[n] * p;
  }
}

__global__ void adam_kernel(long n, float* __restrict__ theta, const float* __restrict__ g,
                            float* __restrict__ m, float* __restrict__ v, float lr, float b1,
                            float b2, float eps, float c1, float c2) {
  for (long i = blockIdx.x * (long)blockDim.x + threadIdx.x; i < n;
       i += (long)gridDim.x * blockDim.x) {
    const float gi = g[i];
    const float mi = b1 * m[i] + (1.0f - b1) * gi;
    const float vi = b2 * v[i] + (1.0f - b2) * gi * gi;
    m[i] = mi;
    v[i] = vi;
    theta[i] -= lr * (mi * c1) / (sqrtf(vi * c2) + eps);
  }
}

// FP16 transposed copies of W1, W2, W3 (padding entries untouched: zero).
__global__ void refresh_half(const float* __restrict__ theta, h16* __restrict__ w16) {
  const long n = (long)NF * NH + (long)NH * NH + (long)NH * NO;
  for (long i = blockIdx.x * (long)blockDim.x + threadIdx.x; i < n;
       i += (long)gridDim.x * blockDim.x) {
    if (i < (long)NF * NH) {
      const int in = (int)(i / NH), out = (int)(i % NH);
      w16[H1 + (long)out * NFP + in] = (h16)theta[OW1 + i];
    } else if (i < (long)NF * NH + (long)NH * NH) {
      const long j = i - (long)NF * NH;
      const int in = (int)(j / NH), out = (int)(j % NH);
      w16[H2 + (long)out * NH + in] = (h16)theta[OW2 + j];
    } else {
      const long j = i - (long)NF * NH - (long)NH * NH;
      const int in = (int)(j / NO), out = (int)(j % NO);
      w16[H3 + (long)out * NH + in] = (h16)theta[OW3 + j];
    }
  }
}

__global__ void fill_f32(long n, float* __restrict__ p) {
  for (long i = blockIdx.x * (long)blockDim.x + threadIdx.x; i < n;
       i += (long)gridDim.x * blockDim.x)
    p[i] = 0.0f;
}
__global__ void fill_h16(long n, h16* __restrict__ p) {
  for (long i = blockIdx.x * (long)blockDim.x + threadIdx.x; i < n;
       i += (long)gridDim.x * blockDim.x)
    p[i] = (h16)0.0f;
}

inline unsigned grid1(long n) { return (unsigned)std::max<long>(1, std::min<long>((n + 255) / 256, 2048)); }

}  // namespace

struct agf2_mlp_s {
  int device = 0;
  agf2::DevBuf params;   // theta, grad, m, v (float) then the half weights
  agf2::DevBuf act;      // activations of the last forward
  agf2::DevBuf bwd;      // backward scratch: dZ2, dZ1
  agf2::DevBuf split;    // split-K partial sums of the weight gradients
  float *theta = nullptr, *grad = nullptr, *m = nullptr, *v = nullptr;
  h16* w16 = nullptr;
  long t = 0;            // Adam steps taken
  int rows = -1;         // rows of the kept activations
  h16 *X16 = nullptr, *A1 = nullptr, *A2 = nullptr;
  float *Z1 = nullptr, *Z2 = nullptr;
};

namespace agf2 {
namespace {

agf2_mlp_s& net_of(agf2_mlp_t p, const Handle& h) {
  if (!p) throw Error{AGF2_ERR_ARG, "NULL network"};
  if (p->device != h.device) throw Error{AGF2_ERR_ARG, "network lives on another device"};
  return *p;
}

void ensure_act(agf2_mlp_s& net, int rows) {
  const long r = std::max(rows, 1);
  const long bytes = r * NFP * 2 + 2 * r * NH * 4 + 2 * r * NH * 2 + 4 * 256;
  char* base = static_cast<char*>(net.act.get(bytes));
  auto take = [&](long b) {
    char* p = base;
    base += (b + 255) / 256 * 256;
    return p;
  };
  net.X16 = reinterpret_cast<h16*>(take(r * NFP * 2));
  net.Z1 = reinterpret_cast<float*>(take(r * NH * 4));
  net.Z2 = reinterpret_cast<float*>(take(r * NH * 4));
  net.A1 = reinterpret_cast<h16*>(take(r * NH * 2));
  net.A2 = reinterpret_cast<h16*>(take(r * NH * 2));
}

void forward(agf2_mlp_s& net, int rows, const float* X, float* Y, hipStream_t st) {
  ensure_act(net, rows);
  hipLaunchKernelGGL(pack_features, dim3(grid1((long)rows * NFP)), dim3(256), 0, st, rows, X,
                     net.X16);
  AGF2_CHECK_LAUNCH();
  const unsigned gr = (unsigned)((rows + 63) / 64);
  hipLaunchKernelGGL(linear_fwd<true>, dim3(gr, NH / 64), dim3(256), 0, st, net.X16, NFP, rows,
                     NFP, net.w16 + H1, net.theta + OB1, NH, net.Z1, NH, net.A1, NH);
  AGF2_CHECK_LAUNCH();
  hipLaunchKernelGGL(linear_fwd<true>, dim3(gr, NH / 64), dim3(256), 0, st, net.A1, NH, rows,
                     NH, net.w16 + H2, net.theta + OB2, NH, net.Z2, NH, net.A2, NH);
  AGF2_CHECK_LAUNCH();
  hipLaunchKernelGGL(linear_fwd<false>, dim3(gr, 1), dim3(256), 0, st, net.A2, NH, rows, NH,
                     net.w16 + H3, net.theta + OB3, NO, Y, NO, static_cast<h16*>(nullptr), 0);
  AGF2_CHECK_LAUNCH();
  net.rows = rows;
}

// C = op(A) op(B) (with the GELU-derivative epilogue when G is set), split
// over K into fixed-order partial sums when K is long.
template <class TA, class TB>
void gemm(int M, int N, int K, const TA* A, long sAm, long sAk, const TB* B, long sBk, long sBn,
          float* C, long ldc, const float* G, long ldg, DevBuf& scratch, hipStream_t st) {
  const int nsplit = G ? 1 : std::max(1, std::min(64, K / 512));
  int kchunk = (K + nsplit - 1) / nsplit;
  kchunk = (kchunk + 15) / 16 * 16;
  const int ns = std::max(1, (K + kchunk - 1) / kchunk);
  const dim3 grid((unsigned)((M + 63) / 64), (unsigned)((N + 63) / 64), (unsigned)ns);
  if (ns == 1) {
    hipLaunchKernelGGL((gemm_f32<TA, TB>), grid, dim3(256), 0, st, M, N, K, kchunk, A, sAm, sAk,
                       B, sBk, sBn, C, ldc, 0L, G, ldg);
    AGF2_CHECK_LAUNCH();
    return;
  }
  if (ldc != N) throw Error{AGF2_ERR_ARG, "split GEMM needs a packed output"};
  float* part = scratch.as<float>((long)ns * M * N);
  hipLaunchKernelGGL((gemm_f32<TA, TB>), grid, dim3(256), 0, st, M, N, K, kchunk, A, sAm, sAk, B,
                     sBk, sBn, part, (long)N, (long)M * N, static_cast<const float*>(nullptr), 0L);
  AGF2_CHECK_LAUNCH();
  hipLaunchKernelGGL(sum_parts, dim3(grid1((long)M * N)), dim3(256), 0, st, part, (long)M * N, ns,
                     (long)M * N, C);
  AGF2_CHECK_LAUNCH();
}

void backward(agf2_mlp_s& net, int rows, const float* dY, hipStream_t st) {
  if (net.rows != rows) throw Error{AGF2_ERR_ARG, "backward needs the forward pass of the same rows"};
  const long r = rows;
  float* dZ2 = net.bwd.as<float>(2 * r * NH + 64);
  float* dZ1 = dZ2 + r * NH;
  DevBuf& scratch_split = net.split;
  // dW3 = A2^T dY, db3 = colsum dY
  gemm<h16, float>(NH, NO, rows, net.A2, 1, NH, dY, NO, 1, net.grad + OW3, NO, nullptr, 0,
                   scratch_split, st);
  hipLaunchKernelGGL(col_sums, dim3(1), dim3(256), 0, st, rows, NO, dY, net.grad + OB3);
  AGF2_CHECK_LAUNCH();
  // dZ2 = (dY W3^T) * gelu'(Z2); W3^T(o, h) = W3t[o][h]
  gemm<float, h16>(rows, NH, NO, dY, NO, 1, net.w16 + H3, NH, 1, dZ2, NH, net.Z2, NH,
                   scratch_split, st);
  gemm<h16, float>(NH, NH, rows, net.A1, 1, NH, dZ2, NH, 1, net.grad + OW2, NH, nullptr, 0,
                   scratch_split, st);
  hipLaunchKernelGGL(col_sums, dim3(1), dim3(256), 0, st, rows, NH, dZ2, net.grad + OB2);
  AGF2_CHECK_LAUNCH();
  gemm<float, h16>(rows, NH, NH, dZ2, NH, 1, net.w16 + H2, NH, 1, dZ1, NH, net.Z1, NH,
                   scratch_split, st);
  gemm<h16, float>(NF, NH, rows, net.X16, 1, NFP, dZ1, NH, 1, net.grad + OW1, NH, nullptr, 0,
                   scratch_split, st);
  hipLaunchKernelGGL(col_sums, dim3(1), dim3(256), 0, st, rows, NH, dZ1, net.grad + OB1);
  AGF2_CHECK_LAUNCH();
}

}  // namespace
}  // namespace agf2

using namespace agf2;

extern "C" {

agf2_status agf2_mlp_create(agf2_handle_t hh, agf2_mlp_t* out) {
  return guarded(hh, [&](Handle& h) {
    AGF2_REQUIRE(out, "NULL output");
    *out = nullptr;
    std::unique_ptr<agf2_mlp_s> net(new agf2_mlp_s());
    net->device = h.device;
    const long fbytes = 4 * NPARAM * 4;
    char* base = static_cast<char*>(net->params.get(fbytes + 256 + NHALF * 2));
    net->theta = reinterpret_cast<float*>(base);
    net->grad = net->theta + NPARAM;
    net->m = net->grad + NPARAM;
    net->v = net->m + NPARAM;
    net->w16 = reinterpret_cast<h16*>(base + (fbytes + 255) / 256 * 256);
    hipLaunchKernelGGL(fill_f32, dim3(grid1(4 * NPARAM)), dim3(256), 0, h.stream, 4 * NPARAM,
                       net->theta);
    AGF2_CHECK_LAUNCH();
    hipLaunchKernelGGL(fill_h16, dim3(grid1(NHALF)), dim3(256), 0, h.stream, NHALF, net->w16);
    AGF2_CHECK_LAUNCH();
    AGF2_HIP(hipStreamSynchronize(h.stream));
    *out = net.release();
  });
}

agf2_status agf2_mlp_destroy(agf2_mlp_t net) {
  if (!net) return AGF2_OK;
  int prev = 0;
  (void)hipGetDevice(&prev);
  (void)hipSetDevice(net->device);
  (void)hipDeviceSynchronize();
  net->params.release();
  net->act.release();
  net->bwd.release();
  net->split.release();
  delete net;
  (void)hipSetDevice(prev);
  return AGF2_OK;
}

agf2_status agf2_mlp_set_params(agf2_handle_t hh, agf2_mlp_t p, const float* params) {
  return guarded(hh, [&](Handle& h) {
    agf2_mlp_s& net = net_of(p, h);
    AGF2_REQUIRE(params, "NULL parameters");
    AGF2_HIP(hipMemcpyAsync(net.theta, params, NPARAM * sizeof(float), hipMemcpyHostToDevice,
                            h.stream));
    hipLaunchKernelGGL(fill_f32, dim3(grid1(3 * NPARAM)), dim3(256), 0, h.stream, 3 * NPARAM,
                       net.grad);
    AGF2_CHECK_LAUNCH();
    hipLaunchKernelGGL(refresh_half, dim3(grid1(NPARAM)), dim3(256), 0, h.stream, net.theta,
                       net.w16);
    AGF2_CHECK_LAUNCH();
    net.t = 0;
    AGF2_HIP(hipStreamSynchronize(h.stream));
  });
}

agf2_status agf2_mlp_get_params(agf2_handle_t hh, agf2_mlp_t p, float* params) {
  return guarded(hh, [&](Handle& h) {
    agf2_mlp_s& net = net_of(p, h);
    AGF2_REQUIRE(params, "NULL output");
    AGF2_HIP(hipMemcpyAsync(params, net.theta, NPARAM * sizeof(float), hipMemcpyDeviceToHost,
                            h.stream));
    AGF2_HIP(hipStreamSynchronize(h.stream));
  });
}

agf2_status agf2_mlp_get_grad(agf2_handle_t hh, agf2_mlp_t p, float* grad) {
  return guarded(hh, [&](Handle& h) {
    agf2_mlp_s& net = net_of(p, h);
    AGF2_REQUIRE(grad, "NULL output");
    AGF2_HIP(hipMemcpyAsync(grad, net.grad, NPARAM * sizeof(float), hipMemcpyDeviceToHost,
                            h.stream));
    AGF2_HIP(hipStreamSynchronize(h.stream));
  });
}

agf2_status agf2_mlp_features(agf2_handle_t hh, int nphys, int nocc, const double* e_mf,
                              const double* m0, float* X, double* scale) {
  return guarded(hh, [&](Handle& h) {
    AGF2_REQUIRE(nphys >= 2 && nocc >= 1 && nocc < nphys, "need 1 <= nocc < nphys");
    AGF2_REQUIRE(e_mf && m0 && X && scale, "NULL pointer");
    FiniteCheck(h).add(e_mf, nphys, "e_mf").add(m0, 4L * nphys * nphys, "m0").run();
    hipLaunchKernelGGL(features_kernel, dim3(1), dim3(256), 0, h.stream, nphys, nocc, e_mf, m0, X,
                       scale);
    AGF2_CHECK_LAUNCH();
  });
}

agf2_status agf2_mlp_forward(agf2_handle_t hh, agf2_mlp_t p, int rows, const float* X, float* Y) {
  return guarded(hh, [&](Handle& h) {
    agf2_mlp_s& net = net_of(p, h);
    AGF2_REQUIRE(rows >= 1 && X && Y, "bad rows or NULL pointer");
    forward(net, rows, X, Y, h.stream);
  });
}

agf2_status agf2_mlp_loss_grad(agf2_handle_t hh, int nphys, const float* Y, const double* m0,
                               const double* mconv, const double* scale, float* dY,
                               double* loss) {
  return guarded(hh, [&](Handle& h) {
    AGF2_REQUIRE(nphys >= 1 && nphys <= 65535, "bad nphys");
    AGF2_REQUIRE(Y && m0 && mconv && scale && dY && loss, "NULL pointer");
    FiniteCheck(h)
        .add(m0, 4L * nphys * nphys, "m0")
        .add(mconv, 4L * nphys * nphys, "mconv")
        .add(scale, 4, "scale")
        .run();
    double* lpart = h.ws_mlp[0].as<double>(4L * nphys);
    hipLaunchKernelGGL(head_loss, dim3(nphys, NMOM), dim3(256), 0, h.stream, nphys, Y, m0, mconv,
                       scale, dY, lpart);
    AGF2_CHECK_LAUNCH();
    hipLaunchKernelGGL(add_sum, dim3(1), dim3(1), 0, h.stream, 4L * nphys, lpart, loss);
    AGF2_CHECK_LAUNCH();
  });
}

agf2_status agf2_mlp_backward(agf2_handle_t hh, agf2_mlp_t p, int rows, const float* dY) {
  return guarded(hh, [&](Handle& h) {
    agf2_mlp_s& net = net_of(p, h);
    AGF2_REQUIRE(rows >= 1 && dY, "bad rows or NULL pointer");
    backward(net, rows, dY, h.stream);
  });
}

agf2_status agf2_mlp_adam_step(agf2_handle_t hh, agf2_mlp_t p, float lr, float beta1,
                               float beta2, float eps) {
  return guarded(hh, [&](Handle& h) {
    agf2_mlp_s& net = net_of(p, h);
    AGF2_REQUIRE(lr > 0.f && beta1 >= 0.f && beta1 < 1.f && beta2 >= 0.f && beta2 < 1.f &&
                     eps >= 0.f,
                 "bad Adam hyperparameters");
    net.t += 1;
    const float c1 = (float)(1.0 / (1.0 - std::pow((double)beta1, (double)net.t)));
    const float c2 = (float)(1.0 / (1.0 - std::pow((double)beta2, (double)net.t)));
    hipLaunchKernelGGL(adam_kernel, dim3(grid1(NPARAM)), dim3(256), 0, h.stream, NPARAM,
                       net.theta, net.grad, net.m, net.v, lr, beta1, beta2, eps, c1, c2);
    AGF2_CHECK_LAUNCH();
    hipLaunchKernelGGL(refresh_half, dim3(grid1(NPARAM)), dim3(256), 0, h.stream, net.theta,
                       net.w16);
    AGF2_CHECK_LAUNCH();
  });
}

agf2_status agf2_mlp_predict_correction(agf2_handle_t hh, agf2_mlp_t p, int nphys, int nocc,
                                        const double* e_mf, const double* m0, double* dm) {
  return guarded(hh, [&](Handle& h) {
    agf2_mlp_s& net = net_of(p, h);
    AGF2_REQUIRE(nphys >= 2 && nocc >= 1 && nocc < nphys, "need 1 <= nocc < nphys");
    AGF2_REQUIRE(e_mf && m0 && dm, "NULL pointer");
    FiniteCheck(h).add(e_mf, nphys, "e_mf").add(m0, 4L * nphys * nphys, "m0").run();
    char* ws = static_cast<char*>(h.ws_mlp[1].get((long)nphys * (NF + NO) * 4 + 512));
    float* X = reinterpret_cast<float*>(ws);
    float* Y = X + (long)nphys * NF;
    double* s = reinterpret_cast<double*>(ws + ((long)nphys * (NF + NO) * 4 + 255) / 256 * 256);
    hipLaunchKernelGGL(features_kernel, dim3(1), dim3(256), 0, h.stream, nphys, nocc, e_mf, m0, X,
                       s);
    AGF2_CHECK_LAUNCH();
    forward(net, nphys, X, Y, h.stream);
    hipLaunchKernelGGL(correction_kernel, dim3(grid1(4L * nphys * nphys)), dim3(256), 0,
                       h.stream, nphys, Y, m0, s, dm);
    AGF2_CHECK_LAUNCH();
  });
}

}  // extern "C"
