// FP64 MFMA GEMM for the library's O(N^4) steps (pole-basis DF transforms,
// exchange build, density build): 64x64 output tiles, 16-deep K steps staged
// through LDS in [k][m] layout, four waves each owning a 32x32 quadrant made
// of 2x2 v_mfma_f64_16x16x4 blocks. Global loads run one K step ahead of the
// MFMAs (register prefetch + double-buffered LDS).
#include "agf2_internal.h"

namespace agf2 {
namespace {

typedef double d4 __attribute__((ext_vector_type(4)));

constexpr int BM = 64, BN = 64, BK = 16, NT = 256;
constexpr int LDS_LD = BM + 1;  // odd stride: conflict-free transposed stores

template <bool A_MC, bool B_NC>
__global__ __launch_bounds__(NT) void gemm_f64_kernel(Gemm g, int Npad) {
  __shared__ double As[2][BK][LDS_LD];
  __shared__ double Bs[2][BK][LDS_LD];
  const int tid = threadIdx.x;
  const int lane = tid & 63, wave = tid >> 6;
  const int tiles_m = (g.M + BM - 1) / BM;
  const int tm = blockIdx.x % tiles_m, tn = blockIdx.x / tiles_m;
  if (g.lower && tn > tm) return;   // uniform over the workgroup
  const int b = blockIdx.y, s = blockIdx.z;
  const int m0 = tm * BM, n0 = tn * BN;
  const int r_per = (g.R + g.nsplit - 1) / g.nsplit;
  const int r0 = s * r_per, r1 = min(g.R, r0 + r_per);
  const int ktiles = (g.K + BK - 1) / BK;
  const int nsteps = max(0, r1 - r0) * ktiles;
  const double* Ab = g.A + (long)b * g.sAb;
  const double* Bb = g.B + (long)b * g.sBb;

  // thread -> (row, k) of the 4 elements it moves per operand and step
  int am[4], ak[4], bn[4], bk[4];
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    if (A_MC) { am[i] = tid % 64; ak[i] = tid / 64 + 4 * i; }
    else      { ak[i] = tid % 16; am[i] = tid / 16 + 16 * i; }
    if (B_NC) { bn[i] = tid % 64; bk[i] = tid / 64 + 4 * i; }
    else      { bk[i] = tid % 16; bn[i] = tid / 16 + 16 * i; }
  }

  double ra[4], rb[4];
  auto load = [&](int step) {
    const int r = r0 + step / ktiles;
    const int kb = (step % ktiles) * BK;
    const double* A = Ab + (long)r * g.sAr;
    const double* B = Bb + (long)r * g.sBr;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const int m = m0 + am[i], k = kb + ak[i];
      ra[i] = (m < g.M && k < g.K) ? A[(long)m * g.sAm + (long)k * g.sAk] : 0.0;
      const int n = n0 + bn[i], kk = kb + bk[i];
      rb[i] = (n < g.N && kk < g.K) ? B[(long)kk * g.sBk + (long)n * g.sBn] : 0.0;
    }
  };
  auto store = [&](int buf) {
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      As[buf][ak[i]][am[i]] = ra[i];
      Bs[buf][bk[i]][bn[i]] = rb[i];
    }
  };

  const int wm = (wave & 1) * 32, wn = (wave >> 1) * 32;
  const int fr = lane & 15, fk = lane >> 4;
  d4 acc[2][2];
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j) acc[i][j] = d4{0.0, 0.0, 0.0, 0.0};

  if (nsteps > 0) {
    load(0);
    store(0);
    __syncthreads();
  }
  for (int step = 0; step < nsteps; ++step) {
    const int buf = step & 1;
    if (step + 1 < nsteps) load(step + 1);
#pragma unroll
    for (int kk = 0; kk < BK; kk += 4) {
      double a[2], bb[2];
#pragma unroll
      for (int i = 0; i < 2; ++i) a[i] = As[buf][kk + fk][wm + 16 * i + fr];
#pragma unroll
      for (int j = 0; j < 2; ++j) bb[j] = Bs[buf][kk + fk][wn + 16 * j + fr];
#pragma unroll
      for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j)
          acc[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[i], bb[j], acc[i][j], 0, 0, 0);
    }
    if (step + 1 < nsteps) store(buf ^ 1);
    __syncthreads();
  }

  double* C = g.C + (long)b * g.sCb + (long)s * g.sCs;
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int m = m0 + wm + 16 * i + fk + 4 * r;
        const int n = n0 + wn + 16 * j + fr;
        if (m >= g.M) continue;
        double* c = C + (long)m * g.sCm + (long)n * g.sCn;
        if (n < g.N) {
          const double v = g.alpha * acc[i][j][r];
          *c = (g.beta != 0.0) ? v + g.beta * *c : v;
        } else if (n < Npad) {
          *c = 0.0;
        }
      }
}

__global__ void sum_slices_kernel(const double* in, long stride, int nslice,
                                  long n, double* out, double scale, int add) {
  for (long i = blockIdx.x * (long)blockDim.x + threadIdx.x; i < n;
       i += (long)gridDim.x * blockDim.x) {
    double acc = 0.0;
    for (int s = 0; s < nslice; ++s) acc += in[s * stride + i];
    acc *= scale;
    out[i] = add ? out[i] + acc : acc;
  }
}

}  // namespace

int gemm_f64_slots() {
  static int cached = 0;
  if (cached > 0) return cached;
  int dev = 0, cus = 0, per = 0;
  AGF2_HIP(hipGetDevice(&dev));
  AGF2_HIP(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
  AGF2_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, gemm_f64_kernel<true, true>, NT, 0));
  cached = std::max(1, cus) * std::max(1, per);
  return cached;
}

int gemm_f64_tiles(int M, int N) { return ((M + BM - 1) / BM) * ((N + BN - 1) / BN); }

void gemm_f64_padded(const Gemm& g, int Npad, hipStream_t stream) {
  if (g.M <= 0 || g.N <= 0) return;
  const bool amc = (g.sAm == 1);
  const bool bnc = (g.sBn == 1);
  if (!amc && g.sAk != 1)
    throw Error{AGF2_ERR_ARG, "gemm_f64: A needs a unit stride"};
  if (!bnc && g.sBk != 1)
    throw Error{AGF2_ERR_ARG, "gemm_f64: B needs a unit stride"};
  if (g.batch > 65535 || g.nsplit > 65535)
    throw Error{AGF2_ERR_ARG, "gemm_f64: batch too large"};
  const int tiles = ((g.M + BM - 1) / BM) * ((g.N + BN - 1) / BN);
  dim3 grid(tiles, g.batch, g.nsplit);
  if (amc && bnc)
    hipLaunchKernelGGL((gemm_f64_kernel<true, true>), grid, dim3(NT), 0, stream, g, Npad);
  else if (amc)
    hipLaunchKernelGGL((gemm_f64_kernel<true, false>), grid, dim3(NT), 0, stream, g, Npad);
  else if (bnc)
    hipLaunchKernelGGL((gemm_f64_kernel<false, true>), grid, dim3(NT), 0, stream, g, Npad);
  else
    hipLaunchKernelGGL((gemm_f64_kernel<false, false>), grid, dim3(NT), 0, stream, g, Npad);
  AGF2_CHECK_LAUNCH();
}

void gemm_f64(const Gemm& g, hipStream_t stream) { gemm_f64_padded(g, g.N, stream); }

void sum_slices(const double* in, long slice_stride, int nslice, long n,
                double* out, double scale, bool add, hipStream_t stream) {
  if (n <= 0) return;
  const int threads = 256;
  const long blocks = std::min<long>((n + threads - 1) / threads, 4096);
  hipLaunchKernelGGL(sum_slices_kernel, dim3(blocks), dim3(threads), 0, stream,
                     in, slice_stride, nslice, n, out, scale, add ? 1 : 0);
  AGF2_CHECK_LAUNCH();
}

}  // namespace agf2
