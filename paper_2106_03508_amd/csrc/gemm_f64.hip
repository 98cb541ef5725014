// FP64 MFMA GEMM for the library's O(N^4) steps (pole-basis DF transforms,
// exchange build, density build). Square output tiles of BT x BT (128 for
// large products, 64 for small ones), 16-deep K steps, four waves each owning
// a (BT/2) x (BT/2) quadrant of v_mfma_f64_16x16x4 blocks. Operand tiles sit in
// LDS as [row][k] with rows padded to 18 doubles: each lane reads its four k
// values of a block row with two ds_read_b128, and the padding keeps both the
// row-contiguous and the k-contiguous staging stores free of bank conflicts.
// Global loads run one K step ahead of the MFMAs (register prefetch +
// double-buffered LDS). Within one MFMA step lane group g = lane / 16 sums
// k = 4 g + j (j = 0..3): the same relabelling of k on both operands.
#include "agf2_internal.h"

namespace agf2 {
namespace {

typedef double d4 __attribute__((ext_vector_type(4)));

constexpr int BK = 16, NT = 256;
constexpr int LDK = BK + 2;

// Workgroups are dealt to the 8 XCDs round-robin (workgroup w on XCD w % 8):
// give each XCD one contiguous range of the tile order, so the tiles that
// share operand rows run under one L2.
__device__ __forceinline__ long xcd_order(long w, long G) {
  const long per = G / 8, rem = G % 8;
  const long xcd = w % 8, slot = w / 8;
  return xcd < rem ? xcd * (per + 1) + slot : rem * (per + 1) + (xcd - rem) * per + slot;
}

template <int BT, bool A_MC, bool B_NC>
__global__ __launch_bounds__(NT, 2) void gemm_f64_kernel(Gemm g, int Npad, int tiles_m,
                                                         int tiles_n, long total) {
  constexpr int E = BT * BK / NT;   // elements per thread per operand and K step
  constexpr int WT = BT / 2;        // quadrant side
  constexpr int MI = WT / 16;       // MFMA blocks per quadrant side
  __shared__ __align__(16) double As[2][BT][LDK];
  __shared__ __align__(16) double Bs[2][BT][LDK];
  const int tid = threadIdx.x;
  const int lane = tid & 63, wave = tid >> 6;
  // tile order: n tiles fastest, then m tiles, then the batch
  long t = xcd_order(blockIdx.x, total);
  const int tn = (int)(t % tiles_n);
  t /= tiles_n;
  const int tm = (int)(t % tiles_m);
  const int b = (int)(t / tiles_m);
  if (g.lower && tn > tm) return;   // uniform over the workgroup
  const int m0 = tm * BT, n0 = tn * BT;
  const int nsteps = (g.K + BK - 1) / BK;

  // thread -> (row, k) of its E elements per operand: along the contiguous
  // direction of each operand in global memory. Rows past the edge read the
  // last row (their outputs are never stored); in the last, ragged K step, k
  // past K reads k = K - 1 and is replaced by zero.
  auto srow_a = [&](int i) { return A_MC ? tid % BT : tid / BK + (NT / BK) * i; };
  auto srow_b = [&](int i) { return B_NC ? tid % BT : tid / BK + (NT / BK) * i; };
  auto sk_a = [&](int i) { return A_MC ? tid / BT + (NT / BT) * i : tid % BK; };
  auto sk_b = [&](int i) { return B_NC ? tid / BT + (NT / BT) * i : tid % BK; };
  long ao[E], bo[E];   // element offsets of (row, k) within the K step
#pragma unroll
  for (int i = 0; i < E; ++i) {
    ao[i] = (long)min(m0 + srow_a(i), g.M - 1) * g.sAm + (long)sk_a(i) * g.sAk;
    bo[i] = (long)min(n0 + srow_b(i), g.N - 1) * g.sBn + (long)sk_b(i) * g.sBk;
  }
  const double* Ab = g.A + (long)b * g.sAb;
  const double* Bb = g.B + (long)b * g.sBb;

  double ra[E], rb[E];
  int lkb = 0;   // first k of the next load
  auto load = [&]() {
    const double* A = Ab + (long)lkb * g.sAk;
    const double* B = Bb + (long)lkb * g.sBk;
    if (lkb + BK <= g.K) {   // uniform: a whole K step
#pragma unroll
      for (int i = 0; i < E; ++i) {
        ra[i] = A[ao[i]];
        rb[i] = B[bo[i]];
      }
    } else {
#pragma unroll
      for (int i = 0; i < E; ++i) {
        const int ka = lkb + sk_a(i), kb = lkb + sk_b(i);
        const double va = A[ao[i] + (long)(min(ka, g.K - 1) - ka) * g.sAk];
        const double vb = B[bo[i] + (long)(min(kb, g.K - 1) - kb) * g.sBk];
        ra[i] = ka < g.K ? va : 0.0;
        rb[i] = kb < g.K ? vb : 0.0;
      }
    }
    lkb += BK;
  };
  auto store = [&](int buf) {
#pragma unroll
    for (int i = 0; i < E; ++i) {
      As[buf][srow_a(i)][sk_a(i)] = ra[i];
      Bs[buf][srow_b(i)][sk_b(i)] = rb[i];
    }
  };

  const int wm = (wave & 1) * WT, wn = (wave >> 1) * WT;
  const int fr = lane & 15, fk = lane >> 4;
  d4 acc[MI][MI];
#pragma unroll
  for (int i = 0; i < MI; ++i)
#pragma unroll
    for (int j = 0; j < MI; ++j) acc[i][j] = d4{0.0, 0.0, 0.0, 0.0};

  if (nsteps > 0) {
    load();
    store(0);
    __syncthreads();
  }
  for (int step = 0; step < nsteps; ++step) {
    const int buf = step & 1;
    if (step + 1 < nsteps) load();
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      double2 a[MI], bb[MI];
#pragma unroll
      for (int i = 0; i < MI; ++i)
        a[i] = *reinterpret_cast<const double2*>(&As[buf][wm + 16 * i + fr][4 * fk + 2 * h]);
#pragma unroll
      for (int j = 0; j < MI; ++j)
        bb[j] = *reinterpret_cast<const double2*>(&Bs[buf][wn + 16 * j + fr][4 * fk + 2 * h]);
#pragma unroll
      for (int i = 0; i < MI; ++i)
#pragma unroll
        for (int j = 0; j < MI; ++j)
          acc[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[i].x, bb[j].x, acc[i][j], 0, 0, 0);
#pragma unroll
      for (int i = 0; i < MI; ++i)
#pragma unroll
        for (int j = 0; j < MI; ++j)
          acc[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[i].y, bb[j].y, acc[i][j], 0, 0, 0);
    }
    if (step + 1 < nsteps) store(buf ^ 1);
    __syncthreads();
  }

  double* C = g.C + (long)b * g.sCb;
#pragma unroll
  for (int i = 0; i < MI; ++i)
#pragma unroll
    for (int j = 0; j < MI; ++j)
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

namespace {

template <int BT>
void launch_tiles(const Gemm& g, int Npad, bool amc, bool bnc, hipStream_t stream) {
  const int tm = (g.M + BT - 1) / BT, tn = (Npad + BT - 1) / BT;
  const long total = (long)tm * tn * g.batch;
  if (total * NT >= (1L << 32))
    throw Error{AGF2_ERR_ARG, "gemm_f64: product too large for one launch"};
  const dim3 grid((unsigned)total), block(NT);
  if (amc && bnc)
    hipLaunchKernelGGL((gemm_f64_kernel<BT, true, true>), grid, block, 0, stream, g, Npad, tm, tn, total);
  else if (amc)
    hipLaunchKernelGGL((gemm_f64_kernel<BT, true, false>), grid, block, 0, stream, g, Npad, tm, tn, total);
  else if (bnc)
    hipLaunchKernelGGL((gemm_f64_kernel<BT, false, true>), grid, block, 0, stream, g, Npad, tm, tn, total);
  else
    hipLaunchKernelGGL((gemm_f64_kernel<BT, false, false>), grid, block, 0, stream, g, Npad, tm, tn, total);
  AGF2_CHECK_LAUNCH();
}

// Resident workgroups of the 128-tile kernel on the current device.
int slots_128() {
  static int cached = 0;
  if (cached > 0) return cached;
  int dev = 0, cus = 0, per = 0;
  AGF2_HIP(hipGetDevice(&dev));
  AGF2_HIP(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
  AGF2_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, gemm_f64_kernel<128, true, true>,
                                                        NT, 0));
  cached = std::max(1, cus) * std::max(1, per);
  return cached;
}

}  // namespace

void gemm_f64_padded(const Gemm& g, int Npad, hipStream_t stream) {
  if (g.M <= 0 || g.N <= 0) return;
  const bool amc = (g.sAm == 1);
  const bool bnc = (g.sBn == 1);
  if (!amc && g.sAk != 1)
    throw Error{AGF2_ERR_ARG, "gemm_f64: A needs a unit stride"};
  if (!bnc && g.sBk != 1)
    throw Error{AGF2_ERR_ARG, "gemm_f64: B needs a unit stride"};
  if (g.batch < 1 || Npad < g.N)
    throw Error{AGF2_ERR_ARG, "gemm_f64: bad batch or padding"};
  // 128-wide tiles once they fill the resident slots twice over (smaller
  // products keep the 64-wide tiles, four times as many workgroups)
  const long t128 = (long)((g.M + 127) / 128) * ((Npad + 127) / 128) * g.batch;
  if (t128 >= 2L * slots_128())
    launch_tiles<128>(g, Npad, amc, bnc, stream);
  else
    launch_tiles<64>(g, Npad, amc, bnc, stream);
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
