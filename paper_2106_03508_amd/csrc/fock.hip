// Fock-matrix build (DF Coulomb and exchange), extended-Hamiltonian assembly
// and the small elementwise / reduction kernels of the Fock loop, the
// compression and the energy.
#include <algorithm>
#include <cmath>

#include "agf2_internal.h"

namespace agf2 {

namespace {

constexpr int RT = 256;

// rho[Q] = sum_rs L[Q][r][s] D[r][s] = tr(D L_Q), read off the diagonal of
// slice Q of X = D [L_Q ...]   (one workgroup per Q)
__global__ __launch_bounds__(RT) void rho_kernel(const double* X, int N, double* rho) {
  __shared__ double red[RT];
  const long nn = (long)N * N;
  const double* XQ = X + blockIdx.x * nn;
  double acc = 0.0;
  for (int i = threadIdx.x; i < N; i += RT) acc += XQ[(long)i * (N + 1)];
  red[threadIdx.x] = acc;
  __syncthreads();
  for (int s = RT / 2; s > 0; s >>= 1) {
    if (threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
    __syncthreads();
  }
  if (threadIdx.x == 0) rho[blockIdx.x] = red[0];
}

// F = h + alpha * (sum_Q rho_Q L[Q] - 1/2 K)
__global__ void fock_combine_kernel(const double* L, const double* rho, int Q, int N,
                                    const double* h, const double* K, double alpha,
                                    double* F) {
  const long nn = (long)N * N;
  for (long i = blockIdx.x * (long)blockDim.x + threadIdx.x; i < nn;
       i += (long)gridDim.x * blockDim.x) {
    double j = 0.0;
    for (int q = 0; q < Q; ++q) j += rho[q] * L[q * nn + i];
    // K is symmetric and only its lower triangle is built
    const int p = (int)(i / N), r = (int)(i % N);
    const long kl = p >= r ? i : (long)r * N + p;
    F[i] = h[i] + alpha * (j - 0.5 * K[kl]);
  }
}

__global__ void hext_kernel(int N, int naux, const double* F, const double* e,
                            const double* v, double shift, double* H) {
  const int n = N + naux;
  const long tot = (long)n * n;
  for (long idx = blockIdx.x * (long)blockDim.x + threadIdx.x; idx < tot;
       idx += (long)gridDim.x * blockDim.x) {
    const int r = (int)(idx / n), c = (int)(idx % n);
    double val;
    if (r < N && c < N) val = F[(long)r * N + c];
    else if (r < N) val = v[(long)r * naux + (c - N)];
    else if (c < N) val = v[(long)c * naux + (r - N)];
    else val = (r == c) ? e[r - N] + shift : 0.0;
    H[idx] = val;
  }
}

// w[l] = sum_{p < nphys} evecs[l][p]^2  (one wave per l)
__global__ void colweight_kernel(int nphys, int npole, const double* ev, double* w) {
  const int l = blockIdx.x * (blockDim.x / 64) + threadIdx.x / 64;
  const int lane = threadIdx.x & 63;
  if (l >= npole) return;
  const double* row = ev + (long)l * npole;
  double acc = 0.0;
  for (int p = lane; p < nphys; p += 64) acc += row[p] * row[p];
  for (int off = 32; off > 0; off >>= 1) acc += __shfl_down(acc, off, 64);
  if (lane == 0) w[l] = acc;
}

// u[p][l] = evecs[l][p], p < N
__global__ void extract_kernel(int N, int npole, const double* ev, double* u) {
  const long tot = (long)N * npole;
  for (long idx = blockIdx.x * (long)blockDim.x + threadIdx.x; idx < tot;
       idx += (long)gridDim.x * blockDim.x) {
    const int p = (int)(idx / npole), l = (int)(idx % npole);
    u[idx] = ev[(long)l * npole + p];
  }
}

// per-block partial sums of a[i]*b[i]
__global__ __launch_bounds__(RT) void dot_kernel(long n, const double* a, const double* b,
                                                 double* part) {
  __shared__ double red[RT];
  double acc = 0.0;
  for (long i = blockIdx.x * (long)RT + threadIdx.x; i < n; i += (long)gridDim.x * RT)
    acc += a[i] * b[i];
  red[threadIdx.x] = acc;
  __syncthreads();
  for (int s = RT / 2; s > 0; s >>= 1) {
    if (threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
    __syncthreads();
  }
  if (threadIdx.x == 0) part[blockIdx.x] = red[0];
}

__global__ void axpby_kernel(long n, double a, const double* x, double b, double* y) {
  for (long i = blockIdx.x * (long)blockDim.x + threadIdx.x; i < n;
       i += (long)gridDim.x * blockDim.x)
    y[i] = a * x[i] + (b == 0.0 ? 0.0 : b * y[i]);
}

__global__ void symmetrize_kernel(int N, double* A) {
  const long tot = (long)N * N;
  for (long idx = blockIdx.x * (long)blockDim.x + threadIdx.x; idx < tot;
       idx += (long)gridDim.x * blockDim.x) {
    const int r = (int)(idx / N), c = (int)(idx % N);
    if (r <= c) continue;
    const double s = 0.5 * (A[idx] + A[(long)c * N + r]);
    A[idx] = s;
    A[(long)c * N + r] = s;
  }
}

inline long nblocks(long n) { return std::max<long>(1, std::min<long>((n + 255) / 256, 8192)); }

// ------------------------------------------------------------ exchange product
// Lower-triangle TS x TS tiles (TS = 32 WB) of P_s += sum_k L[x][k] Y[y][k]
// over the stacked column index k = Q N + r of one chunk of slices, with
//   L[x][k] = L_Q[x][r]       (slice Q of the chunk, row-major N x N)
//   Y[y][k] = (L_Q D)[y][r]   (same layout).
// K = sum_Q L_Q D L_Q is symmetric, so only these tiles are formed: half the
// flops of the full product. Workgroup items are (tile, split of k); split s
// adds into partial slot s, and the slots are summed in a fixed order after
// the last chunk. Four waves each own a quadrant of WB x WB MFMA blocks.
typedef double d4 __attribute__((ext_vector_type(4)));
constexpr int BK = 16;

struct ExchLower {
  const double* L;   // first slice of the chunk
  const double* Y;
  int N, K, kper;    // K = slices x N columns
  double* part;      // [nsplit][N][N], accumulated
  int tiles;         // lower-triangle tile count
  long items;        // tiles x nsplit
};

// Round-robin dispatch places workgroup w on XCD w % 8; remap so that each
// XCD receives one contiguous range of items (split-major: one k range per L2).
__device__ __forceinline__ long xcd_remap(long w, long G) {
  const long per = G / 8, rem = G % 8;
  const long xcd = w % 8, slot = w / 8;
  return xcd < rem ? xcd * (per + 1) + slot : rem * (per + 1) + (xcd - rem) * per + slot;
}

template <int WB>
__global__ __launch_bounds__(RT, 2) void exchange_lower_kernel(ExchLower a) {
  constexpr int TS = 32 * WB, LDL = TS + 1, RPT = TS / 16;
  __shared__ double X[2][BK][LDL], Yl[2][BK][LDL];
  const long item = xcd_remap(blockIdx.x, a.items);
  const int t = (int)(item % a.tiles), s = (int)(item / a.tiles);
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  int xt = (int)((sqrt(8.0 * t + 1.0) - 1.0) * 0.5);
  while ((xt + 1) * (xt + 2) / 2 <= t) ++xt;
  while (xt * (xt + 1) / 2 > t) --xt;
  const int yt = t - xt * (xt + 1) / 2;
  const int k0 = s * a.kper, k1 = min(a.K, k0 + a.kper);
  if (k1 <= k0) return;   // uniform over the workgroup
  const int x0 = xt * TS, y0 = yt * TS;
  const int N = a.N;
  const long nn = (long)N * N;
  // loader: thread -> column k0 + step*BK + tid % 16, rows tid/16 + 16 i; rows
  // past N read row N - 1 (their outputs are not stored). Row offsets are
  // below the chunk's element count, which the host keeps below 2^31.
  const int lk = tid & 15, lr = tid >> 4;
  int ox[RPT], oy[RPT];
#pragma unroll
  for (int i = 0; i < RPT; ++i) {
    ox[i] = min(x0 + lr + 16 * i, N - 1) * N;
    oy[i] = min(y0 + lr + 16 * i, N - 1) * N;
  }
  double rx[RPT], ry[RPT];
  auto load = [&](int kb) {
    const int k = kb + lk;
    const bool kin = k < k1;
    const int q = k / N;
    const int lo = q * N * N + (k - q * N);
#pragma unroll
    for (int i = 0; i < RPT; ++i) {
      rx[i] = kin ? a.L[ox[i] + lo] : 0.0;
      ry[i] = kin ? a.Y[oy[i] + lo] : 0.0;
    }
  };
  auto store = [&](int buf) {
#pragma unroll
    for (int i = 0; i < RPT; ++i) {
      X[buf][lk][lr + 16 * i] = rx[i];
      Yl[buf][lk][lr + 16 * i] = ry[i];
    }
  };
  const int wm = (wave & 1) * 16 * WB, wn = (wave >> 1) * 16 * WB;
  const int fr = lane & 15, fk = lane >> 4;
  d4 acc[WB][WB];
#pragma unroll
  for (int i = 0; i < WB; ++i)
#pragma unroll
    for (int j = 0; j < WB; ++j) acc[i][j] = d4{0.0, 0.0, 0.0, 0.0};
  const int nsteps = (k1 - k0 + BK - 1) / BK;
  load(k0);
  store(0);
  __syncthreads();
  for (int step = 0; step < nsteps; ++step) {
    const int buf = step & 1;
    if (step + 1 < nsteps) load(k0 + (step + 1) * BK);
#pragma unroll
    for (int kk = 0; kk < BK; kk += 4) {
      double xa[WB], yb[WB];
#pragma unroll
      for (int i = 0; i < WB; ++i) xa[i] = X[buf][kk + fk][wm + 16 * i + fr];
#pragma unroll
      for (int j = 0; j < WB; ++j) yb[j] = Yl[buf][kk + fk][wn + 16 * j + fr];
#pragma unroll
      for (int i = 0; i < WB; ++i)
#pragma unroll
        for (int j = 0; j < WB; ++j)
          acc[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(xa[i], yb[j], acc[i][j], 0, 0, 0);
    }
    if (step + 1 < nsteps) store(buf ^ 1);
    __syncthreads();
  }
  double* P = a.part + (long)s * nn;
#pragma unroll
  for (int i = 0; i < WB; ++i)
#pragma unroll
    for (int j = 0; j < WB; ++j)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int x = x0 + wm + 16 * i + fk + 4 * r;
        const int y = y0 + wn + 16 * j + fr;
        if (x >= N || y >= N) continue;
        P[(long)x * N + y] += acc[i][j][r];
      }
}

// Splits of the stacked columns for one chunk of kfull columns: the count
// (at most 256 and 512 MB of partials, at least 8 K steps each) that
// minimises rounds of resident workgroups times K steps per item, fewest
// splits on ties.
template <int WB>
int exchange_splits(int N, int tiles, int kfull) {
  static int slots = 0;
  if (slots == 0) {
    int dev = 0, cus = 0, per = 0;
    AGF2_HIP(hipGetDevice(&dev));
    AGF2_HIP(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
    AGF2_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, exchange_lower_kernel<WB>, RT,
                                                          0));
    slots = std::max(1, cus) * std::max(1, per);
  }
  const long cap = std::min<long>(256, (1L << 26) / ((long)N * N));
  const int hi = (int)std::max<long>(1, std::min<long>(cap, kfull / (8 * BK)));
  int best = 1;
  long best_cost = -1;
  for (int ns = 1; ns <= hi; ++ns) {
    const long rounds = ((long)tiles * ns + slots - 1) / slots;
    const long steps = ((kfull + ns - 1) / ns + BK - 1) / BK;
    if (best_cost < 0 || rounds * steps < best_cost) {
      best_cost = rounds * steps;
      best = ns;
    }
  }
  return best;
}

// K's lower triangle += sum_Q L_Q (L_Q D)^T for the chunks of slices, X the
// (L_Q D) of one chunk; partial slots zeroed here. Also rho[Q] = tr(L_Q D).
template <int WB>
void exchange_lower(Handle& h, int N, int Q, int QC, const double* L, const double* D,
                    double* X, double* K, double* rho) {
  hipStream_t st = h.stream;
  const long nn = (long)N * N;
  const int ts = 32 * WB, tiles_side = (N + ts - 1) / ts;
  const int tiles = tiles_side * (tiles_side + 1) / 2;
  const int nsplit = exchange_splits<WB>(N, tiles, QC * N);
  double* Kp = h.ws_fock[2].as<double>((long)nsplit * nn);
  fill_zero(Kp, (long)nsplit * nn, st);
  for (int q0 = 0; q0 < Q; q0 += QC) {
    const int qn = std::min(QC, Q - q0);
    // one GEMM over the chunk, X_Q = L_Q D for its slices stacked as rows:
    // X[n][m] = sum_k L[q0 N^2 + n N + k] D[k N + m], n over qn N rows
    Gemm g;
    g.M = qn * N; g.N = N; g.K = N;
    g.A = L + (long)q0 * nn; g.sAm = N; g.sAk = 1;
    g.B = D; g.sBk = N; g.sBn = 1;
    g.C = X; g.sCm = N; g.sCn = 1;
    gemm_f64(g, st);
    hipLaunchKernelGGL(rho_kernel, dim3(qn), dim3(RT), 0, st, X, N, rho + q0);
    AGF2_CHECK_LAUNCH();
    ExchLower a;
    a.L = L + (long)q0 * nn;
    a.Y = X;
    a.N = N;
    a.K = qn * N;
    a.kper = (a.K + nsplit - 1) / nsplit;
    a.kper = (a.kper + BK - 1) / BK * BK;
    a.part = Kp;
    a.tiles = tiles;
    a.items = (long)tiles * nsplit;
    hipLaunchKernelGGL(exchange_lower_kernel<WB>, dim3((unsigned)a.items), dim3(RT), 0, st, a);
    AGF2_CHECK_LAUNCH();
  }
  sum_slices(Kp, nn, nsplit, nn, K, 1.0, false, st);
}

}  // namespace

void fock_build(Handle& h, int N, int Q, const double* L, const double* hcore,
                const double* D, double alpha, double* F) {
  hipStream_t st = h.stream;
  const long nn = (long)N * N;
  ProfScope ps(h, "fock.jk", 3.0 * Q * (double)nn * N + 2.0 * Q * (double)nn,
               8.0 * (3.0 * Q * nn + 3.0 * nn));
  double* rho = h.ws_fock[0].as<double>(Q);
  // exchange K = sum_Q L_Q D L_Q, Q processed in chunks of qn slices:
  //   X = D [L_Q ...], one rocBLAS GEMM of N x (qn N) x N (column-major view:
  //       the memory of L_Q and D reads as L_Q and D, both symmetric); slice Q
  //       of X, read row-major, is L_Q D;
  //   K's lower triangle += sum_Q L_Q (L_Q D)^T by exchange_lower_kernel,
  //       split over the stacked columns into partial slots (same slots for
  //       every chunk), summed in a fixed order at the end.
  // 2QN^3 + QN^3 flops instead of 4QN^3 for two full products.
  const long chunk_bytes = 1L << 30;
  const int QC = (int)std::max<long>(1, std::min<long>(Q, chunk_bytes / (8 * nn)));
  // the exchange kernel indexes one chunk with 32-bit offsets (N <= 46340)
  if ((long)QC * nn >= (1L << 31))
    throw Error{AGF2_ERR_ARG, "agf2_fock_build: nphys too large for one exchange chunk"};
  double* X = h.ws_fock[1].as<double>((long)QC * nn);
  double* K = h.ws_fock[3].as<double>(nn);
  // 128-wide tiles (four MFMA blocks a side per wave) when their padded lower
  // triangle is within 8% of the 64-wide tiles' (e.g. N = 705-768, 833-896,
  // 961-1024), else 64-wide
  auto padded = [N](long ts) {
    const long t = (N + ts - 1) / ts;
    return t * (t + 1) / 2 * ts * ts;
  };
  if (padded(128) <= 1.08 * padded(64))
    exchange_lower<4>(h, N, Q, QC, L, D, X, K, rho);
  else
    exchange_lower<2>(h, N, Q, QC, L, D, X, K, rho);
  hipLaunchKernelGGL(fock_combine_kernel, dim3(nblocks(nn)), dim3(256), 0, st, L, rho,
                     Q, N, hcore, K, alpha, F);
  AGF2_CHECK_LAUNCH();
}

void build_hext(int N, int naux, const double* F, const double* e, const double* v,
                double shift, double* H, hipStream_t s) {
  const long n = (long)(N + naux) * (N + naux);
  hipLaunchKernelGGL(hext_kernel, dim3(nblocks(n)), dim3(256), 0, s, N, naux, F, e, v,
                     shift, H);
  AGF2_CHECK_LAUNCH();
}

void column_weights(int nphys, int npole, const double* ev, double* w, hipStream_t s) {
  hipLaunchKernelGGL(colweight_kernel, dim3((npole + 3) / 4), dim3(256), 0, s, nphys,
                     npole, ev, w);
  AGF2_CHECK_LAUNCH();
}

void extract_poles(int N, int npole, const double* ev, double* u, hipStream_t s) {
  const long n = (long)N * npole;
  hipLaunchKernelGGL(extract_kernel, dim3(nblocks(n)), dim3(256), 0, s, N, npole, ev, u);
  AGF2_CHECK_LAUNCH();
}

double dot_f64(Handle& h, long n, const double* a, const double* b) {
  const int blocks = (int)std::max<long>(1, std::min<long>((n + RT - 1) / RT, 512));
  double* part = h.ws_red.as<double>(512);
  hipLaunchKernelGGL(dot_kernel, dim3(blocks), dim3(RT), 0, h.stream, n, a, b, part);
  AGF2_CHECK_LAUNCH();
  AGF2_HIP(hipMemcpyAsync(h.host_red, part, blocks * sizeof(double), hipMemcpyDeviceToHost,
                          h.stream));
  AGF2_HIP(hipStreamSynchronize(h.stream));
  double s = 0.0;
  for (int i = 0; i < blocks; ++i) s += h.host_red[i];
  return s;
}

void axpby_f64(long n, double a, const double* x, double b, double* y, hipStream_t s) {
  hipLaunchKernelGGL(axpby_kernel, dim3(nblocks(n)), dim3(256), 0, s, n, a, x, b, y);
  AGF2_CHECK_LAUNCH();
}

void symmetrize_f64(int N, double* A, hipStream_t s) {
  hipLaunchKernelGGL(symmetrize_kernel, dim3(nblocks((long)N * N)), dim3(256), 0, s, N, A);
  AGF2_CHECK_LAUNCH();
}

}  // namespace agf2
