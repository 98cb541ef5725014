// Fock-matrix build (DF Coulomb and exchange), extended-Hamiltonian assembly
// and the small elementwise / reduction kernels of the Fock loop, the
// compression and the energy.
#include <algorithm>
#include <cmath>

#include "agf2_internal.h"

namespace agf2 {
void gemm_f64_padded(const Gemm& g, int Npad, hipStream_t stream);

namespace {

constexpr int RT = 256;

// rho[Q] = sum_rs L[Q][r][s] D[r][s]   (one workgroup per Q)
__global__ __launch_bounds__(RT) void rho_kernel(const double* L, const double* D,
                                                 int N, double* rho) {
  __shared__ double red[RT];
  const long nn = (long)N * N;
  const double* LQ = L + blockIdx.x * nn;
  double acc = 0.0;
  for (long i = threadIdx.x; i < nn; i += RT) acc += LQ[i] * D[i];
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

}  // namespace

void fock_build(Handle& h, int N, int Q, const double* L, const double* hcore,
                const double* D, double alpha, double* F) {
  hipStream_t st = h.stream;
  const long nn = (long)N * N;
  ProfScope ps(h, "fock.jk", 4.0 * Q * (double)nn * N + 4.0 * Q * (double)nn,
               8.0 * (3.0 * Q * nn + 3.0 * nn));
  double* rho = h.ws_fock[0].as<double>(Q);
  hipLaunchKernelGGL(rho_kernel, dim3(Q), dim3(RT), 0, st, L, D, N, rho);
  AGF2_CHECK_LAUNCH();
  // exchange K = sum_Q L_Q D L_Q, Q processed in chunks of qn slices, as
  // plain products on rocBLAS (column-major view: the memory of L_Q and D reads
  // as L_Q and D, both symmetric):
  //   X_Q = D L_Q, stored stacked as rows Q*N .. Q*N+N-1 of one (qn N) x N
  //         matrix (strided-batched GEMM);
  //   P_g = [L_Q ...] [X_Q; ...] over the G slices of group g, one GEMM of
  //         inner size G*N per group (strided-batched over the groups);
  //   K   = sum of the group partials of all chunks (fixed order).
  // Groups of about 8 slices keep each GEMM's inner size near 8N: one GEMM of
  // inner size qn N measured 1.7x slower, the library's own lower-triangle
  // GEMM reached ~25 TFLOP/s here.
  const long chunk_bytes = 1L << 30;
  const int QC = (int)std::max<long>(1, std::min<long>(Q, chunk_bytes / (8 * nn)));
  const int GS = std::max(1, std::min(8, QC));           // slices per group
  const int GMAX = (QC + GS - 1) / GS;                      // groups per chunk
  double* X = h.ws_fock[1].as<double>((long)QC * nn);
  double* Kp = h.ws_fock[2].as<double>((long)GMAX * nn);   // group k of every chunk adds to slot k
  double* K = h.ws_fock[3].as<double>(nn);
  auto check = [](rocblas_status bs, const char* what) {
    if (bs != rocblas_status_success)
      throw Error{AGF2_ERR_HIP, std::string(what) + ": " + rocblas_status_to_string(bs)};
  };
  for (int q0 = 0; q0 < Q; q0 += QC) {
    const int qn = std::min(QC, Q - q0);
    const double one = 1.0, zero = 0.0, beta = q0 == 0 ? 0.0 : 1.0;   // chunk 0 has GMAX groups
    const long ldx = (long)qn * N;
    check(rocblas_dgemm_strided_batched(h.blas, rocblas_operation_none, rocblas_operation_none,
                                        N, N, N, &one, D, N, 0, L + (long)q0 * nn, N, nn, &zero,
                                        X, ldx, N, qn),
          "rocblas_dgemm_strided_batched");
    const int full = qn / GS, rest = qn - full * GS;
    if (full > 0)
      check(rocblas_dgemm_strided_batched(
                h.blas, rocblas_operation_none, rocblas_operation_none, N, N, GS * N, &one,
                L + (long)q0 * nn, N, (long)GS * nn, X, ldx, (long)GS * N, &beta, Kp, N, nn,
                full),
            "rocblas_dgemm_strided_batched");
    if (rest > 0)
      check(rocblas_dgemm(h.blas, rocblas_operation_none, rocblas_operation_none, N, N, rest * N,
                          &one, L + (long)(q0 + full * GS) * nn, N, X + (long)full * GS * N, ldx,
                          &beta, Kp + (long)full * nn, N),
            "rocblas_dgemm");
  }
  sum_slices(Kp, nn, GMAX, nn, K, 1.0, false, st);
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
