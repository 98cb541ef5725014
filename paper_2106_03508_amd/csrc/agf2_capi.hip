// C ABI of the library (declared in include/agf2.h): argument checks, the
// handle, and the host-side orchestration of compression, Fock loop and
// energy around the device kernels.
#include <rocsolver/rocsolver.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <exception>
#include <new>

#include "agf2_internal.h"

namespace agf2 {

void* DevBuf::get(size_t need) {
  if (need == 0) need = 1;
  if (need <= bytes) return ptr;
  if (ptr) {
    // kernels queued on any stream may still read the old buffer
    AGF2_HIP(hipDeviceSynchronize());
    AGF2_HIP(hipFree(ptr));
    ptr = nullptr;
    bytes = 0;
  }
  if (hipMalloc(&ptr, need) != hipSuccess) {
    ptr = nullptr;
    (void)hipGetLastError();
    throw Error{AGF2_ERR_NOMEM, "device workspace allocation of " +
                                    std::to_string(need) + " bytes failed"};
  }
  bytes = need;
  return ptr;
}

void DevBuf::release() {
  if (ptr) (void)hipFree(ptr);
  ptr = nullptr;
  bytes = 0;
}

ProfScope::ProfScope(Handle& hh, const char* name, double flops, double bytes)
    : h(hh), on(hh.profiling) {
  if (!on) return;
  rec.name = name;
  rec.flops = flops;
  rec.bytes = bytes;
  AGF2_HIP(hipEventCreate(&rec.start));
  AGF2_HIP(hipEventCreate(&rec.stop));
  AGF2_HIP(hipEventRecord(rec.start, h.stream));
}

// Folds the pending records into the totals once their stop events have
// completed (stream order: the last one's completion implies all). Errors
// are not thrown from here (it also runs in a destructor): a record whose
// time cannot be read is dropped.
static hipError_t prof_drain(Handle& h) noexcept {
  if (h.prof_pending.empty()) return hipSuccess;
  const hipError_t sync = hipEventSynchronize(h.prof_pending.back().stop);
  for (auto& r : h.prof_pending) {
    float ms = 0.f;
    if (sync == hipSuccess && hipEventElapsedTime(&ms, r.start, r.stop) == hipSuccess) {
      ProfTotal& t = h.prof_total[r.name];
      t.launches += 1;
      t.ms += ms;
      t.flops += r.flops;
      t.bytes += r.bytes;
    }
    (void)hipEventDestroy(r.start);
    (void)hipEventDestroy(r.stop);
  }
  h.prof_pending.clear();
  return sync;
}

// At most this many timed launches hold their two events at once; a longer
// run folds the completed ones (one wait on the last stop event).
constexpr size_t PROF_PENDING_MAX = 2048;

ProfScope::~ProfScope() {
  if (!on) return;
  if (hipEventRecord(rec.stop, h.stream) != hipSuccess) {
    (void)hipEventDestroy(rec.start);
    (void)hipEventDestroy(rec.stop);
    return;
  }
  h.prof_pending.push_back(rec);
  if (h.prof_pending.size() >= PROF_PENDING_MAX) (void)prof_drain(h);
}

static void prof_flush(Handle& h) {
  AGF2_HIP(prof_drain(h));
}

// One bit of *flag per array: set when any element is NaN or infinite (a
// vote per wave, one atomic per wave that saw one).
__global__ __launch_bounds__(256) void nonfinite_kernel(long n, const double* x,
                                                        unsigned bit, unsigned* flag) {
  int bad = 0;
  for (long i = blockIdx.x * 256L + threadIdx.x; i < n; i += (long)gridDim.x * 256)
    bad |= !(std::fabs(x[i]) <= 1.7976931348623157e308);
  if (__any(bad) && (threadIdx.x & 63) == 0) atomicOr(flag, 1u << bit);
}

FiniteCheck& FiniteCheck::add(const double* p, long n, const char* what) {
  if (p && n > 0) {
    if (ptr.size() >= 32) throw Error{AGF2_ERR_ARG, "internal: too many arrays in one check"};
    ptr.push_back(p);
    len.push_back(n);
    name.push_back(what);
  }
  return *this;
}

void FiniteCheck::run() {
  if (ptr.empty()) return;
  unsigned* flag = h.ws_check.as<unsigned>(1);
  AGF2_HIP(hipMemsetAsync(flag, 0, sizeof(unsigned), h.stream));
  for (size_t k = 0; k < ptr.size(); ++k) {
    const int nb = (int)std::max<long>(1, std::min<long>((len[k] + 255) / 256, 2048));
    hipLaunchKernelGGL(nonfinite_kernel, dim3(nb), dim3(256), 0, h.stream, len[k], ptr[k],
                       (unsigned)k, flag);
    AGF2_CHECK_LAUNCH();
  }
  unsigned hf = 0;
  AGF2_HIP(hipMemcpyAsync(&hf, flag, sizeof(unsigned), hipMemcpyDeviceToHost, h.stream));
  AGF2_HIP(hipStreamSynchronize(h.stream));
  for (size_t k = 0; k < ptr.size(); ++k)
    if (hf & (1u << k))
      throw Error{AGF2_ERR_ARG, name[k] + " holds a non-finite value (NaN or infinity)"};
}

Handle::~Handle() {
  (void)hipDeviceSynchronize();
  destroy_batch_plan(batch);
  for (auto& r : prof_pending) {
    (void)hipEventDestroy(r.start);
    (void)hipEventDestroy(r.stop);
  }
  for (auto& b : ws_moments) b.release();
  for (auto& b : ws_fock) b.release();
  for (auto& b : ws_misc) b.release();
  for (auto& b : ws_run) b.release();
  for (auto& b : ws_mlp) b.release();
  ws_spec.release();
  ws_red.release();
  ws_check.release();
  if (host_red) (void)hipHostFree(host_red);
  if (blas) rocblas_destroy_handle(blas);
  if (own_stream && stream) (void)hipStreamDestroy(stream);
}

namespace {

#define AGF2_BLAS(call)                                                     \
  do {                                                                      \
    rocblas_status s_ = (call);                                             \
    if (s_ != rocblas_status_success)                                       \
      throw ::agf2::Error{AGF2_ERR_HIP, std::string(#call) + ": " +         \
                                            rocblas_status_to_string(s_)};  \
  } while (0)

double* host_scratch(Handle& h, size_t n) {
  if (n > h.host_red_n) {
    if (h.host_red) AGF2_HIP(hipHostFree(h.host_red));
    h.host_red = nullptr;
    AGF2_HIP(hipHostMalloc(reinterpret_cast<void**>(&h.host_red), n * sizeof(double)));
    h.host_red_n = n;
  }
  return h.host_red;
}

int read_info(Handle& h, const int* d_info) {
  int info = 0;
  AGF2_HIP(hipMemcpyAsync(&info, d_info, sizeof(int), hipMemcpyDeviceToHost, h.stream));
  AGF2_HIP(hipStreamSynchronize(h.stream));
  return info;
}

// ------------------------------------------------------------ small kernels

__global__ void zero_colmajor_upper(int N, double* A) {
  const long tot = (long)N * N;
  for (long idx = blockIdx.x * (long)blockDim.x + threadIdx.x; idx < tot;
       idx += (long)gridDim.x * blockDim.x) {
    const int i = (int)(idx % N), j = (int)(idx / N);   // A(i, j) at i + j N
    if (i < j) A[idx] = 0.0;
  }
}

// M[c][d] *= 1/sqrt(s_c s_d) (k x k);  S(p, c) = Z(p, off+c) sqrt(s_{off+c})
__global__ void eig_sqrt_scale(int N, int k, int off, const double* s, double* M,
                               const double* Z, double* S) {
  const long tk = (long)k * k, tn = (long)N * k;
  for (long idx = blockIdx.x * (long)blockDim.x + threadIdx.x; idx < tk + tn;
       idx += (long)gridDim.x * blockDim.x) {
    if (idx < tk) {
      const int c = (int)(idx / k), d = (int)(idx % k);
      M[idx] /= sqrt(s[off + c] * s[off + d]);
    } else {
      const long j = idx - tk;
      const int c = (int)(j / N), p = (int)(j % N);
      S[j] = Z[(long)(off + c) * N + p] * sqrt(s[off + c]);
    }
  }
}

// per-block partials of  sum_{l<nl, k<nk} c[l][k]^2 / (sgn * (el[l] - ek[k]))
__global__ __launch_bounds__(256) void gm_sum_kernel(int nl, int nk, const double* c,
                                                     const double* el, const double* ek,
                                                     double sgn, double* part) {
  __shared__ double red[256];
  const long tot = (long)nl * nk;
  double acc = 0.0;
  for (long idx = blockIdx.x * 256L + threadIdx.x; idx < tot; idx += (long)gridDim.x * 256) {
    const int l = (int)(idx / nk), k = (int)(idx % nk);
    const double x = c[idx];
    acc += x * x / (sgn * (el[l] - ek[k]));
  }
  red[threadIdx.x] = acc;
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if (threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
    __syncthreads();
  }
  if (threadIdx.x == 0) part[blockIdx.x] = red[0];
}

// per-block partials of 1/2 sum (h + F) * D
__global__ __launch_bounds__(256) void e1b_kernel(long n, const double* hc, const double* F,
                                                  const double* D, double* part) {
  __shared__ double red[256];
  double acc = 0.0;
  for (long i = blockIdx.x * 256L + threadIdx.x; i < n; i += (long)gridDim.x * 256)
    acc += (hc[i] + F[i]) * D[i];
  red[threadIdx.x] = acc;
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if (threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
    __syncthreads();
  }
  if (threadIdx.x == 0) part[blockIdx.x] = 0.5 * red[0];
}

__global__ void sqdiff_kernel(long n, const double* a, const double* b, double* out) {
  for (long i = blockIdx.x * (long)blockDim.x + threadIdx.x; i < n;
       i += (long)gridDim.x * blockDim.x)
    out[i] = a[i] - b[i];
}

// M[i][j] = P[i][j] / (lam[no + j] - lam[i]) over the occupied x virtual poles
__global__ void newton_weights_kernel(long n, int nv, int no, const double* P,
                                      const double* lam, double* M) {
  for (long k = blockIdx.x * (long)blockDim.x + threadIdx.x; k < n;
       k += (long)gridDim.x * blockDim.x) {
    const int i = (int)(k / nv), j = (int)(k % nv);
    M[k] = P[k] / (lam[no + j] - lam[i]);
  }
}

// D[x][y] += a (G[x][y] + G[y][x])
__global__ void add_sym_kernel(int N, double a, const double* G, double* D) {
  const long nn = (long)N * N;
  for (long k = blockIdx.x * (long)blockDim.x + threadIdx.x; k < nn;
       k += (long)gridDim.x * blockDim.x) {
    const int x = (int)(k / N), y = (int)(k % N);
    D[k] += a * (G[k] + G[(long)y * N + x]);
  }
}

__global__ void add_scalar_kernel(long n, double d, double* x) {
  for (long i = blockIdx.x * (long)blockDim.x + threadIdx.x; i < n;
       i += (long)gridDim.x * blockDim.x)
    x[i] += d;
}

inline int nblk(long n) { return (int)std::max<long>(1, std::min<long>((n + 255) / 256, 4096)); }

double reduce_partials(Handle& h, const double* part, int nb) {
  double* hp = host_scratch(h, std::max<size_t>(nb, 4096));
  AGF2_HIP(hipMemcpyAsync(hp, part, nb * sizeof(double), hipMemcpyDeviceToHost, h.stream));
  AGF2_HIP(hipStreamSynchronize(h.stream));
  double s = 0.0;
  for (int i = 0; i < nb; ++i) s += hp[i];
  return s;
}

// ------------------------------------------------------------ compression

int compress_impl(Handle& h, int N, const double* m0, const double* m1, double tol,
                  double* e_aux, double* v_aux) {
  hipStream_t st = h.stream;
  const long nn = (long)N * N;
  ProfScope ps(h, "compress", 12.0 * (double)nn * N, 8.0 * 6.0 * nn);
  double* A = h.ws_misc[0].as<double>(nn);
  double* B = h.ws_misc[1].as<double>(nn);
  double* E = h.ws_misc[2].as<double>(2L * N + 8);
  int* info = reinterpret_cast<int*>(E + 2L * N);
  AGF2_HIP(hipMemcpyAsync(A, m0, nn * sizeof(double), hipMemcpyDeviceToDevice, st));
  AGF2_HIP(hipMemcpyAsync(B, m1, nn * sizeof(double), hipMemcpyDeviceToDevice, st));
  if (tol == 0.0) {
    // column-major view: A = Lc Lc^T with Lc lower
    AGF2_BLAS(rocsolver_dpotrf(h.blas, rocblas_fill_lower, N, A, N, info));
    const int inf = read_info(h, info);
    if (inf != 0)
      throw Error{AGF2_ERR_NOT_PD, "zeroth moment is not positive definite (Cholesky pivot " +
                                       std::to_string(inf) + ")"};
    hipLaunchKernelGGL(zero_colmajor_upper, dim3(nblk(nn)), dim3(256), 0, st, N, A);
    AGF2_CHECK_LAUNCH();
    const double one = 1.0;
    AGF2_BLAS(rocblas_dtrsm(h.blas, rocblas_side_left, rocblas_fill_lower,
                            rocblas_operation_none, rocblas_diagonal_non_unit, N, N, &one, A, N,
                            B, N));
    AGF2_BLAS(rocblas_dtrsm(h.blas, rocblas_side_right, rocblas_fill_lower,
                            rocblas_operation_transpose, rocblas_diagonal_non_unit, N, N, &one,
                            A, N, B, N));
    symmetrize_f64(N, B, st);
    AGF2_BLAS(rocsolver_dsyevd(h.blas, rocblas_evect_original, rocblas_fill_lower, N, B, N,
                               e_aux, E, info));
    if (read_info(h, info) != 0) throw Error{AGF2_ERR_HIP, "syevd failed in compression"};
    // v_aux[p][k] = sum_j Lc(p, j) W(j, k)
    Gemm g;
    g.M = N; g.N = N; g.K = N;
    g.A = A; g.sAm = 1; g.sAk = N;
    g.B = B; g.sBk = 1; g.sBn = N;
    g.C = v_aux; g.sCm = N; g.sCn = 1;
    gemm_f64(g, st);
    return N;
  }
  // eigen square root of m0 keeping s > tol * s_max
  AGF2_BLAS(rocsolver_dsyevd(h.blas, rocblas_evect_original, rocblas_fill_lower, N, A, N, E,
                             E + N, info));
  if (read_info(h, info) != 0) throw Error{AGF2_ERR_HIP, "syevd failed in compression"};
  double* hs = host_scratch(h, N);
  AGF2_HIP(hipMemcpyAsync(hs, E, N * sizeof(double), hipMemcpyDeviceToHost, st));
  AGF2_HIP(hipStreamSynchronize(st));
  const double smax = hs[N - 1];
  int k = 0;
  for (int i = N - 1; i >= 0 && hs[i] > tol * smax && smax > 0.0; --i) ++k;
  if (k == 0) throw Error{AGF2_ERR_NOT_PD, "zeroth moment has no positive eigenvalue"};
  const int off = N - k;
  double* T1 = h.ws_misc[3].as<double>((long)N * k);
  double* M = h.ws_misc[4].as<double>((long)k * k);
  double* S = h.ws_misc[5].as<double>((long)N * k);
  // T1[p][c] = sum_r m1[p][r] Z(r, off + c)
  Gemm g1;
  g1.M = N; g1.N = k; g1.K = N;
  g1.A = B; g1.sAm = N; g1.sAk = 1;
  g1.B = A + (long)off * N; g1.sBk = 1; g1.sBn = N;
  g1.C = T1; g1.sCm = k; g1.sCn = 1;
  gemm_f64(g1, st);
  // M[c][d] = sum_p Z(p, off + c) T1[p][d]
  Gemm g2;
  g2.M = k; g2.N = k; g2.K = N;
  g2.A = A + (long)off * N; g2.sAm = N; g2.sAk = 1;
  g2.B = T1; g2.sBk = k; g2.sBn = 1;
  g2.C = M; g2.sCm = k; g2.sCn = 1;
  gemm_f64(g2, st);
  hipLaunchKernelGGL(eig_sqrt_scale, dim3(nblk((long)k * k + (long)N * k)), dim3(256), 0, st,
                     N, k, off, E, M, A, S);
  AGF2_CHECK_LAUNCH();
  symmetrize_f64(k, M, st);
  AGF2_HIP(hipMemsetAsync(e_aux, 0, N * sizeof(double), st));
  AGF2_HIP(hipMemsetAsync(v_aux, 0, nn * sizeof(double), st));
  AGF2_BLAS(rocsolver_dsyevd(h.blas, rocblas_evect_original, rocblas_fill_lower, k, M, k,
                             e_aux, E + N, info));
  if (read_info(h, info) != 0) throw Error{AGF2_ERR_HIP, "syevd failed in compression"};
  // v[p][c'] = sum_c S(p, c) W(c, c')
  Gemm g3;
  g3.M = N; g3.N = k; g3.K = k;
  g3.A = S; g3.sAm = 1; g3.sAk = N;
  g3.B = M; g3.sBk = 1; g3.sBn = k;
  g3.C = v_aux; g3.sCm = N; g3.sCn = 1;
  gemm_f64(g3, st);
  return k;
}

// ------------------------------------------------------- Lanczos blocks

// I (N x N)
__global__ void set_identity(int N, double* A) {
  const long nn = (long)N * N;
  for (long i = blockIdx.x * (long)blockDim.x + threadIdx.x; i < nn;
       i += (long)gridDim.x * blockDim.x)
    A[i] = (i / N == i % N) ? 1.0 : 0.0;
}

// column-major n x n T: block at (r0, c0) = src (N x N, column-major) or its
// transpose
__global__ void put_block(int n, double* T, int r0, int c0, int N, const double* src,
                          int trans) {
  const long nn = (long)N * N;
  for (long i = blockIdx.x * (long)blockDim.x + threadIdx.x; i < nn;
       i += (long)gridDim.x * blockDim.x) {
    const int r = (int)(i % N), c = (int)(i / N);
    T[(long)(r0 + r) + (long)(c0 + c) * n] = trans ? src[(long)c + (long)r * N] : src[i];
  }
}

}  // namespace

// Compression of one part to nb blocks of block Lanczos from its moments
// m[0 .. 2nb-1] (compression section, more than one block). Column-major
// throughout (the symmetric inputs read the same either way):
//   Lc Lc^T = T(0); M(n) = Lc^-1 T(n) Lc^-T, M(0) = I;
//   Lanczos vectors as matrix polynomials Q_j = sum_m H^m Q_0 C_j[m], so
//   <Q_i|H^p|Q_j> = sum_{m,l} C_i[m]^T M(m+l+p) C_j[l];
//   A_j = <Q_j|H|Q_j>; R = H Q_{j-1} - Q_{j-1} A_{j-1} - Q_{j-2} B_{j-1}^T;
//   Lg Lg^T = <R|R>, B_j = Lg^T, C_j = R Lg^-T;
//   T = blocks A_j on the diagonal, B_j below, B_j^T above; T = W e W^T;
//   v_aux = Lc W[0:N] (row-major [N][nb N]), e_aux = e.
int compress_lanczos_impl(Handle& h, int N, int nb, const double* m, double* e_aux,
                          double* v_aux) {
  const long nn = (long)N * N;
  if (nb == 1) return compress_impl(h, N, m, m + nn, 0.0, e_aux, v_aux);
  hipStream_t st = h.stream;
  const int nm = 2 * nb, n = nb * N;
  const long ncoef = (long)nb * (nb + 1) / 2;
  ProfScope ps(h, "compress", (4.0 * nb * nb * nb + 2.0 * nm) * (double)nn * N +
                                  9.0 * (double)n * n * n,
               8.0 * (nm + 2.0 * nb) * nn);
  double* Lc = h.ws_misc[0].as<double>(nn);
  double* M = h.ws_misc[1].as<double>(nm * nn);
  double* C = h.ws_misc[3].as<double>(ncoef * nn);   // C_j[m] at (j(j+1)/2 + m) nn
  double* R = h.ws_misc[4].as<double>((long)nb * nn);
  double* A = h.ws_misc[5].as<double>(2L * nb * nn);   // A_j, then Lg_j
  double* Lg = A + (long)nb * nn;
  double* tmp = h.ws_misc[6].as<double>(2 * nn);
  double* T = h.ws_misc[7].as<double>((long)n * n + 2L * n + 8);
  double* E = T + (long)n * n;
  int* info = reinterpret_cast<int*>(E + 2L * n);
  auto coef = [&](int j, int k) { return C + ((long)j * (j + 1) / 2 + k) * nn; };
  auto mm = [&](double* Cm, const double* Am, bool ta, const double* Bm, bool tb, double alpha,
                double beta) {
    Gemm g;
    g.M = N; g.N = N; g.K = N;
    g.A = Am; g.sAm = ta ? N : 1; g.sAk = ta ? 1 : N;
    g.B = Bm; g.sBk = tb ? N : 1; g.sBn = tb ? 1 : N;
    g.C = Cm; g.sCm = 1; g.sCn = N;
    g.alpha = alpha; g.beta = beta;
    gemm_f64(g, st);
  };
  const double one = 1.0;
  // Cholesky factor of T(0)
  AGF2_HIP(hipMemcpyAsync(Lc, m, nn * sizeof(double), hipMemcpyDeviceToDevice, st));
  AGF2_BLAS(rocsolver_dpotrf(h.blas, rocblas_fill_lower, N, Lc, N, info));
  if (const int inf = read_info(h, info))
    throw Error{AGF2_ERR_NOT_PD, "zeroth moment is not positive definite (Cholesky pivot " +
                                     std::to_string(inf) + ")"};
  hipLaunchKernelGGL(zero_colmajor_upper, dim3(nblk(nn)), dim3(256), 0, st, N, Lc);
  AGF2_CHECK_LAUNCH();
  // orthonormalised moments
  hipLaunchKernelGGL(set_identity, dim3(nblk(nn)), dim3(256), 0, st, N, M);
  AGF2_CHECK_LAUNCH();
  for (int k = 1; k < nm; ++k) {
    double* Mk = M + k * nn;
    AGF2_HIP(hipMemcpyAsync(Mk, m + k * nn, nn * sizeof(double), hipMemcpyDeviceToDevice, st));
    AGF2_BLAS(rocblas_dtrsm(h.blas, rocblas_side_left, rocblas_fill_lower,
                            rocblas_operation_none, rocblas_diagonal_non_unit, N, N, &one, Lc, N,
                            Mk, N));
    AGF2_BLAS(rocblas_dtrsm(h.blas, rocblas_side_right, rocblas_fill_lower,
                            rocblas_operation_transpose, rocblas_diagonal_non_unit, N, N, &one,
                            Lc, N, Mk, N));
    symmetrize_f64(N, Mk, st);
  }
  // out = sum_{a<ni, b<nj} Ci[a]^T M(a+b+p) Cj[b]
  auto inner = [&](const double* Ci, int ni, const double* Cj, int nj, int p, double* out) {
    for (int a = 0; a < ni; ++a) {
      for (int b = 0; b < nj; ++b)
        mm(tmp, M + (a + b + p) * nn, false, Cj + b * nn, false, 1.0, b == 0 ? 0.0 : 1.0);
      mm(out, Ci + a * nn, true, tmp, false, 1.0, a == 0 ? 0.0 : 1.0);
    }
    symmetrize_f64(N, out, st);
  };
  hipLaunchKernelGGL(set_identity, dim3(nblk(nn)), dim3(256), 0, st, N, coef(0, 0));
  AGF2_CHECK_LAUNCH();
  inner(coef(0, 0), 1, coef(0, 0), 1, 1, A);
  for (int j = 1; j < nb; ++j) {
    // coefficients of R = H Q_{j-1} - Q_{j-1} A_{j-1} - Q_{j-2} B_{j-1}^T
    fill_zero(R, (long)(j + 1) * nn, st);
    for (int k = 0; k < j; ++k) {
      axpby_f64(nn, 1.0, coef(j - 1, k), 1.0, R + (k + 1) * nn, st);
      mm(R + k * nn, coef(j - 1, k), false, A + (long)(j - 1) * nn, false, -1.0, 1.0);
    }
    if (j >= 2)   // B_{j-1}^T = Lg_{j-1}
      for (int k = 0; k < j - 1; ++k)
        mm(R + k * nn, coef(j - 2, k), false, Lg + (long)(j - 1) * nn, false, -1.0, 1.0);
    double* L_j = Lg + (long)j * nn;
    inner(R, j + 1, R, j + 1, 0, L_j);
    AGF2_BLAS(rocsolver_dpotrf(h.blas, rocblas_fill_lower, N, L_j, N, info));
    if (const int inf = read_info(h, info))
      throw Error{AGF2_ERR_NOT_PD, "Lanczos block " + std::to_string(j) +
                                       " is not positive definite (Cholesky pivot " +
                                       std::to_string(inf) + ")"};
    hipLaunchKernelGGL(zero_colmajor_upper, dim3(nblk(nn)), dim3(256), 0, st, N, L_j);
    AGF2_CHECK_LAUNCH();
    for (int k = 0; k <= j; ++k) {
      AGF2_BLAS(rocblas_dtrsm(h.blas, rocblas_side_right, rocblas_fill_lower,
                              rocblas_operation_transpose, rocblas_diagonal_non_unit, N, N, &one,
                              L_j, N, R + k * nn, N));
      AGF2_HIP(hipMemcpyAsync(coef(j, k), R + k * nn, nn * sizeof(double),
                              hipMemcpyDeviceToDevice, st));
    }
    inner(coef(j, 0), j + 1, coef(j, 0), j + 1, 1, A + (long)j * nn);
  }
  // block tridiagonal matrix and its eigendecomposition
  fill_zero(T, (long)n * n, st);
  for (int j = 0; j < nb; ++j) {
    hipLaunchKernelGGL(put_block, dim3(nblk(nn)), dim3(256), 0, st, n, T, j * N, j * N, N,
                       A + (long)j * nn, 0);
    if (j > 0) {
      // below: B_j = Lg_j^T; above: B_j^T = Lg_j
      hipLaunchKernelGGL(put_block, dim3(nblk(nn)), dim3(256), 0, st, n, T, j * N, (j - 1) * N,
                         N, Lg + (long)j * nn, 1);
      hipLaunchKernelGGL(put_block, dim3(nblk(nn)), dim3(256), 0, st, n, T, (j - 1) * N, j * N,
                         N, Lg + (long)j * nn, 0);
    }
    AGF2_CHECK_LAUNCH();
  }
  AGF2_BLAS(rocsolver_dsyevd(h.blas, rocblas_evect_original, rocblas_fill_lower, n, T, n, e_aux,
                             E, info));
  if (read_info(h, info) != 0) throw Error{AGF2_ERR_HIP, "syevd failed in compression"};
  // v_aux[p][k] = sum_j Lc(p, j) W(j, k)
  Gemm g;
  g.M = N; g.N = n; g.K = N;
  g.A = Lc; g.sAm = 1; g.sAk = N;
  g.B = T; g.sBk = 1; g.sBn = n;
  g.C = v_aux; g.sCm = n; g.sCn = 1;
  gemm_f64(g, st);
  return n;
}

namespace {

// ------------------------------------------------------------ Fock loop

struct Aufbau {
  int n = 0;
  double count = 0.0;
  double mu = 0.0;
};

// Fill poles in ascending energy with 2|u_l|^2 electrons each; n* minimises
// |c_n - nelec| (first minimum -> smaller n on ties); mu midway.
Aufbau aufbau(int npole, const double* lam, const double* w, double nelec) {
  Aufbau a;
  double c = 0.0, best = std::fabs(0.0 - nelec);
  a.n = 0; a.count = 0.0;
  for (int n = 1; n <= npole; ++n) {
    c += 2.0 * w[n - 1];
    const double d = std::fabs(c - nelec);
    if (d < best) { best = d; a.n = n; a.count = c; }
  }
  if (a.n > 0 && a.n < npole) a.mu = 0.5 * (lam[a.n - 1] + lam[a.n]);
  else if (a.n == 0) a.mu = lam[0] - 1.0;
  else a.mu = lam[npole - 1] + 1.0;
  return a;
}

struct FockLoop {
  Handle& h;
  int N, Q, naux, n;
  const double* L; const double* e; const double* v;
  double nelec;
  double* H; double* lam; double* work; int* info; double* w;
  // host copies of the eigenvalues and pole weights of the last solve, in a
  // buffer of the loop's own (not the handle's shared scratch, which other
  // calls may reallocate)
  std::vector<double> hbuf;
  double* hlam; double* hw;
  double solved_shift = NAN;
  const double* solved_F = nullptr;
  double last_change = 0.0;   // |shift change| of the previous fit
  int n_eig = 0;

  FockLoop(Handle& hh, int N_, int Q_, int naux_, const double* L_, const double* e_,
           const double* v_, double nelec_)
      : h(hh), N(N_), Q(Q_), naux(naux_), n(N_ + naux_), L(L_), e(e_), v(v_), nelec(nelec_) {
    H = h.ws_fock[4].as<double>((long)n * n);
    lam = h.ws_fock[5].as<double>(3L * n + 8);
    work = lam + n;
    w = lam + 2L * n;
    info = reinterpret_cast<int*>(lam + 3L * n);
    hbuf.assign(2L * n, 0.0);
    hlam = hbuf.data();
    hw = hlam + n;
  }

  // eigendecomposition of the extended Hamiltonian at `shift`; host copies of
  // the eigenvalues and physical weights; returns the aufbau.
  Aufbau solve(const double* F, double shift) {
    hipStream_t st = h.stream;
    build_hext(N, naux, F, e, v, shift, H, st);
    {
      // nominal flop count of a symmetric eigendecomposition with vectors
      ProfScope ps(h, "fock.syevd", 9.0 * (double)n * n * n, 8.0 * 2.0 * n * n);
      AGF2_BLAS(rocsolver_dsyevd(h.blas, rocblas_evect_original, rocblas_fill_lower, n, H, n,
                                 lam, work, info));
    }
    column_weights(N, n, H, w, st);
    AGF2_HIP(hipMemcpyAsync(hlam, lam, n * sizeof(double), hipMemcpyDeviceToHost, st));
    AGF2_HIP(hipMemcpyAsync(hw, w, n * sizeof(double), hipMemcpyDeviceToHost, st));
    int inf = 0;
    AGF2_HIP(hipMemcpyAsync(&inf, info, sizeof(int), hipMemcpyDeviceToHost, st));
    AGF2_HIP(hipStreamSynchronize(st));
    if (inf != 0) throw Error{AGF2_ERR_HIP, "syevd failed on the extended Hamiltonian"};
    ++n_eig;
    solved_shift = shift;
    solved_F = F;
    return aufbau(n, hlam, hw, nelec);
  }

  // the last eigendecomposition no longer belongs to the contents of F
  void invalidate() { solved_F = nullptr; solved_shift = NAN; }

  // Newton step -g0 / (dN/dDelta) at the last eigendecomposition, from the
  // first-order response to the common auxiliary shift (eigenvectors l = rows
  // of the row-major view of H, physical part = first N columns):
  //   P = C_o^T C_v, M_ij = P_ij / (lam_j - lam_i), dN/dDelta = 4 sum M.P.
  // NAN when the derivative is not positive and finite; leaves P and M in the
  // workspace.
  double newton_step(int no, double g0) {
    const int nv = n - no;
    if (no <= 0 || nv <= 0) return NAN;
    hipStream_t st = h.stream;
    const long ov = (long)no * nv;
    double* P = h.ws_fock[1].as<double>(2 * ov + (long)N * nv + (long)N * N);
    double* M = P + ov;
    Gemm g;
    g.M = no; g.N = nv; g.K = N;
    g.A = H; g.sAm = n; g.sAk = 1;
    g.B = H + (long)no * n; g.sBk = 1; g.sBn = n;
    g.C = P; g.sCm = nv; g.sCn = 1;
    gemm_f64(g, st);
    hipLaunchKernelGGL(newton_weights_kernel, dim3(nblk(ov)), dim3(256), 0, st, ov, nv, no, P,
                       lam, M);
    AGF2_CHECK_LAUNCH();
    const double dN = 4.0 * dot_f64(h, ov, M, P);
    // an occupied and a virtual pole at the same energy make M infinite:
    // no step then (the caller falls back to the bracketing fit)
    return (dN > 0.0 && std::isfinite(dN)) ? -g0 / dN : NAN;
  }

  // If the Newton step is at most max_step, adds step x dD/dDelta to D (the
  // exact density at the last solve), with dD/dDelta = 2 (G + G^T) and
  // G = C_o M C_v^T, and returns the step; otherwise returns NAN and leaves D
  // alone.
  double first_order(int no, double g0, double max_step, double* D) {
    const double step = newton_step(no, g0);
    if (!(std::fabs(step) <= max_step)) return NAN;
    hipStream_t st = h.stream;
    const int nv = n - no;
    const long ov = (long)no * nv;
    double* P = h.ws_fock[1].as<double>(2 * ov + (long)N * nv + (long)N * N);
    double* M = P + ov;
    double* T = M + ov;
    double* G = T + (long)N * nv;
    Gemm t;
    t.M = N; t.N = nv; t.K = no;
    t.A = H; t.sAm = 1; t.sAk = n;
    t.B = M; t.sBk = nv; t.sBn = 1;
    t.C = T; t.sCm = nv; t.sCn = 1;
    gemm_f64(t, st);
    Gemm u;
    u.M = N; u.N = N; u.K = nv;
    u.A = T; u.sAm = nv; u.sAk = 1;
    u.B = H + (long)no * n; u.sBk = n; u.sBn = 1;
    u.C = G; u.sCm = N; u.sCn = 1;
    gemm_f64(u, st);
    hipLaunchKernelGGL(add_sym_kernel, dim3(nblk((long)N * N)), dim3(256), 0, st, N,
                       2.0 * step, G, D);
    AGF2_CHECK_LAUNCH();
    return step;
  }

  double count_n(int nocc) const {
    double c = 0.0;
    for (int l = 0; l < nocc; ++l) c += 2.0 * hw[l];
    return c;
  }

  // common shift of the auxiliary energies giving the right electron count:
  // bracket by doubling steps, then Illinois regula falsi (count is
  // non-decreasing in the shift for a fixed number of occupied poles).
  double fit_shift(const double* F, double shift0, const agf2_fock_opts& o, double tol) {
    Aufbau a = (solved_shift == shift0 && solved_F == F) ? aufbau(n, hlam, hw, nelec)
                                                         : solve(F, shift0);
    double shift = shift0;
    int nocc = a.n;
    double cnt = a.count;
    // Newton steps with the analytic derivative while each at least halves
    // the error at an unchanged occupied count (one eigensolve per step)
    for (int it = 0; it < 8; ++it) {
      const double g0 = cnt - nelec;
      if (std::fabs(g0) < tol) return shift;
      const double step = newton_step(nocc, g0);
      if (!(std::fabs(step) <= o.bracket)) break;
      const Aufbau an = solve(F, shift + step);
      const double g1 = count_n(nocc) - nelec;
      if (!(std::fabs(g1) <= 0.5 * std::fabs(g0))) break;   // (solve kept; bracketing re-solves)
      last_change = std::fabs(step);
      shift += step;
      nocc = an.n;
      cnt = an.count;
    }
    for (int rep = 0; rep < 8; ++rep) {
      const double g0 = cnt - nelec;
      if (std::fabs(g0) < tol) return shift;
      auto g = [&](double d) {
        solve(F, d);
        return count_n(nocc) - nelec;
      };
      const double dir = g0 < 0 ? 1.0 : -1.0;
      // first bracket step: four times the previous fit's change of the shift
      // (the change shrinks from one density cycle to the next), never more
      // than step0; a miss costs a doubling
      double step = o.step0;
      if (last_change > 0.0) step = std::min(o.step0, std::max(4.0 * last_change, 1e-7));
      double a_ = shift, ga = g0, b = a_, gb = ga;
      while (true) {
        b = shift + dir * std::min(step, o.bracket);
        gb = g(b);
        if (gb == 0.0 || (gb > 0) != (ga > 0) || step >= o.bracket) break;
        a_ = b; ga = gb;
        step *= 2.0;
      }
      double x = b;
      if (!((gb > 0) == (ga > 0) && gb != 0.0)) {
        int side = 0;
        for (int it = 0; it < 100; ++it) {
          if (gb == 0.0) { x = b; break; }
          x = b - gb * (b - a_) / (gb - ga);
          const double gx = g(x);
          if (std::fabs(gx) < tol) break;
          if ((gx > 0) == (gb > 0)) {
            b = x; gb = gx;
            if (side == -1) ga *= 0.5;
            side = -1;
          } else {
            a_ = b; ga = gb;
            b = x; gb = gx;
            side = +1;
          }
        }
      }
      last_change = std::fabs(x - shift);
      shift = x;
      // the last count was evaluated at x: reuse that eigendecomposition
      Aufbau an = (solved_shift == shift && solved_F == F) ? aufbau(n, hlam, hw, nelec)
                                                           : solve(F, shift);
      cnt = an.count;
      if (an.n == nocc) return shift;
      nocc = an.n;
    }
    return shift;
  }
};

// largest shift step the Fock loop takes to first order instead of refitting
constexpr double kNewtonMax = 1e-3;

// tiny dense solve (partial pivoting) for DIIS
bool solve_small(int n, std::vector<double> A, std::vector<double>& b) {
  for (int c = 0; c < n; ++c) {
    int piv = c;
    for (int r = c + 1; r < n; ++r)
      if (std::fabs(A[r * n + c]) > std::fabs(A[piv * n + c])) piv = r;
    if (A[piv * n + c] == 0.0) return false;
    if (piv != c) {
      for (int k = 0; k < n; ++k) std::swap(A[c * n + k], A[piv * n + k]);
      std::swap(b[c], b[piv]);
    }
    for (int r = c + 1; r < n; ++r) {
      const double f = A[r * n + c] / A[c * n + c];
      for (int k = c; k < n; ++k) A[r * n + k] -= f * A[c * n + k];
      b[r] -= f * b[c];
    }
  }
  for (int r = n - 1; r >= 0; --r) {
    double s = b[r];
    for (int k = r + 1; k < n; ++k) s -= A[r * n + k] * b[k];
    b[r] = s / A[r * n + r];
  }
  return true;
}

}  // namespace

// DIIS over device vectors: x = sum_k c_k x_k minimising |sum_k c_k e_k| with
// sum_k c_k = 1.
struct Diis {
  Handle& h;
  long len;
  int space;
  double* store;           // [space][2][len]: x then e
  std::vector<int> order;  // slots, oldest first
  std::vector<double> B;   // space x space overlaps by slot
  Diis(Handle& hh, long len_, int space_, DevBuf& buf)
      : h(hh), len(len_), space(space_), B((size_t)space_ * space_, 0.0) {
    store = buf.as<double>((long)std::max(space_, 1) * 2 * len_);
  }
  // x (in/out), e: error vector of x
  void update(double* x, const double* e) {
    if (space <= 0) return;
    int slot;
    if ((int)order.size() < space) {
      slot = (int)order.size();
    } else {
      slot = order.front();
      order.erase(order.begin());
    }
    order.push_back(slot);
    double* xs = store + (long)slot * 2 * len;
    double* es = xs + len;
    AGF2_HIP(hipMemcpyAsync(xs, x, len * sizeof(double), hipMemcpyDeviceToDevice, h.stream));
    AGF2_HIP(hipMemcpyAsync(es, e, len * sizeof(double), hipMemcpyDeviceToDevice, h.stream));
    for (int o : order) {
      const double d = dot_f64(h, len, es, store + (long)o * 2 * len + len);
      B[slot * space + o] = B[o * space + slot] = d;
    }
    const int n = (int)order.size();
    if (n < 2) return;
    std::vector<double> A((size_t)(n + 1) * (n + 1), 0.0), rhs(n + 1, 0.0);
    for (int a = 0; a < n; ++a)
      for (int b = 0; b < n; ++b) A[a * (n + 1) + b] = B[order[a] * space + order[b]];
    for (int a = 0; a < n; ++a) A[n * (n + 1) + a] = A[a * (n + 1) + n] = -1.0;
    rhs[n] = -1.0;
    if (!solve_small(n + 1, A, rhs)) return;
    for (int a = 0; a < n; ++a)
      axpby_f64(len, rhs[a], store + (long)order[a] * 2 * len, a == 0 ? 0.0 : 1.0, x,
                h.stream);
  }
};


FockLoopResult fock_loop_impl(Handle& h, int nphys, int naux, const double* Lpq,
                              const double* hcore, int nelec, int naux_se, double* e_se,
                              const double* v_se, double* rdm1, double* fock, double* e_pole,
                              double* u_pole, const agf2_fock_opts& o) {
  if (nelec <= 0 || nelec % 2 != 0 || nelec >= 2 * (nphys + naux_se))
    throw Error{AGF2_ERR_NELEC, "nelec must be even and in (0, 2 * npole)"};
  AGF2_REQUIRE(o.max_cycle >= 1 && o.tol_rdm1 > 0 && o.tol_nelec > 0 && o.bracket > 0 &&
                   o.step0 > 0 && o.diis_space >= 0,
               "bad Fock-loop options");
  hipStream_t s = h.stream;
  const int N = nphys;
  const long nn = (long)N * N;
  FockLoop fl(h, N, naux, naux_se, Lpq, e_se, v_se, (double)nelec);
  double* F = h.ws_fock[6].as<double>(3 * nn);
  double* Fn = F + nn;
  double* Dn = Fn + nn;
  Diis diis(h, nn, o.diis_space, h.ws_fock[7]);
  fock_build(h, N, naux, Lpq, hcore, rdm1, 1.0, F);
  double d = 0.0;
  bool converged = false;
  int cycle = 0;
  Aufbau a;
  double err_prev = INFINITY;
  // D = 2 sum_{l < n*} phi_l phi_l^T (physical block) of the last solve into Dn
  auto density = [&]() {
    a = aufbau(fl.n, fl.hlam, fl.hw, (double)nelec);
    Gemm g;
    g.M = N; g.N = N; g.K = a.n;
    g.A = fl.H; g.sAm = 1; g.sAk = fl.n;
    g.B = fl.H; g.sBn = 1; g.sBk = fl.n;
    g.C = Dn; g.sCm = N; g.sCn = 1; g.alpha = 2.0;
    if (a.n > 0) gemm_f64(g, s);
    else AGF2_HIP(hipMemsetAsync(Dn, 0, nn * sizeof(double), s));
  };
  // fit the shift at F to tolerance tol, then the density at the fitted shift
  auto fit_and_density = [&](double tol) {
    d = fl.fit_shift(F, d, o, tol);
    if (!(fl.solved_shift == d && fl.solved_F == F)) fl.solve(F, d);
    density();
  };
  for (cycle = 1; cycle <= o.max_cycle; ++cycle) {
    // the electron count is fitted to tol_nelec once the density has
    // settled; earlier cycles, whose density is still moving, to 0.01 x its
    // last change (at most 1e-6)
    const double tol_c = std::max(o.tol_nelec, std::min(1e-6, 1e-2 * err_prev));
    // Solve at the current shift. If the count misses tol_c by a Newton step
    // of at most kNewtonMax, take that step and the density to first order in
    // it (no further eigensolve); otherwise fit the shift to tol_c.
    bool first_order = false;
    {
      const Aufbau a0 = (fl.solved_shift == d && fl.solved_F == F)
                            ? aufbau(fl.n, fl.hlam, fl.hw, (double)nelec)
                            : fl.solve(F, d);
      const double g0 = a0.count - (double)nelec;
      if (std::fabs(g0) < tol_c) {
        density();
      } else {
        density();
        const double step = fl.first_order(a0.n, g0, kNewtonMax, Dn);
        if (std::isfinite(step)) {
          d += step;
          fl.last_change = std::fabs(step);
          first_order = true;
        } else {
          fit_and_density(tol_c);
        }
      }
    }
    // Frobenius norm of the change of D
    hipLaunchKernelGGL(sqdiff_kernel, dim3(nblk(nn)), dim3(256), 0, s, nn, Dn, rdm1, Fn);
    AGF2_CHECK_LAUNCH();
    const double err = std::sqrt(dot_f64(h, nn, Fn, Fn));
    err_prev = err;
    if (err < o.tol_rdm1) {
      // converged: the returned density is exact and meets tol_nelec (same F,
      // so no new J/K)
      if (first_order || tol_c > o.tol_nelec) fit_and_density(o.tol_nelec);
      AGF2_HIP(hipMemcpyAsync(rdm1, Dn, nn * sizeof(double), hipMemcpyDeviceToDevice, s));
      converged = true;
      break;
    }
    AGF2_HIP(hipMemcpyAsync(rdm1, Dn, nn * sizeof(double), hipMemcpyDeviceToDevice, s));
    fock_build(h, N, naux, Lpq, hcore, rdm1, 1.0, Fn);
    // error vector F[D] - F, stored in Dn (free now)
    hipLaunchKernelGGL(sqdiff_kernel, dim3(nblk(nn)), dim3(256), 0, s, nn, Fn, F, Dn);
    AGF2_CHECK_LAUNCH();
    diis.update(Fn, Dn);
    AGF2_HIP(hipMemcpyAsync(F, Fn, nn * sizeof(double), hipMemcpyDeviceToDevice, s));
    fl.invalidate();
  }
  if (!converged) {
    // cycle limit: the last F has not been diagonalised yet. Fit the shift
    // there, so that the returned poles are eigenpairs of the returned Fock
    // matrix and shifted auxiliaries, and the density is that of these poles.
    fit_and_density(o.tol_nelec);
    AGF2_HIP(hipMemcpyAsync(rdm1, Dn, nn * sizeof(double), hipMemcpyDeviceToDevice, s));
  }
  if (cycle > o.max_cycle) cycle = o.max_cycle;
  AGF2_HIP(hipMemcpyAsync(fock, F, nn * sizeof(double), hipMemcpyDeviceToDevice, s));
  AGF2_HIP(hipMemcpyAsync(e_pole, fl.lam, fl.n * sizeof(double), hipMemcpyDeviceToDevice, s));
  extract_poles(N, fl.n, fl.H, u_pole, s);
  if (naux_se > 0) {
    hipLaunchKernelGGL(add_scalar_kernel, dim3(nblk(naux_se)), dim3(256), 0, s,
                       (long)naux_se, d, e_se);
    AGF2_CHECK_LAUNCH();
  }
  AGF2_HIP(hipStreamSynchronize(s));
  FockLoopResult r;
  r.nocc_pole = a.n;
  r.mu = a.mu;
  r.shift = d;
  r.n_cycle = cycle;
  r.converged = converged;
  return r;
}

void energy_impl(Handle& h, int nphys, const double* hcore, const double* fock,
                 const double* rdm1, int npole, int nocc_pole, const double* e_pole,
                 const double* u_pole, int naux_occ, const double* e_se_occ,
                 const double* v_se_occ, int naux_vir, const double* e_se_vir,
                 const double* v_se_vir, double* e_1b, double* e_2b) {
  hipStream_t s = h.stream;
  const long nn = (long)nphys * nphys;
  double* part = h.ws_red.as<double>(4096);
  const int nb1 = nblk(nn);
  hipLaunchKernelGGL(e1b_kernel, dim3(nb1), dim3(256), 0, s, nn, hcore, fock, rdm1, part);
  AGF2_CHECK_LAUNCH();
  const double e1 = reduce_partials(h, part, nb1);
  double e2 = 0.0;
  const int nv = npole - nocc_pole;
  // occupied poles x greater auxiliaries
  if (nocc_pole > 0 && naux_vir > 0) {
    double* c = h.ws_misc[6].as<double>((long)nocc_pole * naux_vir);
    Gemm g;
    g.M = nocc_pole; g.N = naux_vir; g.K = nphys;
    g.A = u_pole; g.sAm = 1; g.sAk = npole;
    g.B = v_se_vir; g.sBn = 1; g.sBk = naux_vir;
    g.C = c; g.sCm = naux_vir; g.sCn = 1;
    gemm_f64(g, s);
    const int nb = nblk((long)nocc_pole * naux_vir);
    hipLaunchKernelGGL(gm_sum_kernel, dim3(nb), dim3(256), 0, s, nocc_pole, naux_vir, c,
                       e_pole, e_se_vir, 1.0, part);
    AGF2_CHECK_LAUNCH();
    e2 += reduce_partials(h, part, nb);
  }
  // virtual poles x lesser auxiliaries: (u_l.v_k)^2 / (e_k - lam_l)
  if (nv > 0 && naux_occ > 0) {
    double* c = h.ws_misc[6].as<double>((long)nv * naux_occ);
    Gemm g;
    g.M = nv; g.N = naux_occ; g.K = nphys;
    g.A = u_pole + nocc_pole; g.sAm = 1; g.sAk = npole;
    g.B = v_se_occ; g.sBn = 1; g.sBk = naux_occ;
    g.C = c; g.sCm = naux_occ; g.sCn = 1;
    gemm_f64(g, s);
    const int nb = nblk((long)nv * naux_occ);
    hipLaunchKernelGGL(gm_sum_kernel, dim3(nb), dim3(256), 0, s, nv, naux_occ, c,
                       e_pole + nocc_pole, e_se_occ, -1.0, part);
    AGF2_CHECK_LAUNCH();
    e2 += reduce_partials(h, part, nb);
  }
  *e_1b = e1;
  *e_2b = e2;
}

void build_moments(Handle& h, agf2_precision prec, int N, int Q, const double* L, int npole,
                   int nocc, const double* e, const double* u, double* m0o, double* m1o,
                   double* m0v, double* m1v) {
  if (prec == AGF2_FP64)
    build_moments_f64(h, N, Q, L, npole, nocc, e, u, m0o, m1o, m0v, m1v);
  else if (prec == AGF2_SPLIT_BF16 || prec == AGF2_SPLIT_FP16)
    build_moments_split(h, N, Q, L, npole, nocc, e, u, m0o, m1o, m0v, m1v,
                        prec == AGF2_SPLIT_FP16);
  else
    throw Error{AGF2_ERR_ARG, "unknown precision mode"};
}

int compress_part(Handle& h, int N, const double* m0, const double* m1, double tol,
                  double* e_aux, double* v_aux) {
  return compress_impl(h, N, m0, m1, tol, e_aux, v_aux);
}

}  // namespace agf2

using namespace agf2;

extern "C" {

void agf2_fock_opts_default(agf2_fock_opts* o) {
  if (!o) return;
  o->tol_rdm1 = 1e-8;
  o->tol_nelec = 1e-10;
  o->bracket = 2.0;
  o->step0 = 0.01;
  o->max_cycle = 50;
  o->diis_space = 8;
}

agf2_status agf2_create(agf2_handle_t* out, int device, void* stream) {
  if (!out) return AGF2_ERR_ARG;
  *out = nullptr;
  int ndev = 0;
  if (hipGetDeviceCount(&ndev) != hipSuccess || device < 0 || device >= ndev) {
    (void)hipGetLastError();
    return device < 0 ? AGF2_ERR_ARG : AGF2_ERR_HIP;
  }
  Handle* h = new (std::nothrow) Handle();
  if (!h) return AGF2_ERR_NOMEM;
  h->device = device;
  int prev = 0;
  (void)hipGetDevice(&prev);
  if (hipSetDevice(device) != hipSuccess) { delete h; return AGF2_ERR_HIP; }
  agf2_status st = AGF2_OK;
  h->stream = static_cast<hipStream_t>(stream);   // NULL: default stream
  if (st == AGF2_OK && rocblas_create_handle(&h->blas) != rocblas_status_success) st = AGF2_ERR_HIP;
  if (st == AGF2_OK && rocblas_set_stream(h->blas, h->stream) != rocblas_status_success) st = AGF2_ERR_HIP;
  if (st == AGF2_OK && hipHostMalloc(reinterpret_cast<void**>(&h->host_red), 4096 * sizeof(double)) != hipSuccess)
    st = AGF2_ERR_HIP;
  else if (st == AGF2_OK) h->host_red_n = 4096;
  if (st == AGF2_OK) {
    // the device address of the allocation-free spectral function's scratch
    try {
      (void)noalloc_scratch(device);
    } catch (const Error&) {
      st = AGF2_ERR_HIP;
    }
  }
  (void)hipSetDevice(prev);
  if (st != AGF2_OK) { delete h; return st; }
  *out = reinterpret_cast<agf2_handle_t>(h);
  return AGF2_OK;
}

agf2_status agf2_destroy(agf2_handle_t hh) {
  if (!hh) return AGF2_ERR_ARG;
  Handle* h = reinterpret_cast<Handle*>(hh);
  int prev = 0;
  (void)hipGetDevice(&prev);
  (void)hipSetDevice(h->device);
  delete h;
  (void)hipSetDevice(prev);
  return AGF2_OK;
}

const char* agf2_last_error(agf2_handle_t hh) {
  if (!hh) return "invalid (NULL) agf2 handle";
  return reinterpret_cast<Handle*>(hh)->last_error.c_str();
}

agf2_status agf2_profile_enable(agf2_handle_t hh, int enable) {
  return guarded(hh, [&](Handle& h) {
    prof_flush(h);
    if (enable) h.prof_total.clear();
    h.profiling = enable != 0;
  });
}

int agf2_profile_count(agf2_handle_t hh) {
  int n = 0;
  agf2_status st = guarded(hh, [&](Handle& h) {
    prof_flush(h);
    h.prof_names.clear();
    for (auto& kv : h.prof_total) h.prof_names.push_back(kv.first);
    n = (int)h.prof_names.size();
  });
  return st == AGF2_OK ? n : (int)st;
}

agf2_status agf2_profile_get(agf2_handle_t hh, int idx, const char** name, long* launches,
                             double* ms, double* flops, double* bytes) {
  return guarded(hh, [&](Handle& h) {
    AGF2_REQUIRE(idx >= 0 && idx < (int)h.prof_names.size(), "profile index out of range");
    AGF2_REQUIRE(name && launches && ms && flops && bytes, "NULL argument");
    const ProfTotal& t = h.prof_total[h.prof_names[idx]];
    *name = h.prof_names[idx].c_str();
    *launches = t.launches;
    *ms = t.ms;
    *flops = t.flops;
    *bytes = t.bytes;
  });
}

agf2_status agf2_synchronize(agf2_handle_t hh) {
  return guarded(hh, [&](Handle& h) { AGF2_HIP(hipStreamSynchronize(h.stream)); });
}

agf2_status agf2_build_moments(agf2_handle_t hh, agf2_precision prec, int nphys, int naux,
                               const double* Lpq, int npole, int nocc_pole,
                               const double* e_pole, const double* u_pole, double* m0_occ,
                               double* m1_occ, double* m0_vir, double* m1_vir) {
  return guarded(hh, [&](Handle& h) {
    AGF2_REQUIRE(nphys >= 1 && naux >= 1, "nphys and naux must be >= 1");
    AGF2_REQUIRE(npole >= 2 && nocc_pole >= 1 && nocc_pole < npole,
                 "need 1 <= nocc_pole < npole");
    AGF2_REQUIRE(Lpq && e_pole && u_pole && m0_occ && m1_occ && m0_vir && m1_vir,
                 "NULL array argument");
    FiniteCheck(h)
        .add(Lpq, (long)naux * nphys * nphys, "Lpq")
        .add(e_pole, npole, "e_pole")
        .add(u_pole, (long)nphys * npole, "u_pole")
        .run();
    build_moments(h, prec, nphys, naux, Lpq, npole, nocc_pole, e_pole, u_pole, m0_occ, m1_occ,
                  m0_vir, m1_vir);
  });
}

agf2_status agf2_build_moments_n(agf2_handle_t hh, agf2_precision prec, int nmom, int nphys,
                                 int naux, const double* Lpq, int npole, int nocc_pole,
                                 const double* e_pole, const double* u_pole, double* m_occ,
                                 double* m_vir) {
  return guarded(hh, [&](Handle& h) {
    AGF2_REQUIRE(nmom >= 2 && nmom % 2 == 0 && nmom <= 16, "nmom must be even, 2..16");
    AGF2_REQUIRE(nphys >= 1 && naux >= 1, "nphys and naux must be >= 1");
    AGF2_REQUIRE(npole >= 2 && nocc_pole >= 1 && nocc_pole < npole,
                 "need 1 <= nocc_pole < npole");
    AGF2_REQUIRE(Lpq && e_pole && u_pole && m_occ && m_vir, "NULL array argument");
    AGF2_REQUIRE(prec == AGF2_FP64 || nmom == 2,
                 "moments beyond the first are built in AGF2_FP64 only");
    FiniteCheck(h)
        .add(Lpq, (long)naux * nphys * nphys, "Lpq")
        .add(e_pole, npole, "e_pole")
        .add(u_pole, (long)nphys * npole, "u_pole")
        .run();
    const long nn = (long)nphys * nphys;
    if (prec != AGF2_FP64) {
      build_moments(h, prec, nphys, naux, Lpq, npole, nocc_pole, e_pole, u_pole, m_occ,
                    m_occ + nn, m_vir, m_vir + nn);
      return;
    }
    std::vector<double*> uo(nmom), uv(nmom);
    for (int k = 0; k < nmom; ++k) {
      uo[k] = m_occ + k * nn;
      uv[k] = m_vir + k * nn;
    }
    build_moments_f64_n(h, nphys, naux, Lpq, npole, nocc_pole, e_pole, u_pole, nmom / 2,
                        uo.data(), uv.data());
  });
}

agf2_status agf2_compress_lanczos(agf2_handle_t hh, int nphys, int nmom, const double* m,
                                  int* naux_out, double* e_aux, double* v_aux) {
  return guarded(hh, [&](Handle& h) {
    AGF2_REQUIRE(nphys >= 1, "nphys must be >= 1");
    AGF2_REQUIRE(nmom >= 2 && nmom % 2 == 0 && nmom <= 16, "nmom must be even, 2..16");
    AGF2_REQUIRE(m && naux_out && e_aux && v_aux, "NULL argument");
    *naux_out = 0;
    FiniteCheck(h).add(m, (long)nmom * nphys * nphys, "m").run();
    if (nmom == 2) {
      // one block: the compression itself, with v_aux's row stride nphys
      *naux_out = compress_impl(h, nphys, m, m + (long)nphys * nphys, 0.0, e_aux, v_aux);
      return;
    }
    *naux_out = compress_lanczos_impl(h, nphys, nmom / 2, m, e_aux, v_aux);
  });
}

agf2_status agf2_fock_build(agf2_handle_t hh, int nphys, int naux, const double* Lpq,
                            const double* hcore, const double* rdm1, double alpha,
                            double* fock) {
  return guarded(hh, [&](Handle& h) {
    AGF2_REQUIRE(nphys >= 1 && naux >= 1, "nphys and naux must be >= 1");
    AGF2_REQUIRE(nphys <= 46340, "nphys must be <= 46340");
    AGF2_REQUIRE(Lpq && hcore && rdm1 && fock, "NULL array argument");
    AGF2_REQUIRE(fock != hcore && fock != rdm1, "fock may not alias an input");
    const long nn = (long)nphys * nphys;
    FiniteCheck(h).add(Lpq, naux * nn, "Lpq").add(hcore, nn, "hcore").add(rdm1, nn, "rdm1").run();
    fock_build(h, nphys, naux, Lpq, hcore, rdm1, alpha, fock);
  });
}

agf2_status agf2_compress(agf2_handle_t hh, int nphys, const double* m0, const double* m1,
                          double tol, int* naux_out, double* e_aux, double* v_aux) {
  return guarded(hh, [&](Handle& h) {
    AGF2_REQUIRE(nphys >= 1, "nphys must be >= 1");
    AGF2_REQUIRE(m0 && m1 && naux_out && e_aux && v_aux, "NULL argument");
    AGF2_REQUIRE(tol >= 0.0 && tol < 1.0, "tol must be in [0, 1)");
    *naux_out = 0;
    const long nn = (long)nphys * nphys;
    FiniteCheck(h).add(m0, nn, "m0").add(m1, nn, "m1").run();
    *naux_out = compress_impl(h, nphys, m0, m1, tol, e_aux, v_aux);
  });
}

agf2_status agf2_fock_loop(agf2_handle_t hh, int nphys, int naux, const double* Lpq,
                           const double* hcore, int nelec, int naux_se, double* e_se,
                           const double* v_se, double* rdm1, double* fock, double* e_pole,
                           double* u_pole, int* nocc_pole, double* mu, double* shift,
                           int* n_cycle, const agf2_fock_opts* opts) {
  agf2_status conv = AGF2_OK;
  agf2_status st = guarded(hh, [&](Handle& h) {
    AGF2_REQUIRE(nphys >= 1 && naux >= 1 && naux_se >= 0, "bad sizes");
    AGF2_REQUIRE(Lpq && hcore && rdm1 && fock && e_pole && u_pole && nocc_pole && mu &&
                     shift && n_cycle && (naux_se == 0 || (e_se && v_se)),
                 "NULL argument");
    const long nn = (long)nphys * nphys;
    FiniteCheck(h)
        .add(Lpq, naux * nn, "Lpq")
        .add(hcore, nn, "hcore")
        .add(rdm1, nn, "rdm1")
        .add(e_se, naux_se, "e_se")
        .add(v_se, (long)nphys * naux_se, "v_se")
        .run();
    agf2_fock_opts o;
    agf2_fock_opts_default(&o);
    if (opts) o = *opts;
    FockLoopResult r = fock_loop_impl(h, nphys, naux, Lpq, hcore, nelec, naux_se, e_se, v_se,
                                      rdm1, fock, e_pole, u_pole, o);
    *nocc_pole = r.nocc_pole;
    *mu = r.mu;
    *shift = r.shift;
    *n_cycle = r.n_cycle;
    if (!r.converged) conv = AGF2_ERR_NO_CONVERGE;
  });
  if (st == AGF2_OK && conv != AGF2_OK) {
    reinterpret_cast<Handle*>(hh)->last_error = "Fock loop reached max_cycle";
    return conv;
  }
  return st;
}

agf2_status agf2_energy_gf(agf2_handle_t hh, int nphys, const double* hcore, const double* fock,
                           const double* rdm1, int npole, int nocc_pole, const double* e_pole,
                           const double* u_pole, int naux_occ, const double* e_se_occ,
                           const double* v_se_occ, int naux_vir, const double* e_se_vir,
                           const double* v_se_vir, double* e_1b, double* e_2b) {
  return guarded(hh, [&](Handle& h) {
    AGF2_REQUIRE(nphys >= 1 && npole >= 1 && nocc_pole >= 0 && nocc_pole <= npole &&
                     naux_occ >= 0 && naux_vir >= 0,
                 "bad sizes");
    AGF2_REQUIRE(hcore && fock && rdm1 && e_pole && u_pole && e_1b && e_2b, "NULL argument");
    AGF2_REQUIRE((naux_occ == 0 || (e_se_occ && v_se_occ)) &&
                     (naux_vir == 0 || (e_se_vir && v_se_vir)),
                 "NULL auxiliary argument");
    const long nn = (long)nphys * nphys;
    FiniteCheck(h)
        .add(hcore, nn, "hcore")
        .add(fock, nn, "fock")
        .add(rdm1, nn, "rdm1")
        .add(e_pole, npole, "e_pole")
        .add(u_pole, (long)nphys * npole, "u_pole")
        .add(e_se_occ, naux_occ, "e_se_occ")
        .add(v_se_occ, (long)nphys * naux_occ, "v_se_occ")
        .add(e_se_vir, naux_vir, "e_se_vir")
        .add(v_se_vir, (long)nphys * naux_vir, "v_se_vir")
        .run();
    energy_impl(h, nphys, hcore, fock, rdm1, npole, nocc_pole, e_pole, u_pole, naux_occ,
                e_se_occ, v_se_occ, naux_vir, e_se_vir, v_se_vir, e_1b, e_2b);
  });
}

agf2_status agf2_spectral_function(agf2_handle_t hh, int nphys, int npole,
                                   const double* e_pole, const double* u_pole,
                                   const double* weight, int nomega, const double* omega,
                                   double eta, double* A) {
  return guarded(hh, [&](Handle& h) {
    AGF2_REQUIRE(nphys >= 1 && npole >= 1 && nomega >= 0, "bad sizes");
    AGF2_REQUIRE(eta > 0.0 && std::isfinite(eta), "eta must be positive");
    AGF2_REQUIRE(e_pole && u_pole && (nomega == 0 || (omega && A)), "NULL argument");
    FiniteCheck(h)
        .add(e_pole, npole, "e_pole")
        .add(u_pole, (long)nphys * npole, "u_pole")
        .add(weight, nphys, "weight")
        .add(omega, nomega, "omega")
        .run();
    spectral_function(h, nphys, npole, e_pole, u_pole, weight, nomega, omega, eta, A);
  });
}

agf2_status agf2_spectral_function_noalloc(agf2_handle_t hh, int nphys, int npole,
                                           const double* e_pole, const double* u_pole,
                                           const double* weight, int nomega,
                                           const double* omega, double eta, double* A) {
  return guarded(hh, [&](Handle& h) {
    AGF2_REQUIRE(nphys >= 1 && npole >= 1 && nomega >= 0, "bad sizes");
    AGF2_REQUIRE(eta > 0.0 && std::isfinite(eta), "eta must be positive");
    AGF2_REQUIRE(e_pole && u_pole && (nomega == 0 || (omega && A)), "NULL argument");
    spectral_function_noalloc(h, nphys, npole, e_pole, u_pole, weight, nomega, omega, eta, A);
  });
}

}  // extern "C"
