// Internal declarations shared by the library's translation units.
#pragma once

#include <hip/hip_runtime.h>
#include <rocblas/rocblas.h>

#include <cstddef>
#include <cstdint>
#include <exception>
#include <new>
#include <map>
#include <string>
#include <vector>

#include "../../include/agf2.h"

namespace agf2 {

// Error carried from the implementation to the C boundary.
struct Error {
  agf2_status status;
  std::string msg;
};

#define AGF2_HIP(call)                                                        \
  do {                                                                        \
    hipError_t e_ = (call);                                                   \
    if (e_ != hipSuccess)                                                     \
      throw ::agf2::Error{AGF2_ERR_HIP, std::string(#call) + ": " +           \
                                            hipGetErrorString(e_)};           \
  } while (0)

#define AGF2_CHECK_LAUNCH() AGF2_HIP(hipGetLastError())

#define AGF2_REQUIRE(cond, text)                                              \
  do {                                                                        \
    if (!(cond)) throw ::agf2::Error{AGF2_ERR_ARG, text};                     \
  } while (0)

// A device buffer that grows on demand and is reused across calls.
struct DevBuf {
  void* ptr = nullptr;
  size_t bytes = 0;
  void* get(size_t need);
  template <class T> T* as(size_t n) { return static_cast<T*>(get(n * sizeof(T))); }
  void release();
};

struct Handle;

// v_mfma_f64_16x16x4f64 lane layout (gfx950): lane l supplies A[l % 16][l / 16]
// and B[l / 16][l % 16]; accumulator register r of lane l holds
// D[l / 16 + 4 r][l % 16].

// ---------------------------------------------------------------- GEMM
// C[b][m][n] = alpha * sum_k A(b,m,k) B(b,k,n) + beta * C[b][m][n]
// Addresses: A + b*sAb + m*sAm + k*sAk (likewise B and C). Either sAm or sAk
// must be 1, and either sBn or sBk must be 1 (the contiguous one is used for
// coalescing); C is written with lanes along n, so sCn = 1 coalesces.
struct Gemm {
  int M = 0, N = 0, K = 0;
  int batch = 1;
  const double* A = nullptr;
  long sAb = 0, sAm = 0, sAk = 0;
  const double* B = nullptr;
  long sBb = 0, sBk = 0, sBn = 0;
  double* C = nullptr;
  long sCb = 0, sCm = 0, sCn = 0;
  double alpha = 1.0, beta = 0.0;
  bool lower = false;   // square outputs: only tiles on or below the diagonal are written
};
void gemm_f64(const Gemm& g, hipStream_t stream);
void gemm_f64_padded(const Gemm& g, int Npad, hipStream_t stream);

// Sum `nslice` [rows][cols] slices spaced `slice_stride` apart into out
// (fixed order), optionally scaling: out = scale * sum_s in[s] (+ out if add).
void sum_slices(const double* in, long slice_stride, int nslice, long n,
                double* out, double scale, bool add, hipStream_t stream);

// ---------------------------------------------------------------- moments
// FP64 slab tile job: pole pairs pair0.. of one part of one system.
struct SlabF64 {
  const double* R; long sRp, sRx;   // R[p][x][Qp]
  const double* S; long sSp, sSc;   // S[q][c][Qp]
  const double* ep; const double* ec;
  int N, nc, Qp;
  const int* pi; const int* pj; const long* pcol;
  int pair0, npairs; long col_base;
  double* Z; long ldz; double* w;
  int tiles_x, tiles_c;             // tiles_c for the chosen inner tile width
};
// FP64 SYRK job: lower-triangle tiles of U0 += Z Z^T, U1 += Z diag(w) Z^T.
struct SyrkF64 {
  const double* Z; long ldz; const double* w;
  int N; long K; long kper; int nsplit;
  double* part; long part_stride;   // per split: [2][N][N]
  int tiles;                        // lower-triangle tile count
};
int slab_f64_tc(int nc);            // default inner tile width for nc
long slab_f64_tiles(const SlabF64& a);
void launch_slab_f64(int tc, const SlabF64& a, hipStream_t st);
void launch_syrk_f64(const SyrkF64& a, hipStream_t st);
// Persistent grouped launches over `njobs` jobs: job j owns the global work
// indices [prefix[j], prefix[j+1]) (its tiles in order; prefix[njobs] =
// total), and `grid` workgroups stride over [0, total). A SYRK job's local
// index l is tile l % tiles of K split l / tiles.
void launch_slab_f64_grouped(int tc, const SlabF64* jobs, const long* prefix, int njobs,
                             long total, int grid, hipStream_t st);
void launch_syrk_f64_grouped(const SyrkF64* jobs, const long* prefix, int njobs, long total,
                             int grid, hipStream_t st);
// Workgroups that fill the device for a grouped launch (kind 0 slab of width
// tc, kind 1 SYRK): compute units x resident workgroups per unit.
int grouped_grid_f64(int kind, int tc);
void fill_zero(double* p, long n, hipStream_t st);
void reduce_moment_partials(const double* part, long part_stride, int nsplit, int N,
                            double* U0, double* U1, hipStream_t st);
// True when u (N x npole) is exactly the identity: the pole-basis transforms
// may then take u = nullptr (a relayout of L instead of a product).
bool poles_are_identity(Handle& h, int N, int npole, const double* u);
void pole_transform_f64(int N, int Q, int Qp, const double* L, const double* u, int npole,
                        int p0, int np, double* T, hipStream_t st);
void lov_transform_f64(int N, int Q, int Qp, const double* u, int npole, int o, int v,
                       const double* Lxv, double* Lov, hipStream_t st);
void build_moments_f64(Handle& h, int N, int Q, const double* L, int npole,
                       int nocc, const double* e, const double* u, double* m0o,
                       double* m1o, double* m0v, double* m1v);
// Moments 0 .. 2 npm - 1 of each part (Uo[k], Uv[k] are [N][N] outputs).
void build_moments_f64_n(Handle& h, int N, int Q, const double* L, int npole, int nocc,
                         const double* e, const double* u, int npm, double* const* Uo,
                         double* const* Uv);
// Compression of one part to nblock Lanczos blocks from its moments
// m[0 .. 2 nblock - 1] ([N][N] each, contiguous); returns nblock * N.
int compress_lanczos_impl(Handle& h, int N, int nblock, const double* m, double* e_aux,
                          double* v_aux);
void build_moments_split(Handle& h, int N, int Q, const double* L, int npole,
                         int nocc, const double* e, const double* u,
                         double* m0o, double* m1o, double* m0v, double* m1v,
                         bool fp16);

// ---------------------------------------------------------------- Fock / misc
void fock_build(Handle& h, int N, int Q, const double* L, const double* hcore,
                const double* D, double alpha, double* F);
void build_hext(int N, int naux, const double* F, const double* e,
                const double* v, double shift, double* H, hipStream_t s);
void column_weights(int nrows_phys, int npole, const double* evecs_rowmajor,
                    double* w, hipStream_t s);
void extract_poles(int N, int npole, const double* evecs, double* u,
                   hipStream_t s);
double dot_f64(Handle& h, long n, const double* a, const double* b);
void axpby_f64(long n, double a, const double* x, double b, double* y,
               hipStream_t s);
void symmetrize_f64(int N, double* A, hipStream_t s);

// Non-finite input check: each array added is scanned on the device (one
// launch per array, one host synchronisation in run()); run() throws
// AGF2_ERR_ARG naming the first array that holds a NaN or an infinity.
// Arrays of length 0 or NULL pointers are skipped; at most 32 per check.
struct FiniteCheck {
  Handle& h;
  std::vector<const double*> ptr;
  std::vector<long> len;
  std::vector<std::string> name;
  explicit FiniteCheck(Handle& hh) : h(hh) {}
  FiniteCheck& add(const double* p, long n, const char* what);
  void run();
};

// Per-kernel-class timing: hipEvents recorded on the handle's stream around
// each launch of a class, with the launch's algorithmic flop and byte counts.
struct ProfRecord {
  std::string name;
  hipEvent_t start, stop;
  double flops, bytes;
};
struct ProfTotal {
  long launches = 0;
  double ms = 0.0, flops = 0.0, bytes = 0.0;
};

struct FockLoopResult {
  int nocc_pole = 0;
  double mu = 0.0, shift = 0.0;
  int n_cycle = 0;
  bool converged = false;
};
FockLoopResult fock_loop_impl(Handle& h, int nphys, int naux, const double* Lpq,
                              const double* hcore, int nelec, int naux_se, double* e_se,
                              const double* v_se, double* rdm1, double* fock,
                              double* e_pole, double* u_pole, const agf2_fock_opts& o);
void energy_impl(Handle& h, int nphys, const double* hcore, const double* fock,
                 const double* rdm1, int npole, int nocc_pole, const double* e_pole,
                 const double* u_pole, int naux_occ, const double* e_se_occ,
                 const double* v_se_occ, int naux_vir, const double* e_se_vir,
                 const double* v_se_vir, double* e_1b, double* e_2b);
int compress_part(Handle& h, int N, const double* m0, const double* m1, double tol,
                  double* e_aux, double* v_aux);
void build_moments(Handle& h, agf2_precision prec, int N, int Q, const double* L, int npole,
                   int nocc, const double* e, const double* u, double* m0o, double* m1o,
                   double* m0v, double* m1v);

// Broadened spectral function of the poles (spectrum.hip).
void spectral_function(Handle& h, int nphys, int npole, const double* e_pole,
                       const double* u_pole, const double* weight, int nomega,
                       const double* omega, double eta, double* A);
// The allocation-free variant over the device's static scratch array, and
// the per-device address of that array (resolved at the first call for a
// device, which agf2_create makes).
void spectral_function_noalloc(Handle& h, int nphys, int npole, const double* e_pole,
                               const double* u_pole, const double* weight, int nomega,
                               const double* omega, double eta, double* A);
double* noalloc_scratch(int device);

struct BatchPlan;   // batched moment build (moments_batched.hip)
void destroy_batch_plan(BatchPlan* p);

struct Handle {
  int device = 0;
  BatchPlan* batch = nullptr;
  bool profiling = false;
  std::vector<ProfRecord> prof_pending;
  std::map<std::string, ProfTotal> prof_total;
  std::vector<std::string> prof_names;   // stable storage for returned names
  hipStream_t stream = nullptr;
  bool own_stream = false;
  rocblas_handle blas = nullptr;
  std::string last_error;
  // workspace pools
  DevBuf ws_moments[9];
  DevBuf ws_fock[8];
  DevBuf ws_misc[8];
  DevBuf ws_run[8];
  DevBuf ws_mlp[2];   // warm-start loss partials and prediction scratch
  DevBuf ws_spec;     // spectral function: pole weights
  DevBuf ws_red;
  DevBuf ws_check;    // flags of the non-finite input check
  double* host_red = nullptr;   // pinned scratch for small reductions
  size_t host_red_n = 0;
  ~Handle();
};

// RAII scope: records start/stop events around the enclosed launches when
// profiling is on.
struct ProfScope {
  Handle& h;
  ProfRecord rec;
  bool on;
  ProfScope(Handle& hh, const char* name, double flops, double bytes);
  ~ProfScope();
};

// Makes the handle's device current for a scope.
struct DeviceGuard {
  int prev = 0;
  explicit DeviceGuard(int dev) {
    (void)hipGetDevice(&prev);
    AGF2_HIP(hipSetDevice(dev));
  }
  ~DeviceGuard() { (void)hipSetDevice(prev); }
};

// Runs an entry point's body with the handle's device current and turns
// exceptions into status codes (the message kept for agf2_last_error).
template <class F>
agf2_status guarded(agf2_handle_t hh, F&& body) {
  if (!hh) return AGF2_ERR_ARG;
  Handle& h = *reinterpret_cast<Handle*>(hh);
  try {
    DeviceGuard g(h.device);
    body(h);
    h.last_error.clear();
    return AGF2_OK;
  } catch (const Error& e) {
    h.last_error = e.msg;
    return e.status;
  } catch (const std::bad_alloc&) {
    h.last_error = "host allocation failed";
    return AGF2_ERR_NOMEM;
  } catch (const std::exception& e) {
    h.last_error = e.what();
    return AGF2_ERR_HIP;
  }
}

}  // namespace agf2
