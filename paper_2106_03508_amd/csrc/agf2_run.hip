// Outer self-consistent AGF2 loop (agf2_run): sequences the moment build,
// DIIS/damping on the moments, compression, Fock loop and energy on the
// handle's stream, keeping every array on the device.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>
#include <exception>
#include <new>
#include <string>

#include "agf2_internal.h"

namespace agf2 {
namespace {

__global__ void init_reference(int N, int nocc, const double* e_mf, double* e, double* u,
                               double* D) {
  const long nn = (long)N * N;
  for (long idx = blockIdx.x * (long)blockDim.x + threadIdx.x; idx < nn;
       idx += (long)gridDim.x * blockDim.x) {
    const int r = (int)(idx / N), c = (int)(idx % N);
    u[idx] = (r == c) ? 1.0 : 0.0;
    D[idx] = (r == c && r < nocc) ? 2.0 : 0.0;
    if (idx < N) e[idx] = e_mf[idx];
  }
}

// dst[p][off + k] = src[p][k] for k < n (src row stride lds, dst row stride ldd)
__global__ void copy_cols(int N, int n, const double* src, long lds, double* dst, long ldd,
                          int off) {
  const long tot = (long)N * n;
  for (long idx = blockIdx.x * (long)blockDim.x + threadIdx.x; idx < tot;
       idx += (long)gridDim.x * blockDim.x) {
    const int p = (int)(idx / n), k = (int)(idx % n);
    dst[(long)p * ldd + off + k] = src[(long)p * lds + k];
  }
}

// w[t] = sum_p u[p][cols[t]]^2 for t = 0, 1
__global__ void two_col_weights(int N, int npole, const double* u, int c0, int c1, double* w) {
  const int t = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int c = t == 0 ? c0 : c1;
  double acc = 0.0;
  if (c >= 0 && c < npole)
    for (int p = lane; p < N; p += 64) acc += u[(long)p * npole + c] * u[(long)p * npole + c];
  for (int off = 32; off > 0; off >>= 1) acc += __shfl_down(acc, off, 64);
  if (lane == 0) w[t] = acc;
}

inline int nblk(long n) { return (int)std::max<long>(1, std::min<long>((n + 255) / 256, 4096)); }

double now() {
  return std::chrono::duration<double>(std::chrono::steady_clock::now().time_since_epoch())
      .count();
}

}  // namespace

// DIIS on a device vector with the change since the previous iterate as the
// error (the first call only records the iterate).
struct MomentDiis {
  Handle& h;
  long len;
  int space;
  double* prev;
  double* err;
  bool have_prev = false;
  double* store;
  std::vector<int> order;
  std::vector<double> B;
  MomentDiis(Handle& hh, long len_, int space_)
      : h(hh), len(len_), space(space_), B((size_t)std::max(space_, 1) * std::max(space_, 1)) {
    double* w = h.ws_run[5].as<double>(2 * len_ + (long)std::max(space_, 1) * 2 * len_);
    prev = w;
    err = w + len_;
    store = w + 2 * len_;
  }
  void update(double* x) {
    if (space <= 0) return;
    if (!have_prev) {
      AGF2_HIP(hipMemcpyAsync(prev, x, len * sizeof(double), hipMemcpyDeviceToDevice, h.stream));
      have_prev = true;
      return;
    }
    // err = x - prev; prev = x
    axpby_f64(len, 1.0, x, 0.0, err, h.stream);
    axpby_f64(len, -1.0, prev, 1.0, err, h.stream);
    AGF2_HIP(hipMemcpyAsync(prev, x, len * sizeof(double), hipMemcpyDeviceToDevice, h.stream));
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
    AGF2_HIP(hipMemcpyAsync(es, err, len * sizeof(double), hipMemcpyDeviceToDevice, h.stream));
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
    // partial-pivoting solve
    const int m = n + 1;
    for (int c = 0; c < m; ++c) {
      int piv = c;
      for (int r = c + 1; r < m; ++r)
        if (std::fabs(A[r * m + c]) > std::fabs(A[piv * m + c])) piv = r;
      if (A[piv * m + c] == 0.0) return;
      if (piv != c) {
        for (int k = 0; k < m; ++k) std::swap(A[c * m + k], A[piv * m + k]);
        std::swap(rhs[c], rhs[piv]);
      }
      for (int r = c + 1; r < m; ++r) {
        const double f = A[r * m + c] / A[c * m + c];
        for (int k = c; k < m; ++k) A[r * m + k] -= f * A[c * m + k];
        rhs[r] -= f * rhs[c];
      }
    }
    for (int r = m - 1; r >= 0; --r) {
      double t = rhs[r];
      for (int k = r + 1; k < m; ++k) t -= A[r * m + k] * rhs[k];
      rhs[r] = t / A[r * m + r];
    }
    for (int a = 0; a < n; ++a)
      axpby_f64(len, rhs[a], store + (long)order[a] * 2 * len, a == 0 ? 0.0 : 1.0, x, h.stream);
  }
  // History to / from a host blob: prev [len], store [max(space,1)][2][len],
  // B [max(space,1)^2]; the blob pointer advances past what was written/read.
  void save(double*& d, hipStream_t st) const {
    const int sp = std::max(space, 1);
    AGF2_HIP(hipMemcpyAsync(d, prev, len * sizeof(double), hipMemcpyDeviceToHost, st));
    d += len;
    AGF2_HIP(hipMemcpyAsync(d, store, (long)sp * 2 * len * sizeof(double), hipMemcpyDeviceToHost,
                            st));
    d += (long)sp * 2 * len;
    for (size_t k = 0; k < B.size(); ++k) d[k] = B[k];
    d += B.size();
  }
  void restore(bool have, const int* ord, int n, const double* d) {
    const int sp = std::max(space, 1);
    have_prev = have;
    order.assign(ord, ord + n);
    for (int k : order)
      if (k < 0 || k >= space) throw Error{AGF2_ERR_ARG, "state_in is inconsistent"};
    AGF2_HIP(hipMemcpyAsync(prev, d, len * sizeof(double), hipMemcpyHostToDevice, h.stream));
    d += len;
    AGF2_HIP(hipMemcpyAsync(store, d, (long)sp * 2 * len * sizeof(double),
                            hipMemcpyHostToDevice, h.stream));
    d += (long)sp * 2 * len;
    for (size_t k = 0; k < B.size(); ++k) B[k] = d[k];
  }
};

}  // namespace agf2

namespace agf2 {
namespace {

// Saved state of agf2_run between iterations (host blob, see
// agf2_run_state_bytes): a fixed header, then the device arrays in order.
struct RunStateHeader {
  char magic[8];          // "AGF2RUN2"
  int nphys, diis_space, nblock;
  int next_iter;          // index of the next iteration to run
  int npole, nocc_pole;
  int have_prev;          // a previous iteration's E, IP, EA exist
  int diis_have_prev, diis_n;
  int diis_order[64];     // slots, oldest first
  double prev_e, prev_ip, prev_ea;
};

// poles, amplitudes, density, previous moments, moment DIIS history
long state_doubles(int N, int space, int nb) {
  const long nn = (long)N * N;
  const long npmax = (long)N * (1 + 2 * nb), len = 4L * nb * nn;
  const long sp = std::max(space, 1);
  return npmax + (long)N * npmax + nn + len + len + sp * 2 * len + sp * sp;
}

}  // namespace

agf2_status run_impl(Handle& h, const agf2_run_opts* opts, int nphys, int naux, const double* Lpq,
                     const double* hcore, const double* e_mf, int nocc, const double* dm_init,
                     const void* state_in, void* state_out, int max_iter_call,
                     agf2_iter_record* records, int* n_records, int* converged, double* e_pole,
                     double* u_pole, int* nocc_pole, double* rdm1) {
  agf2_status result = AGF2_OK;
  try {
    int prev_dev = 0;
    (void)hipGetDevice(&prev_dev);
    AGF2_HIP(hipSetDevice(h.device));
    struct Restore {
      int d;
      ~Restore() { (void)hipSetDevice(d); }
    } restore{prev_dev};
    agf2_run_opts o;
    agf2_run_opts_default(&o);
    if (opts) o = *opts;
    AGF2_REQUIRE(nphys >= 1 && naux >= 1 && nocc >= 1 && nocc < nphys, "bad sizes");
    AGF2_REQUIRE(Lpq && hcore && e_mf && records && n_records && converged && e_pole && u_pole &&
                     nocc_pole && rdm1,
                 "NULL argument");
    AGF2_REQUIRE(o.max_iter >= 0 && o.diis_space >= 0 && o.diis_space <= 64 &&
                     o.damping >= 0.0 && o.damping < 1.0 && o.nblock >= 1 && o.nblock <= 8,
                 "bad run options");
    AGF2_REQUIRE(o.nblock == 1 || (o.prec == AGF2_FP64 && dm_init == nullptr),
                 "nblock > 1 needs prec AGF2_FP64 and no dm_init");
    hipStream_t st = h.stream;
    const int N = nphys;
    const long nn = (long)N * N;
    const int nb = o.nblock, nmom = 2 * nb;
    const int nmax = N * (1 + 2 * nb);   // poles: N + 2 nb N
    const long nbn = (long)nb * N;       // auxiliaries per part
    FiniteCheck(h)
        .add(Lpq, (long)naux * nn, "Lpq")
        .add(hcore, nn, "hcore")
        .add(e_mf, N, "e_mf")
        .add(dm_init, 4 * nn, "dm_init")
        .run();
    // state
    double* w = h.ws_run[0].as<double>(2L * nmax + 2L * N * nmax + nn + 8);
    double* e_cur = w;
    double* e_new = e_cur + nmax;
    double* u_cur = e_new + nmax;
    double* u_new = u_cur + (long)N * nmax;
    double* small = u_new + (long)N * nmax;   // 2 column weights
    double* m = h.ws_run[1].as<double>(4L * nmom * nn);
    double* mprev = m + 2L * nmom * nn;
    double* a = h.ws_run[2].as<double>(4 * nbn + 4 * N * nbn + nn);
    double* eo = a;
    double* vo = eo + nbn;
    double* ev = vo + N * nbn;
    double* vv = ev + nbn;
    double* e_se = vv + N * nbn;
    double* v_se = e_se + 2 * nbn;
    double* fock = v_se + 2 * N * nbn;
    double* vo_p = h.ws_run[3].as<double>(2 * N * nbn);
    double* vv_p = vo_p + N * nbn;
    int npole = N, nocc_p = nocc;
    MomentDiis diis(h, 2L * nmom * nn, o.diis_space);
    bool conv = false, have_prev = false, fock_failed = false;
    double prev_e = 0, prev_ip = 0, prev_ea = 0;
    int it0 = 0;
    if (state_in) {
      RunStateHeader hd;
      std::memcpy(&hd, state_in, sizeof hd);
      AGF2_REQUIRE(std::memcmp(hd.magic, "AGF2RUN2", 8) == 0, "state_in is not an agf2_run state");
      AGF2_REQUIRE(hd.nphys == N && hd.diis_space == o.diis_space && hd.nblock == nb,
                   "state_in was saved for another nphys, diis_space or nblock");
      AGF2_REQUIRE(hd.npole >= 2 && hd.npole <= nmax && hd.nocc_pole >= 1 &&
                       hd.nocc_pole < hd.npole && hd.next_iter >= 1 &&
                       hd.diis_n >= 0 && hd.diis_n <= o.diis_space,
                   "state_in is inconsistent");
      const double* d = reinterpret_cast<const double*>(static_cast<const char*>(state_in) +
                                                         sizeof hd);
      it0 = hd.next_iter;
      npole = hd.npole;
      nocc_p = hd.nocc_pole;
      have_prev = hd.have_prev != 0;
      prev_e = hd.prev_e;
      prev_ip = hd.prev_ip;
      prev_ea = hd.prev_ea;
      auto up = [&](double* dst, long n) {
        AGF2_HIP(hipMemcpyAsync(dst, d, n * sizeof(double), hipMemcpyHostToDevice, st));
        d += n;
      };
      up(e_cur, nmax);
      up(u_cur, (long)N * nmax);
      up(rdm1, nn);
      up(mprev, 2L * nmom * nn);
      diis.restore(hd.diis_have_prev != 0, hd.diis_order, hd.diis_n, d);
      AGF2_HIP(hipStreamSynchronize(st));
    } else {
      hipLaunchKernelGGL(init_reference, dim3(nblk(nn)), dim3(256), 0, st, N, nocc, e_mf, e_cur,
                         u_cur, rdm1);
      AGF2_CHECK_LAUNCH();
    }
    int nrec = 0;
    int it_end = o.max_iter;
    if (max_iter_call > 0) it_end = std::min(it_end, it0 + max_iter_call - 1);
    int it = it0;
    for (; it <= it_end; ++it) {
      agf2_iter_record rec{};
      rec.iter = it;
      double t0 = now();
      bool warm = (it == 0 && dm_init != nullptr);
      int no = 0, nv = 0;
      for (int attempt = 0; attempt < 2; ++attempt) {
        if (nb == 1) {
          build_moments(h, o.prec, N, naux, Lpq, npole, nocc_p, e_cur, u_cur, m, m + nn,
                        m + 2 * nn, m + 3 * nn);
        } else {
          std::vector<double*> uo(nmom), uv(nmom);
          for (int k = 0; k < nmom; ++k) {
            uo[k] = m + k * nn;
            uv[k] = m + (nmom + k) * nn;
          }
          build_moments_f64_n(h, N, naux, Lpq, npole, nocc_p, e_cur, u_cur, nb, uo.data(),
                              uv.data());
        }
        if (warm) axpby_f64(4 * nn, 1.0, dm_init, 1.0, m, st);
        if (o.damping > 0.0 && it > 0)
          axpby_f64(2L * nmom * nn, o.damping, mprev, 1.0 - o.damping, m, st);
        if (!warm) diis.update(m);
        for (int k = 0; k < 2 * nmom; ++k) symmetrize_f64(N, m + k * nn, st);
        AGF2_HIP(hipStreamSynchronize(st));
        rec.t_moments = now() - t0;
        t0 = now();
        try {
          if (nb == 1) {
            no = compress_part(h, N, m, m + nn, o.compress_tol, eo, vo);
            nv = compress_part(h, N, m + 2 * nn, m + 3 * nn, o.compress_tol, ev, vv);
          } else {
            no = compress_lanczos_impl(h, N, nb, m, eo, vo);
            nv = compress_lanczos_impl(h, N, nb, m + nmom * nn, ev, vv);
          }
        } catch (const Error& e) {
          if (warm && e.status == AGF2_ERR_NOT_PD) {   // fall back to the cold start
            warm = false;
            t0 = now();
            continue;
          }
          throw;
        }
        break;
      }
      if (warm) {
        // a warm-started iteration 0 still seeds the DIIS history
        diis.update(m);
      }
      rec.warm = warm ? 1 : 0;
      AGF2_HIP(hipMemcpyAsync(mprev, m, 2L * nmom * nn * sizeof(double), hipMemcpyDeviceToDevice,
                              st));
      // pack the auxiliaries: e_se = [eo, ev], v_se = [vo | vv]; one block's
      // couplings have row stride N, several blocks' row stride nb N
      const int ns = no + nv;
      const long ldv = nb == 1 ? (long)N : nbn;
      AGF2_HIP(hipMemcpyAsync(e_se, eo, no * sizeof(double), hipMemcpyDeviceToDevice, st));
      AGF2_HIP(hipMemcpyAsync(e_se + no, ev, nv * sizeof(double), hipMemcpyDeviceToDevice, st));
      hipLaunchKernelGGL(copy_cols, dim3(nblk((long)N * no)), dim3(256), 0, st, N, no, vo,
                         ldv, v_se, (long)ns, 0);
      hipLaunchKernelGGL(copy_cols, dim3(nblk((long)N * nv)), dim3(256), 0, st, N, nv, vv,
                         ldv, v_se, (long)ns, no);
      hipLaunchKernelGGL(copy_cols, dim3(nblk((long)N * no)), dim3(256), 0, st, N, no, vo,
                         ldv, vo_p, (long)no, 0);
      hipLaunchKernelGGL(copy_cols, dim3(nblk((long)N * nv)), dim3(256), 0, st, N, nv, vv,
                         ldv, vv_p, (long)nv, 0);
      AGF2_CHECK_LAUNCH();
      AGF2_HIP(hipStreamSynchronize(st));
      rec.t_compress = now() - t0;
      t0 = now();
      FockLoopResult fl = fock_loop_impl(h, N, naux, Lpq, hcore, 2 * nocc, ns, e_se, v_se, rdm1,
                                         fock, e_new, u_new, o.fock);
      rec.t_fock = now() - t0;
      t0 = now();
      const int npole_new = N + ns;
      double e1 = 0, e2 = 0;
      energy_impl(h, N, hcore, fock, rdm1, npole_new, fl.nocc_pole, e_new, u_new, no, e_se,
                  vo_p, nv, e_se + no, vv_p, &e1, &e2);
      // IP / EA and their weights
      hipLaunchKernelGGL(two_col_weights, dim3(1), dim3(128), 0, st, N, npole_new, u_new,
                         fl.nocc_pole - 1, fl.nocc_pole, small);
      AGF2_CHECK_LAUNCH();
      double hv[4] = {0, 0, 0, 0};
      if (fl.nocc_pole >= 1)
        AGF2_HIP(hipMemcpyAsync(&hv[0], e_new + fl.nocc_pole - 1, 2 * sizeof(double),
                                hipMemcpyDeviceToHost, st));
      AGF2_HIP(hipMemcpyAsync(&hv[2], small, 2 * sizeof(double), hipMemcpyDeviceToHost, st));
      AGF2_HIP(hipStreamSynchronize(st));
      rec.t_energy = now() - t0;
      rec.nocc_pole = fl.nocc_pole;
      rec.npole = npole_new;
      rec.fock_cycles = fl.n_cycle;
      rec.fock_converged = fl.converged ? 1 : 0;
      rec.e_1b = e1;
      rec.e_2b = e2;
      rec.e_tot = e1 + e2;
      rec.ip = -hv[0];
      rec.ea = hv[1];
      rec.w_ip = hv[2];
      rec.w_ea = hv[3];
      rec.mu = fl.mu;
      rec.shift = fl.shift;
      records[nrec++] = rec;
      // the new Green's function becomes the current one
      std::swap(e_cur, e_new);
      std::swap(u_cur, u_new);
      npole = npole_new;
      nocc_p = fl.nocc_pole;
      if (!fl.converged) {
        // the density of this iteration is not relaxed: stop here, with the
        // outputs holding this iteration's Green's function and density
        fock_failed = true;
        ++it;
        break;
      }
      if (have_prev && std::fabs(rec.e_tot - prev_e) < o.conv_tol &&
          std::max(std::fabs(rec.ip - prev_ip), std::fabs(rec.ea - prev_ea)) < o.conv_tol_ipea) {
        conv = true;
        ++it;
        break;
      }
      have_prev = true;
      prev_e = rec.e_tot;
      prev_ip = rec.ip;
      prev_ea = rec.ea;
      if (nocc_p < 1 || nocc_p >= npole)
        throw Error{AGF2_ERR_NELEC, "aufbau left no occupied or no virtual pole"};
    }
    AGF2_HIP(hipMemcpyAsync(e_pole, e_cur, npole * sizeof(double), hipMemcpyDeviceToDevice, st));
    AGF2_HIP(hipMemcpyAsync(u_pole, u_cur, (long)N * npole * sizeof(double),
                            hipMemcpyDeviceToDevice, st));
    if (state_out) {
      RunStateHeader hd;
      std::memset(&hd, 0, sizeof hd);
      std::memcpy(hd.magic, "AGF2RUN2", 8);
      hd.nphys = N;
      hd.diis_space = o.diis_space;
      hd.nblock = nb;
      hd.next_iter = it;
      hd.npole = npole;
      hd.nocc_pole = nocc_p;
      hd.have_prev = have_prev ? 1 : 0;
      hd.prev_e = prev_e;
      hd.prev_ip = prev_ip;
      hd.prev_ea = prev_ea;
      hd.diis_have_prev = diis.have_prev ? 1 : 0;
      hd.diis_n = (int)diis.order.size();
      for (int k = 0; k < hd.diis_n; ++k) hd.diis_order[k] = diis.order[k];
      std::memcpy(state_out, &hd, sizeof hd);
      double* d = reinterpret_cast<double*>(static_cast<char*>(state_out) + sizeof hd);
      auto down = [&](const double* src, long n) {
        AGF2_HIP(hipMemcpyAsync(d, src, n * sizeof(double), hipMemcpyDeviceToHost, st));
        d += n;
      };
      down(e_cur, nmax);
      down(u_cur, (long)N * nmax);
      down(rdm1, nn);
      down(mprev, 2L * nmom * nn);
      diis.save(d, st);
    }
    AGF2_HIP(hipStreamSynchronize(st));
    *nocc_pole = nocc_p;
    *n_records = nrec;
    *converged = conv ? 1 : 0;
    h.last_error.clear();
    if (fock_failed) {
      h.last_error = "the Fock loop reached max_cycle at iteration " +
                     std::to_string(records[nrec - 1].iter);
      result = AGF2_ERR_NO_CONVERGE;
    } else if (!conv && it > o.max_iter) {
      h.last_error = "AGF2 reached max_iter without converging";
      result = AGF2_ERR_NO_CONVERGE;
    }
  } catch (const Error& e) {
    h.last_error = e.msg;
    result = e.status;
  } catch (const std::bad_alloc&) {
    h.last_error = "host allocation failed";
    result = AGF2_ERR_NOMEM;
  } catch (const std::exception& e) {
    h.last_error = e.what();
    result = AGF2_ERR_HIP;
  }
  return result;
}

}  // namespace agf2

using namespace agf2;

extern "C" {

void agf2_run_opts_default(agf2_run_opts* o) {
  if (!o) return;
  o->max_iter = 20;
  o->conv_tol = 1e-8;
  o->conv_tol_ipea = 1e-7;
  o->diis_space = 8;
  o->damping = 0.0;
  o->prec = AGF2_FP64;
  o->compress_tol = 0.0;
  agf2_fock_opts_default(&o->fock);
  o->nblock = 1;
}

long agf2_run_state_bytes(int nphys, const agf2_run_opts* opts) {
  agf2_run_opts o;
  agf2_run_opts_default(&o);
  if (opts) o = *opts;
  if (nphys < 1 || o.diis_space < 0 || o.diis_space > 64 || o.nblock < 1 || o.nblock > 8)
    return -1;
  return (long)sizeof(RunStateHeader) + 8L * state_doubles(nphys, o.diis_space, o.nblock);
}

agf2_status agf2_run(agf2_handle_t hh, const agf2_run_opts* opts, int nphys, int naux,
                     const double* Lpq, const double* hcore, const double* e_mf, int nocc,
                     const double* dm_init, agf2_iter_record* records, int* n_records,
                     int* converged, double* e_pole, double* u_pole, int* nocc_pole,
                     double* rdm1) {
  if (!hh) return AGF2_ERR_ARG;
  return run_impl(*reinterpret_cast<Handle*>(hh), opts, nphys, naux, Lpq, hcore, e_mf, nocc,
                  dm_init, nullptr, nullptr, 0, records, n_records, converged, e_pole, u_pole,
                  nocc_pole, rdm1);
}

agf2_status agf2_run_resume(agf2_handle_t hh, const agf2_run_opts* opts, int nphys, int naux,
                            const double* Lpq, const double* hcore, const double* e_mf,
                            int nocc, const double* dm_init, const void* state_in,
                            void* state_out, int max_iter_call, agf2_iter_record* records,
                            int* n_records, int* converged, double* e_pole, double* u_pole,
                            int* nocc_pole, double* rdm1) {
  if (!hh) return AGF2_ERR_ARG;
  return run_impl(*reinterpret_cast<Handle*>(hh), opts, nphys, naux, Lpq, hcore, e_mf, nocc,
                  dm_init, state_in, state_out, max_iter_call, records, n_records, converged,
                  e_pole, u_pole, nocc_pole, rdm1);
}

}  // extern "C"
