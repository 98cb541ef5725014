// Host memory and undefined-behaviour check of the C ABI.
//
// Built together with the library's sources, with the host code of both
// compiled under AddressSanitizer and UndefinedBehaviorSanitizer (device code
// unchanged), and run on a GPU: every entry point and every host-side path of
// the library (argument checks, the Cholesky and eigen square-root
// compressions, the Lanczos-block compression, the Fock loop with its shift
// fit, first-order steps, cycle limit and DIIS, the outer loop with DIIS,
// damping, warm start, Lanczos blocks and checkpoints, the batched build's
// planning and graph replay, the warm-start network, the spectral functions,
// the kernel timers) is called on small seeded inputs, and the returned
// statuses are checked. A sanitizer finding aborts the process with a report;
// the exit status is 0 when every status was the expected one.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <vector>

#include "../include/agf2.h"

namespace {

int failures = 0;

void expect(const char* what, agf2_status got, agf2_status want, agf2_handle_t h) {
  if (got != want) {
    std::printf("FAIL %s: status %d, expected %d (%s)\n", what, (int)got, (int)want,
                h ? agf2_last_error(h) : "");
    ++failures;
  } else {
    std::printf("ok   %s\n", what);
  }
  std::fflush(stdout);
}

#define HIPCHECK(x)                                                        \
  do {                                                                     \
    if ((x) != hipSuccess) {                                               \
      std::printf("HIP failure at line %d: %s\n", __LINE__, #x);           \
      std::exit(2);                                                        \
    }                                                                      \
  } while (0)

// deterministic uniform numbers in [-1, 1)
struct Lcg {
  unsigned long long s;
  explicit Lcg(unsigned long long seed) : s(seed * 6364136223846793005ULL + 1442695040888963407ULL) {}
  double next() {
    s = s * 6364136223846793005ULL + 1442695040888963407ULL;
    return ((s >> 11) * (1.0 / 9007199254740992.0)) * 2.0 - 1.0;
  }
};

struct Dev {
  double* p = nullptr;
  size_t n = 0;
  explicit Dev(size_t n_) : n(n_) { HIPCHECK(hipMalloc(&p, (n ? n : 1) * sizeof(double))); }
  Dev(const std::vector<double>& v) : Dev(v.size()) { put(v); }
  ~Dev() { (void)hipFree(p); }
  void put(const std::vector<double>& v) {
    HIPCHECK(hipMemcpy(p, v.data(), v.size() * sizeof(double), hipMemcpyHostToDevice));
  }
  std::vector<double> get() const {
    std::vector<double> v(n);
    HIPCHECK(hipMemcpy(v.data(), p, n * sizeof(double), hipMemcpyDeviceToHost));
    return v;
  }
  Dev(const Dev&) = delete;
  Dev& operator=(const Dev&) = delete;
};

// a small synthetic system: DF tensor symmetric in (p, q) with decaying
// slices, sorted orbital energies (nocc below zero)
struct System {
  int N, Q, nocc;
  std::vector<double> L, eps;
  System(int N_, int Q_, int nocc_, unsigned seed) : N(N_), Q(Q_), nocc(nocc_) {
    Lcg r(seed);
    L.assign((size_t)Q * N * N, 0.0);
    for (int q = 0; q < Q; ++q) {
      const double s = 0.3 * std::exp(-q / 20.0) / std::sqrt((double)N);
      for (int a = 0; a < N; ++a)
        for (int b = a; b < N; ++b) {
          const double v = s * r.next();
          L[((size_t)q * N + a) * N + b] = v;
          L[((size_t)q * N + b) * N + a] = v;
        }
    }
    eps.resize(N);
    for (int i = 0; i < N; ++i)
      eps[i] = i < nocc ? -1.5 + 1.2 * (i + 0.5) / nocc : 0.1 + 2.9 * (i - nocc + 0.5) / (N - nocc);
  }
};

}  // namespace

int main() {
  int ndev = 0;
  HIPCHECK(hipGetDeviceCount(&ndev));
  if (ndev < 1) {
    std::printf("no GPU\n");
    return 2;
  }
  agf2_handle_t h = nullptr;
  expect("create", agf2_create(&h, 0, nullptr), AGF2_OK, nullptr);
  expect("create rejects a NULL out pointer", agf2_create(nullptr, 0, nullptr), AGF2_ERR_ARG,
         nullptr);
  {
    agf2_handle_t h2 = nullptr;
    expect("create rejects a negative device", agf2_create(&h2, -1, nullptr), AGF2_ERR_ARG,
           nullptr);
  }
  expect("destroy rejects NULL", agf2_destroy(nullptr), AGF2_ERR_ARG, nullptr);
  if (std::strlen(agf2_last_error(nullptr)) == 0) ++failures;
  expect("profile on", agf2_profile_enable(h, 1), AGF2_OK, h);

  System sys(24, 80, 5, 1);
  const int N = sys.N, Q = sys.Q, nocc = sys.nocc;
  const size_t nn = (size_t)N * N;
  Dev L(sys.L), eps(sys.eps);
  std::vector<double> eye(nn, 0.0), D0(nn, 0.0), heps(nn, 0.0);
  for (int i = 0; i < N; ++i) {
    eye[(size_t)i * N + i] = 1.0;
    heps[(size_t)i * N + i] = sys.eps[i];
    if (i < nocc) D0[(size_t)i * N + i] = 2.0;
  }
  Dev U(eye), Dd(D0), hdiag(heps), hcore(nn), fock(nn);
  expect("fock_build (hcore)", agf2_fock_build(h, N, Q, L.p, hdiag.p, Dd.p, -1.0, hcore.p),
         AGF2_OK, h);
  expect("fock_build rejects aliasing", agf2_fock_build(h, N, Q, L.p, hcore.p, Dd.p, 1.0, hcore.p),
         AGF2_ERR_ARG, h);
  expect("fock_build rejects nphys 0", agf2_fock_build(h, 0, Q, L.p, hcore.p, Dd.p, 1.0, fock.p),
         AGF2_ERR_ARG, h);

  // moments in every precision, then the nmom = 4 build
  Dev m(4 * nn);
  for (agf2_precision p : {AGF2_FP64, AGF2_SPLIT_BF16, AGF2_SPLIT_FP16})
    expect("build_moments", agf2_build_moments(h, p, N, Q, L.p, N, nocc, eps.p, U.p, m.p, m.p + nn,
                                               m.p + 2 * nn, m.p + 3 * nn),
           AGF2_OK, h);
  expect("build_moments rejects nocc_pole = npole",
         agf2_build_moments(h, AGF2_FP64, N, Q, L.p, N, N, eps.p, U.p, m.p, m.p + nn, m.p + 2 * nn,
                            m.p + 3 * nn),
         AGF2_ERR_ARG, h);
  Dev mo(4 * nn), mv(4 * nn);
  expect("build_moments_n (4)", agf2_build_moments_n(h, AGF2_FP64, 4, N, Q, L.p, N, nocc, eps.p,
                                                     U.p, mo.p, mv.p),
         AGF2_OK, h);
  expect("build_moments_n rejects split with 4",
         agf2_build_moments_n(h, AGF2_SPLIT_FP16, 4, N, Q, L.p, N, nocc, eps.p, U.p, mo.p, mv.p),
         AGF2_ERR_ARG, h);
  // non-finite input
  {
    std::vector<double> bad = sys.eps;
    bad[3] = NAN;
    Dev eb(bad);
    expect("build_moments rejects NaN", agf2_build_moments(h, AGF2_FP64, N, Q, L.p, N, nocc, eb.p,
                                                           U.p, m.p, m.p + nn, m.p + 2 * nn,
                                                           m.p + 3 * nn),
           AGF2_ERR_ARG, h);
    expect("rebuild", agf2_build_moments(h, AGF2_FP64, N, Q, L.p, N, nocc, eps.p, U.p, m.p,
                                         m.p + nn, m.p + 2 * nn, m.p + 3 * nn),
           AGF2_OK, h);
  }

  // compression: Cholesky, eigen square root, not positive definite, blocks
  Dev eo(N), vo(nn), ev(N), vv(nn);
  int no = 0, nv = 0;
  expect("compress lesser", agf2_compress(h, N, m.p, m.p + nn, 0.0, &no, eo.p, vo.p), AGF2_OK, h);
  expect("compress greater", agf2_compress(h, N, m.p + 2 * nn, m.p + 3 * nn, 0.0, &nv, ev.p, vv.p),
         AGF2_OK, h);
  {
    Dev e2(N), v2(nn);
    int k = 0;
    expect("compress (eigen square root)", agf2_compress(h, N, m.p, m.p + nn, 1e-12, &k, e2.p, v2.p),
           AGF2_OK, h);
    std::vector<double> z(nn, 0.0);
    for (int i = 1; i < N; ++i) z[(size_t)i * N + i] = 1.0;
    Dev zd(z);
    expect("compress rejects a singular m0", agf2_compress(h, N, zd.p, zd.p, 0.0, &k, e2.p, v2.p),
           AGF2_ERR_NOT_PD, h);
    expect("compress keeps N-1 of a singular m0",
           agf2_compress(h, N, zd.p, zd.p, 1e-12, &k, e2.p, v2.p), AGF2_OK, h);
    if (k != N - 1) ++failures;
    Dev eb(2 * N), vb(2 * nn);
    expect("compress_lanczos (2 blocks)", agf2_compress_lanczos(h, N, 4, mo.p, &k, eb.p, vb.p),
           AGF2_OK, h);
    if (k != 2 * N) ++failures;
    expect("compress_lanczos rejects odd nmom", agf2_compress_lanczos(h, N, 3, mo.p, &k, eb.p, vb.p),
           AGF2_ERR_ARG, h);
  }

  // Fock loop: defaults, cycle limit, bad electron number
  std::vector<double> ese(2 * N), vse(2 * nn);
  {
    std::vector<double> a = eo.get(), b = ev.get(), va = vo.get(), vb = vv.get();
    for (int k = 0; k < N; ++k) {
      ese[k] = a[k];
      ese[N + k] = b[k];
    }
    for (int p = 0; p < N; ++p)
      for (int k = 0; k < N; ++k) {
        vse[(size_t)p * 2 * N + k] = va[(size_t)p * N + k];
        vse[(size_t)p * 2 * N + N + k] = vb[(size_t)p * N + k];
      }
  }
  const int npole = 3 * N;
  Dev ep(npole), up((size_t)N * npole);
  int nocc_pole = 0, ncyc = 0;
  double mu = 0, shift = 0;
  {
    Dev es(ese), vs(vse), D(D0);
    expect("fock_loop", agf2_fock_loop(h, N, Q, L.p, hcore.p, 2 * nocc, 2 * N, es.p, vs.p, D.p,
                                       fock.p, ep.p, up.p, &nocc_pole, &mu, &shift, &ncyc, nullptr),
           AGF2_OK, h);
    Dev es2(ese), D2(D0);
    agf2_fock_opts o;
    agf2_fock_opts_default(&o);
    o.max_cycle = 1;
    expect("fock_loop cycle limit", agf2_fock_loop(h, N, Q, L.p, hcore.p, 2 * nocc, 2 * N, es2.p,
                                                   vs.p, D2.p, fock.p, ep.p, up.p, &nocc_pole, &mu,
                                                   &shift, &ncyc, &o),
           AGF2_ERR_NO_CONVERGE, h);
    o.diis_space = 0;
    o.max_cycle = 50;
    Dev es3(ese), D3(D0);
    expect("fock_loop without DIIS", agf2_fock_loop(h, N, Q, L.p, hcore.p, 2 * nocc, 2 * N, es3.p,
                                                    vs.p, D3.p, fock.p, ep.p, up.p, &nocc_pole,
                                                    &mu, &shift, &ncyc, &o),
           AGF2_OK, h);
    expect("fock_loop rejects odd nelec", agf2_fock_loop(h, N, Q, L.p, hcore.p, 9, 2 * N, es3.p,
                                                         vs.p, D3.p, fock.p, ep.p, up.p,
                                                         &nocc_pole, &mu, &shift, &ncyc, nullptr),
           AGF2_ERR_NELEC, h);
    // energy of the first loop's result
    double e1 = 0, e2 = 0;
    Dev eo_s(N), ev_s(N);
    {
      std::vector<double> se = es.get();
      eo_s.put(std::vector<double>(se.begin(), se.begin() + N));
      ev_s.put(std::vector<double>(se.begin() + N, se.end()));
    }
    expect("energy_gf", agf2_energy_gf(h, N, hcore.p, fock.p, D.p, npole, nocc_pole, ep.p, up.p, N,
                                       eo_s.p, vo.p, N, ev_s.p, vv.p, &e1, &e2),
           AGF2_OK, h);
    if (!std::isfinite(e1 + e2)) ++failures;
  }

  // spectral function, allocating and allocation-free
  {
    std::vector<double> om(777);
    for (size_t k = 0; k < om.size(); ++k) om[k] = -3.0 + 6.0 * k / om.size();
    Dev omd(om), A(om.size()), B(om.size()), wt(N);
    expect("spectral_function", agf2_spectral_function(h, N, npole, ep.p, up.p, nullptr,
                                                       (int)om.size(), omd.p, 0.01, A.p),
           AGF2_OK, h);
    expect("spectral_function_noalloc", agf2_spectral_function_noalloc(
                                            h, N, npole, ep.p, up.p, nullptr, (int)om.size(),
                                            omd.p, 0.01, B.p),
           AGF2_OK, h);
    if (A.get() != B.get()) ++failures;
    expect("spectral_function_noalloc rejects too many poles",
           agf2_spectral_function_noalloc(h, N, AGF2_SPECTRUM_NOALLOC_MAX_POLE + 1, ep.p, up.p,
                                          nullptr, 4, omd.p, 0.01, B.p),
           AGF2_ERR_ARG, h);
    expect("spectral_function rejects eta 0", agf2_spectral_function(h, N, npole, ep.p, up.p,
                                                                     nullptr, 4, omd.p, 0.0, A.p),
           AGF2_ERR_ARG, h);
  }

  // outer loop: DIIS, damping, split precision, Lanczos blocks, checkpoints
  {
    std::vector<agf2_iter_record> rec(64);
    int nrec = 0, conv = 0, nop = 0;
    Dev e_out(5 * N), u_out((size_t)N * 5 * N), rdm(nn);
    agf2_run_opts o;
    agf2_run_opts_default(&o);
    expect("run", agf2_run(h, &o, N, Q, L.p, hcore.p, eps.p, nocc, nullptr, rec.data(), &nrec,
                           &conv, e_out.p, u_out.p, &nop, rdm.p),
           AGF2_OK, h);
    o.damping = 0.2;
    o.prec = AGF2_SPLIT_FP16;
    expect("run (split, damping)", agf2_run(h, &o, N, Q, L.p, hcore.p, eps.p, nocc, nullptr,
                                            rec.data(), &nrec, &conv, e_out.p, u_out.p, &nop,
                                            rdm.p),
           AGF2_OK, h);
    agf2_run_opts_default(&o);
    o.nblock = 2;
    expect("run (two Lanczos blocks)", agf2_run(h, &o, N, Q, L.p, hcore.p, eps.p, nocc, nullptr,
                                                rec.data(), &nrec, &conv, e_out.p, u_out.p, &nop,
                                                rdm.p),
           AGF2_OK, h);
    std::vector<unsigned char> st((size_t)agf2_run_state_bytes(N, &o));
    expect("run_resume (first two iterations)",
           agf2_run_resume(h, &o, N, Q, L.p, hcore.p, eps.p, nocc, nullptr, nullptr, st.data(), 2,
                           rec.data(), &nrec, &conv, e_out.p, u_out.p, &nop, rdm.p),
           AGF2_OK, h);
    expect("run_resume (rest)",
           agf2_run_resume(h, &o, N, Q, L.p, hcore.p, eps.p, nocc, nullptr, st.data(), st.data(), 0,
                           rec.data(), &nrec, &conv, e_out.p, u_out.p, &nop, rdm.p),
           AGF2_OK, h);
    std::vector<unsigned char> junk(st.size(), 7);
    expect("run_resume rejects a foreign state",
           agf2_run_resume(h, &o, N, Q, L.p, hcore.p, eps.p, nocc, nullptr, junk.data(), nullptr,
                           0, rec.data(), &nrec, &conv, e_out.p, u_out.p, &nop, rdm.p),
           AGF2_ERR_ARG, h);
    agf2_run_opts_default(&o);
    o.fock.max_cycle = 1;
    expect("run stops on a failed Fock loop",
           agf2_run(h, &o, N, Q, L.p, hcore.p, eps.p, nocc, nullptr, rec.data(), &nrec, &conv,
                    e_out.p, u_out.p, &nop, rdm.p),
           AGF2_ERR_NO_CONVERGE, h);
    agf2_run_opts_default(&o);
    o.max_iter = 1;
    expect("run reaches max_iter", agf2_run(h, &o, N, Q, L.p, hcore.p, eps.p, nocc, nullptr,
                                            rec.data(), &nrec, &conv, e_out.p, u_out.p, &nop,
                                            rdm.p),
           AGF2_ERR_NO_CONVERGE, h);
    Dev dm(4 * nn);
    std::vector<double> z(4 * nn, 0.0);
    for (int i = 0; i < N; ++i) z[(size_t)i * N + i] = -1e3;   // breaks positive definiteness
    dm.put(z);
    agf2_run_opts_default(&o);
    expect("run with a failing warm start", agf2_run(h, &o, N, Q, L.p, hcore.p, eps.p, nocc, dm.p,
                                                     rec.data(), &nrec, &conv, e_out.p, u_out.p,
                                                     &nop, rdm.p),
           AGF2_OK, h);
  }

  // a larger Fock loop: 900 x 900 extended matrices
  {
    System big(300, 200, 60, 2);
    const size_t bn = (size_t)big.N * big.N;
    Dev BL(big.L), Beps(big.eps);
    std::vector<double> e2(bn, 0.0), d2(bn, 0.0), hd(bn, 0.0);
    for (int i = 0; i < big.N; ++i) {
      e2[(size_t)i * big.N + i] = 1.0;
      hd[(size_t)i * big.N + i] = big.eps[i];
      if (i < big.nocc) d2[(size_t)i * big.N + i] = 2.0;
    }
    Dev BU(e2), BD(d2), Bh(hd), Bhc(bn), Bf(bn), Bm(4 * bn), beo(big.N), bvo(bn), bev(big.N),
        bvv(bn);
    expect("fock_build (300)", agf2_fock_build(h, big.N, big.Q, BL.p, Bh.p, BD.p, -1.0, Bhc.p),
           AGF2_OK, h);
    expect("build_moments (300, fp16)",
           agf2_build_moments(h, AGF2_SPLIT_FP16, big.N, big.Q, BL.p, big.N, big.nocc, Beps.p,
                              BU.p, Bm.p, Bm.p + bn, Bm.p + 2 * bn, Bm.p + 3 * bn),
           AGF2_OK, h);
    int a = 0, b = 0;
    expect("compress (300)", agf2_compress(h, big.N, Bm.p, Bm.p + bn, 0.0, &a, beo.p, bvo.p),
           AGF2_OK, h);
    expect("compress (300)", agf2_compress(h, big.N, Bm.p + 2 * bn, Bm.p + 3 * bn, 0.0, &b, bev.p,
                                           bvv.p),
           AGF2_OK, h);
    std::vector<double> es(2 * big.N), vs(2 * bn);
    std::vector<double> ha = beo.get(), hb = bev.get(), va = bvo.get(), vb = bvv.get();
    for (int k = 0; k < big.N; ++k) {
      es[k] = ha[k];
      es[big.N + k] = hb[k];
    }
    for (int p = 0; p < big.N; ++p)
      for (int k = 0; k < big.N; ++k) {
        vs[(size_t)p * 2 * big.N + k] = va[(size_t)p * big.N + k];
        vs[(size_t)p * 2 * big.N + big.N + k] = vb[(size_t)p * big.N + k];
      }
    Dev esd(es), vsd(vs), Dl(d2), bep(3 * big.N), bup((size_t)big.N * 3 * big.N);
    expect("fock_loop (900 x 900)",
           agf2_fock_loop(h, big.N, big.Q, BL.p, Bhc.p, 2 * big.nocc, 2 * big.N, esd.p, vsd.p, Dl.p,
                          Bf.p, bep.p, bup.p, &nocc_pole, &mu, &shift, &ncyc, nullptr),
           AGF2_OK, h);
  }

  // batched build: plan, capture and replay; then a changed batch
  {
    System s1(40, 140, 8, 3), s2(56, 196, 11, 4);
    Dev L1(s1.L), L2(s2.L), e1(s1.eps), e2(s2.eps);
    std::vector<double> i1((size_t)40 * 40, 0.0), i2((size_t)56 * 56, 0.0);
    for (int i = 0; i < 40; ++i) i1[(size_t)i * 40 + i] = 1.0;
    for (int i = 0; i < 56; ++i) i2[(size_t)i * 56 + i] = 1.0;
    Dev u1(i1), u2(i2), o1(4 * 1600), o2(4 * 56 * 56);
    agf2_system sy[2];
    sy[0] = agf2_system{40, 140, L1.p, 40, 8, e1.p, u1.p, o1.p, o1.p + 1600, o1.p + 3200,
                        o1.p + 4800};
    sy[1] = agf2_system{56, 196, L2.p, 56, 11, e2.p, u2.p, o2.p, o2.p + 3136, o2.p + 6272,
                        o2.p + 9408};
    int tw[2] = {0, 0};
    expect("batched (plan)", agf2_build_moments_batched(h, 2, sy, tw), AGF2_OK, h);
    expect("batched (replay)", agf2_build_moments_batched(h, 2, sy, tw), AGF2_OK, h);
    expect("batched (one system)", agf2_build_moments_batched(h, 1, sy, tw), AGF2_OK, h);
    expect("batched rejects 0 systems", agf2_build_moments_batched(h, 0, sy, tw), AGF2_ERR_ARG, h);
  }

  // warm-start network
  {
    agf2_mlp_t net = nullptr;
    expect("mlp_create", agf2_mlp_create(h, &net), AGF2_OK, h);
    std::vector<float> par(AGF2_MLP_NPARAM);
    Lcg r(9);
    for (auto& x : par) x = (float)(0.05 * r.next());
    expect("mlp_set_params", agf2_mlp_set_params(h, net, par.data()), AGF2_OK, h);
    float *X = nullptr, *Y = nullptr, *dY = nullptr;
    double *sc = nullptr, *loss = nullptr;
    HIPCHECK(hipMalloc(&X, (size_t)N * AGF2_MLP_FEATURES * sizeof(float)));
    HIPCHECK(hipMalloc(&Y, (size_t)N * AGF2_MLP_OUTPUTS * sizeof(float)));
    HIPCHECK(hipMalloc(&dY, (size_t)N * AGF2_MLP_OUTPUTS * sizeof(float)));
    HIPCHECK(hipMalloc(&sc, 4 * sizeof(double)));
    HIPCHECK(hipMalloc(&loss, sizeof(double)));
    HIPCHECK(hipMemset(loss, 0, sizeof(double)));
    expect("mlp_features", agf2_mlp_features(h, N, nocc, eps.p, m.p, X, sc), AGF2_OK, h);
    expect("mlp_forward", agf2_mlp_forward(h, net, N, X, Y), AGF2_OK, h);
    expect("mlp_loss_grad", agf2_mlp_loss_grad(h, N, Y, m.p, m.p, sc, dY, loss), AGF2_OK, h);
    expect("mlp_backward", agf2_mlp_backward(h, net, N, dY), AGF2_OK, h);
    expect("mlp_adam_step", agf2_mlp_adam_step(h, net, 1e-3f, 0.9f, 0.999f, 1e-8f), AGF2_OK, h);
    expect("mlp_get_grad", agf2_mlp_get_grad(h, net, par.data()), AGF2_OK, h);
    expect("mlp_get_params", agf2_mlp_get_params(h, net, par.data()), AGF2_OK, h);
    Dev dmo(4 * nn);
    expect("mlp_predict_correction",
           agf2_mlp_predict_correction(h, net, N, nocc, eps.p, m.p, dmo.p), AGF2_OK, h);
    expect("mlp_forward rejects 0 rows", agf2_mlp_forward(h, net, 0, X, Y), AGF2_ERR_ARG, h);
    expect("mlp_destroy", agf2_mlp_destroy(net), AGF2_OK, h);
    (void)hipFree(X);
    (void)hipFree(Y);
    (void)hipFree(dY);
    (void)hipFree(sc);
    (void)hipFree(loss);
  }

  // timers
  {
    const int n = agf2_profile_count(h);
    if (n <= 0) ++failures;
    for (int i = 0; i < n; ++i) {
      const char* name = nullptr;
      long launches = 0;
      double ms = 0, fl = 0, by = 0;
      expect("profile_get", agf2_profile_get(h, i, &name, &launches, &ms, &fl, &by), AGF2_OK, h);
    }
    const char* name = nullptr;
    long launches = 0;
    double ms = 0, fl = 0, by = 0;
    expect("profile_get rejects a bad index",
           agf2_profile_get(h, n, &name, &launches, &ms, &fl, &by), AGF2_ERR_ARG, h);
    expect("profile off", agf2_profile_enable(h, 0), AGF2_OK, h);
  }
  expect("synchronize", agf2_synchronize(h), AGF2_OK, h);
  expect("destroy", agf2_destroy(h), AGF2_OK, nullptr);
  std::printf("%s: %d failure(s)\n", failures ? "FAILED" : "PASSED", failures);
  return failures ? 1 : 0;
}
