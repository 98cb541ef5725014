// Batched FP64 moment build over systems of uneven size (agf2_build_moments_batched).
//
// A job is one part (lesser or greater) of one system. Every system keeps its
// own pole-basis tensors and every job its own Z buffer and split-K partials
// in one workspace. The pole pairs of each job are cut into R rounds of about
// equal Z width, R chosen so that all jobs' Z buffers fit one budget. Round r
// runs one persistent grouped slab launch per inner-tile width over the round-r
// tiles of every job, then one persistent grouped SYRK launch over them; the
// SYRK adds into the partials, which are summed once at the end in a fixed
// order. Within a launch, jobs are ordered by the cost of one tile, most
// expensive first, and workgroups stride over the concatenated tiles.
//
// The sequence (transforms, zero fill, rounds, reductions) is captured once
// into a HIP graph and replayed while the batch (sizes and pointers) stays the
// same; values behind the pointers may change between calls. Before capture,
// the slab's inner-tile width is chosen per size bucket by timing each
// candidate on the batch's first round.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <exception>
#include <memory>
#include <new>

#include "agf2_internal.h"

namespace agf2 {

struct SysKey {
  int N, Q, npole, nocc;
  const void *L, *e, *u, *m0o, *m1o, *m0v, *m1v;
  bool operator==(const SysKey& o) const {
    return N == o.N && Q == o.Q && npole == o.npole && nocc == o.nocc && L == o.L && e == o.e &&
           u == o.u && m0o == o.m0o && m1o == o.m1o && m0v == o.m0v && m1v == o.m1v;
  }
};

struct BatchPlan {
  std::vector<SysKey> key;
  DevBuf ws, pairs, tables;
  hipStream_t stream = nullptr;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  hipEvent_t ev_in = nullptr, ev_out = nullptr;
  std::vector<int> tile_width;   // greater-part width per system
  int rounds = 0;
  double flops = 0.0;            // canonical flops of one build
  ~BatchPlan() {
    if (exec) (void)hipGraphExecDestroy(exec);
    if (graph) (void)hipGraphDestroy(graph);
    if (ev_in) (void)hipEventDestroy(ev_in);
    if (ev_out) (void)hipEventDestroy(ev_out);
    if (stream) (void)hipStreamDestroy(stream);
    ws.release();
    pairs.release();
    tables.release();
  }
};

void destroy_batch_plan(BatchPlan* p) {
  if (p) (void)hipDeviceSynchronize();   // a replay may still be running
  delete p;
}

namespace {

constexpr int BK = 16, TB = 64;
constexpr long ZBUDGET_MAX = 32L << 30;   // bytes of Z over all jobs per round

inline long align64(long n) { return (n + 63) / 64 * 64; }
inline long round16(long n) { return (n + BK - 1) / BK * BK; }

int bucket_of(int nc) { return nc <= 16 ? 0 : nc <= 32 ? 1 : nc <= 64 ? 2 : 3; }

struct Job {
  int sys, part;              // part 0 lesser, 1 greater
  int N, np, nc, Qp, Q;
  long npairs, K;
  long off_pairs;             // into the pair tables
  std::vector<long> colp;     // column offset of each pair, colp[npairs] = K
  std::vector<long> pstart;   // first pair of each round, pstart[R] = npairs
  long cap = 0;               // Z columns (widest round)
  int nsplit = 1; long kper = 0;
  long off_Z = 0, off_part = 0;
  int tc = 16;
  int tiles_n, nlower;
};

void transform_system(hipStream_t st, int N, int Q, int Qp, const double* L, const double* u,
                      int npole, int o, double* Lxo, double* Lxv, double* Lov) {
  const int v = npole - o;
  pole_transform_f64(N, Q, Qp, L, u, npole, 0, o, Lxo, st);
  pole_transform_f64(N, Q, Qp, L, u, npole, o, v, Lxv, st);
  lov_transform_f64(N, Q, Qp, u, npole, o, v, Lxv, Lov, st);
}

// Host blob of launch tables (job structs and tile prefixes), uploaded once.
struct Blob {
  std::vector<char> bytes;
  template <class T> long put(const T* p, long n) {
    const long off = (long)((bytes.size() + 255) / 256 * 256);
    bytes.resize(off + n * sizeof(T));
    std::memcpy(bytes.data() + off, p, n * sizeof(T));
    return off;
  }
};

struct Launch {
  int kind = 0;      // 0 slab, 1 syrk
  int tc = 0;
  long off_jobs = 0, off_prefix = 0;
  int njobs = 0;
  long total = 0;
};

}  // namespace

static BatchPlan* build_plan(int nsys, const agf2_system* sys) {
  std::unique_ptr<BatchPlan> plan(new BatchPlan());
  AGF2_HIP(hipStreamCreateWithFlags(&plan->stream, hipStreamNonBlocking));
  AGF2_HIP(hipEventCreateWithFlags(&plan->ev_in, hipEventDisableTiming));
  AGF2_HIP(hipEventCreateWithFlags(&plan->ev_out, hipEventDisableTiming));
  hipStream_t st = plan->stream;

  // ---- jobs, pair tables, canonical flops
  std::vector<Job> jobs;
  long npairs_tot = 0;
  for (int s = 0; s < nsys; ++s) {
    const agf2_system& y = sys[s];
    plan->key.push_back(SysKey{y.nphys, y.naux, y.npole, y.nocc_pole, y.Lpq, y.e_pole, y.u_pole,
                               y.m0_occ, y.m1_occ, y.m0_vir, y.m1_vir});
    const int o = y.nocc_pole, v = y.npole - y.nocc_pole;
    plan->flops += 2.0 * y.nphys * (double)o * v * (o + v) * (y.naux + 2.0 * y.nphys);
    for (int part = 0; part < 2; ++part) {
      Job j;
      j.sys = s; j.part = part; j.N = y.nphys; j.Q = y.naux; j.Qp = (int)round16(y.naux);
      j.np = part == 0 ? o : v;
      j.nc = part == 0 ? v : o;
      j.npairs = (long)j.np * (j.np + 1) / 2;
      j.colp.reserve(j.npairs + 1);
      long c = 0;
      for (int p = 0; p < j.np; ++p)
        for (int q = p; q < j.np; ++q) {
          j.colp.push_back(c);
          c += (p == q) ? j.nc : 2L * j.nc;
        }
      j.colp.push_back(c);
      j.K = c;
      j.off_pairs = npairs_tot;
      npairs_tot += j.npairs;
      j.tiles_n = (j.N + TB - 1) / TB;
      j.nlower = j.tiles_n * (j.tiles_n + 1) / 2;
      j.tc = slab_f64_tc(j.nc);
      jobs.push_back(std::move(j));
    }
  }
  const int njobs = (int)jobs.size();
  {
    std::vector<int> hpi(npairs_tot), hpj(npairs_tot);
    std::vector<long> hcol(npairs_tot);
    for (const Job& j : jobs) {
      long k = j.off_pairs;
      for (int p = 0; p < j.np; ++p)
        for (int q = p; q < j.np; ++q, ++k) {
          hpi[k] = p; hpj[k] = q; hcol[k] = j.colp[k - j.off_pairs];
        }
    }
    char* T = static_cast<char*>(plan->pairs.get(npairs_tot * (2 * sizeof(int) + sizeof(long))));
    AGF2_HIP(hipMemcpy(T, hcol.data(), npairs_tot * sizeof(long), hipMemcpyHostToDevice));
    AGF2_HIP(hipMemcpy(T + npairs_tot * sizeof(long), hpi.data(), npairs_tot * sizeof(int),
                       hipMemcpyHostToDevice));
    AGF2_HIP(hipMemcpy(T + npairs_tot * (sizeof(long) + sizeof(int)), hpj.data(),
                       npairs_tot * sizeof(int), hipMemcpyHostToDevice));
  }
  const long* dcol = static_cast<const long*>(plan->pairs.ptr);
  const int* dpi = reinterpret_cast<const int*>(dcol + npairs_tot);
  const int* dpj = dpi + npairs_tot;

  // ---- workspace: tensors, partials, then Z for R rounds within the budget
  std::vector<long> off_xo(nsys), off_xv(nsys), off_ov(nsys);
  long ws = 0;
  for (int s = 0; s < nsys; ++s) {
    const agf2_system& y = sys[s];
    const long N = y.nphys, Qp = round16(y.naux), o = y.nocc_pole, v = y.npole - y.nocc_pole;
    off_xo[s] = ws; ws += align64(o * N * Qp);
    off_xv[s] = ws; ws += align64(v * N * Qp);
    off_ov[s] = ws; ws += align64(o * v * Qp);
  }
  size_t free_b = 0, total_b = 0;
  AGF2_HIP(hipMemGetInfo(&free_b, &total_b));
  double zneed = 0.0;
  for (const Job& j : jobs) zneed += 8.0 * (j.N + 1.0) * (double)j.K;
  const double tens_b = 8.0 * ws;
  const double zbudget =
      std::min<double>((double)ZBUDGET_MAX, 0.5 * ((double)free_b - tens_b - (double)(1L << 30)));
  if (zbudget < (double)(256L << 20))
    throw Error{AGF2_ERR_NOMEM, "batched moments: not enough device memory for the batch"};
  int R = std::max(1, (int)std::ceil(zneed / zbudget));
  for (;;) {
    double ztot = 0.0;
    for (Job& j : jobs) {
      const long target = (j.K + R - 1) / R;
      j.pstart.assign(R + 1, j.npairs);
      j.pstart[0] = 0;
      long P = 0;
      for (int r = 1; r < R; ++r) {
        while (P < j.npairs && j.colp[P] < (long)r * target) ++P;
        j.pstart[r] = P;
      }
      j.cap = 0;
      for (int r = 0; r < R; ++r)
        j.cap = std::max(j.cap, j.colp[j.pstart[r + 1]] - j.colp[j.pstart[r]]);
      j.cap = round16(std::max<long>(j.cap, 1));
      ztot += 8.0 * (j.N + 1.0) * (double)j.cap;
    }
    if (ztot <= zbudget || R >= 4096) break;
    R = std::max(R + 1, (int)(R * 1.1));
  }
  plan->rounds = R;
  for (Job& j : jobs) {
    j.nsplit = (int)std::max<long>(1, std::min<long>(64, (j.cap + 4095) / 4096));
    j.kper = round16((j.cap + j.nsplit - 1) / j.nsplit);
    j.nsplit = (int)((j.cap + j.kper - 1) / j.kper);
  }
  const long off_parts = ws;
  for (Job& j : jobs) {
    j.off_part = ws;
    ws += align64((long)j.nsplit * 2 * (long)j.N * j.N);
  }
  const long nparts_total = ws - off_parts;
  for (Job& j : jobs) {
    j.off_Z = ws;
    ws += align64((long)j.N * j.cap + j.cap);
  }
  double* W = plan->ws.as<double>(ws);

  auto slab_job = [&](const Job& j, int tc, int r) {
    const agf2_system& y = sys[j.sys];
    const int N = j.N, o = y.nocc_pole, v = y.npole - y.nocc_pole;
    SlabF64 a{};
    if (j.part == 0) {   // lesser: R = Lxo[i][x][Q], S[j][a][Q] = Lov[j][a][Q]
      a.R = W + off_xo[j.sys]; a.sRp = (long)N * j.Qp; a.sRx = j.Qp;
      a.S = W + off_ov[j.sys]; a.sSp = (long)v * j.Qp; a.sSc = j.Qp;
      a.ep = y.e_pole; a.ec = y.e_pole + o;
    } else {             // greater: R = Lxv[a][x][Q], S[b][i][Q] = Lov[i][b][Q]
      a.R = W + off_xv[j.sys]; a.sRp = (long)N * j.Qp; a.sRx = j.Qp;
      a.S = W + off_ov[j.sys]; a.sSp = j.Qp; a.sSc = (long)v * j.Qp;
      a.ep = y.e_pole + o; a.ec = y.e_pole;
    }
    a.N = N; a.nc = j.nc; a.Qp = j.Qp;
    a.pi = dpi + j.off_pairs; a.pj = dpj + j.off_pairs; a.pcol = dcol + j.off_pairs;
    a.pair0 = (int)j.pstart[r]; a.npairs = (int)(j.pstart[r + 1] - j.pstart[r]);
    a.col_base = j.colp[j.pstart[r]];
    a.Z = W + j.off_Z; a.ldz = j.cap; a.w = W + j.off_Z + (long)N * j.cap;
    a.tiles_x = j.tiles_n; a.tiles_c = (j.nc + tc - 1) / tc;
    return a;
  };
  auto syrk_job = [&](const Job& j, int r) {
    SyrkF64 y{};
    y.Z = W + j.off_Z; y.ldz = j.cap; y.w = W + j.off_Z + (long)j.N * j.cap;
    y.N = j.N; y.K = j.colp[j.pstart[r + 1]] - j.colp[j.pstart[r]];
    y.kper = j.kper; y.nsplit = (int)((y.K + j.kper - 1) / j.kper);
    y.part = W + j.off_part; y.part_stride = 2L * j.N * j.N; y.tiles = j.nlower;
    return y;
  };
  // job order within a launch: per-tile cost, most expensive first
  std::vector<int> slab_order(njobs), syrk_order(njobs);
  for (int k = 0; k < njobs; ++k) slab_order[k] = syrk_order[k] = k;
  std::stable_sort(slab_order.begin(), slab_order.end(),
                   [&](int a, int b) { return jobs[a].Qp > jobs[b].Qp; });
  std::stable_sort(syrk_order.begin(), syrk_order.end(),
                   [&](int a, int b) { return jobs[a].kper > jobs[b].kper; });
  // one launch's tables: jobs (in cost order) selected by `use`, round r
  auto add_slab = [&](Blob& b, int tc, int r, const std::vector<char>& use, Launch& L) {
    std::vector<SlabF64> js;
    std::vector<long> pre{0};
    for (int k : slab_order) {
      if (!use[k]) continue;
      SlabF64 a = slab_job(jobs[k], tc, r);
      if (a.npairs == 0) continue;
      js.push_back(a);
      pre.push_back(pre.back() + slab_f64_tiles(a));
    }
    L.kind = 0; L.tc = tc; L.njobs = (int)js.size(); L.total = pre.back();
    L.off_jobs = js.empty() ? 0 : b.put(js.data(), (long)js.size());
    L.off_prefix = b.put(pre.data(), (long)pre.size());
  };
  auto add_syrk = [&](Blob& b, int r, Launch& L) {
    std::vector<SyrkF64> js;
    std::vector<long> pre{0};
    for (int k : syrk_order) {
      SyrkF64 y = syrk_job(jobs[k], r);
      if (y.K == 0) continue;
      js.push_back(y);
      pre.push_back(pre.back() + (long)y.tiles * y.nsplit);
    }
    L.kind = 1; L.tc = 0; L.njobs = (int)js.size(); L.total = pre.back();
    L.off_jobs = js.empty() ? 0 : b.put(js.data(), (long)js.size());
    L.off_prefix = b.put(pre.data(), (long)pre.size());
  };
  auto run = [&](const Launch& L, const char* base) {
    if (L.total == 0) return;
    if (L.kind == 0)
      launch_slab_f64_grouped(L.tc, reinterpret_cast<const SlabF64*>(base + L.off_jobs),
                              reinterpret_cast<const long*>(base + L.off_prefix), L.njobs,
                              L.total, grouped_grid_f64(0, L.tc), st);
    else
      launch_syrk_f64_grouped(reinterpret_cast<const SyrkF64*>(base + L.off_jobs),
                              reinterpret_cast<const long*>(base + L.off_prefix), L.njobs,
                              L.total, grouped_grid_f64(1, 0), st);
  };

  // ---- eager transforms (the autotuner's slabs read them)
  for (int s = 0; s < nsys; ++s) {
    const agf2_system& y = sys[s];
    transform_system(st, y.nphys, y.naux, (int)round16(y.naux), y.Lpq, y.u_pole, y.npole,
                     y.nocc_pole, W + off_xo[s], W + off_xv[s], W + off_ov[s]);
  }
  AGF2_HIP(hipStreamSynchronize(st));

  // ---- autotuner: slab inner-tile width per size bucket, timed on round 0
  {
    hipEvent_t t0 = nullptr, t1 = nullptr;
    DevBuf tune;
    try {
      AGF2_HIP(hipEventCreate(&t0));
      AGF2_HIP(hipEventCreate(&t1));
      for (int bkt = 0; bkt < 4; ++bkt) {
        std::vector<char> use(njobs, 0);
        bool any = false;
        for (int k = 0; k < njobs; ++k)
          if (bucket_of(jobs[k].nc) == bkt) use[k] = 1, any = true;
        if (!any) continue;
        float best = 1e30f;
        int best_tc = -1;
        for (int tc : {16, 32, 64}) {
          Blob b;
          Launch L;
          add_slab(b, tc, 0, use, L);
          if (L.total == 0) continue;
          char* d = static_cast<char*>(tune.get(b.bytes.size()));
          AGF2_HIP(hipMemcpy(d, b.bytes.data(), b.bytes.size(), hipMemcpyHostToDevice));
          float ms = 1e30f;
          for (int rep = 0; rep < 2; ++rep) {
            AGF2_HIP(hipEventRecord(t0, st));
            run(L, d);
            AGF2_HIP(hipEventRecord(t1, st));
            AGF2_HIP(hipEventSynchronize(t1));
            float m = 0.f;
            AGF2_HIP(hipEventElapsedTime(&m, t0, t1));
            ms = std::min(ms, m);
          }
          if (ms < best) best = ms, best_tc = tc;
        }
        if (best_tc > 0)
          for (int k = 0; k < njobs; ++k)
            if (use[k]) jobs[k].tc = best_tc;
      }
    } catch (...) {
      if (t0) (void)hipEventDestroy(t0);
      if (t1) (void)hipEventDestroy(t1);
      tune.release();
      throw;
    }
    (void)hipEventDestroy(t0);
    (void)hipEventDestroy(t1);
    tune.release();
  }
  plan->tile_width.assign(nsys, 0);
  for (const Job& j : jobs)
    if (j.part == 1) plan->tile_width[j.sys] = j.tc;

  // ---- launch tables for every round
  Blob blob;
  std::vector<Launch> launches;
  for (int r = 0; r < R; ++r) {
    for (int tc : {16, 32, 64}) {
      std::vector<char> use(njobs, 0);
      for (int k = 0; k < njobs; ++k) use[k] = jobs[k].tc == tc;
      Launch L;
      add_slab(blob, tc, r, use, L);
      if (L.total > 0) launches.push_back(L);
    }
    Launch L;
    add_syrk(blob, r, L);
    if (L.total > 0) launches.push_back(L);
  }
  char* dtab = static_cast<char*>(plan->tables.get(blob.bytes.size()));
  AGF2_HIP(hipMemcpy(dtab, blob.bytes.data(), blob.bytes.size(), hipMemcpyHostToDevice));

  // device-filling grids, queried before capture
  for (int tc : {16, 32, 64}) (void)grouped_grid_f64(0, tc);
  (void)grouped_grid_f64(1, 0);

  // ---- capture the build
  AGF2_HIP(hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal));
  try {
    for (int s = 0; s < nsys; ++s) {
      const agf2_system& y = sys[s];
      transform_system(st, y.nphys, y.naux, (int)round16(y.naux), y.Lpq, y.u_pole, y.npole,
                       y.nocc_pole, W + off_xo[s], W + off_xv[s], W + off_ov[s]);
    }
    fill_zero(W + off_parts, nparts_total, st);
    for (const Launch& L : launches) run(L, dtab);
    for (const Job& j : jobs) {
      const agf2_system& y = sys[j.sys];
      reduce_moment_partials(W + j.off_part, 2L * j.N * j.N, j.nsplit, j.N,
                             j.part == 0 ? y.m0_occ : y.m0_vir,
                             j.part == 0 ? y.m1_occ : y.m1_vir, st);
    }
  } catch (...) {
    hipGraph_t g = nullptr;
    (void)hipStreamEndCapture(st, &g);   // leave the stream usable before unwinding
    if (g) (void)hipGraphDestroy(g);
    throw;
  }
  AGF2_HIP(hipStreamEndCapture(st, &plan->graph));
  AGF2_HIP(hipGraphInstantiate(&plan->exec, plan->graph, nullptr, nullptr, 0));
  return plan.release();
}

}  // namespace agf2

using namespace agf2;

extern "C" agf2_status agf2_build_moments_batched(agf2_handle_t hh, int nsys,
                                                  const agf2_system* sys, int* tile_width) {
  if (!hh) return AGF2_ERR_ARG;
  Handle& h = *reinterpret_cast<Handle*>(hh);
  try {
    int prev = 0;
    (void)hipGetDevice(&prev);
    AGF2_HIP(hipSetDevice(h.device));
    struct Restore {
      int d;
      ~Restore() { (void)hipSetDevice(d); }
    } restore{prev};
    AGF2_REQUIRE(nsys >= 1 && sys, "need at least one system");
    std::vector<SysKey> key;
    for (int s = 0; s < nsys; ++s) {
      const agf2_system& y = sys[s];
      AGF2_REQUIRE(y.nphys >= 1 && y.naux >= 1 && y.npole >= 2 && y.nocc_pole >= 1 &&
                       y.nocc_pole < y.npole,
                   "bad system sizes");
      AGF2_REQUIRE(y.nphys <= 65535, "nphys too large");
      AGF2_REQUIRE(y.Lpq && y.e_pole && y.u_pole && y.m0_occ && y.m1_occ && y.m0_vir &&
                       y.m1_vir,
                   "NULL system pointer");
      key.push_back(SysKey{y.nphys, y.naux, y.npole, y.nocc_pole, y.Lpq, y.e_pole, y.u_pole,
                           y.m0_occ, y.m1_occ, y.m0_vir, y.m1_vir});
    }
    // non-finite inputs are rejected on every call (the graph replays the
    // arrays' current values)
    for (int s0 = 0; s0 < nsys; s0 += 10) {
      FiniteCheck chk(h);
      for (int s = s0; s < std::min(nsys, s0 + 10); ++s) {
        const agf2_system& y = sys[s];
        chk.add(y.Lpq, (long)y.naux * y.nphys * y.nphys, "Lpq of a batched system")
            .add(y.e_pole, y.npole, "e_pole of a batched system")
            .add(y.u_pole, (long)y.nphys * y.npole, "u_pole of a batched system");
      }
      chk.run();
    }
    if (!h.batch || !(h.batch->key == key)) {
      destroy_batch_plan(h.batch);
      h.batch = nullptr;
      h.batch = build_plan(nsys, sys);
    }
    BatchPlan& p = *h.batch;
    // the replay runs after the handle stream's earlier work, and the handle
    // stream's later work after the replay
    AGF2_HIP(hipEventRecord(p.ev_in, h.stream));
    AGF2_HIP(hipStreamWaitEvent(p.stream, p.ev_in, 0));
    {
      ProfScope ps(h, "moments.batched", p.flops, 0.0);
      AGF2_HIP(hipGraphLaunch(p.exec, p.stream));
      AGF2_HIP(hipEventRecord(p.ev_out, p.stream));
      AGF2_HIP(hipStreamWaitEvent(h.stream, p.ev_out, 0));
    }
    if (tile_width)
      for (int s = 0; s < nsys; ++s) tile_width[s] = p.tile_width[s];
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
