// FP64 self-energy moment build (zeroth/first moment equations; lesser and
// greater parts of the second-order self-energy).
//
// For one part, with "pair" poles p, q (occupied for the lesser part, virtual
// for the greater part) and "inner" poles c of the other kind:
//   X^{pq}[x][c] = (xp|qc) = sum_Q R[p][x][Q] S[q][c][Q]
//   U0 = sum_{p,q} X^{pq} (2 X^{pq} - X^{qp})^T
//   U1 = same with the weight e_p + e_q - e_c on column c
// Pairing (p,q) with (q,p) turns the summand into a sum of squares,
//   X^{pq}(2X^{pq}-X^{qp})^T + X^{qp}(2X^{qp}-X^{pq})^T
//     = 1/2 (X^{pq}+X^{qp})(...)^T + 3/2 (X^{pq}-X^{qp})(...)^T,
// and X^{pp} X^{pp T} for p = q. The build therefore runs in two kernels:
//   slab:  one workgroup owns a pair p<q and an (x, c) tile (64 x TC). It
//          forms X^{pq} and X^{qp} for that tile in two MFMA accumulators over
//          Q (LDS-staged operand tiles), so each exchange partner (xq|pc) sits
//          in the same lane and register as its direct term (xp|qc). The
//          epilogue writes the columns sqrt(1/2)(X^{pq}+X^{qp}) and
//          sqrt(3/2)(X^{pq}-X^{qp}) of Z and their weight.
//   syrk:  U0 += Z Z^T and U1 += Z diag(w) Z^T on lower-triangle tiles,
//          split over K into per-split float64 partials (no atomics).
// Tile bodies are device functions shared by one-job launches and by the
// persistent grouped launches of the batched build. Partials are summed in a
// fixed order, so results are bitwise reproducible.
#include <algorithm>
#include <cmath>
#include <cstdlib>

#include "agf2_internal.h"

namespace agf2 {

namespace {

typedef double d4 __attribute__((ext_vector_type(4)));
constexpr int TB = 64, BK = 16, NT = 256, LD = TB + 1;

// Round-robin dispatch places workgroup w on XCD w % 8; remap so that each
// XCD receives one contiguous range of logical tiles (operand reuse in its L2).
__device__ __forceinline__ long xcd_remap(long w, long G) {
  const long per = G / 8, rem = G % 8;
  const long xcd = w % 8, slot = w / 8;
  return xcd < rem ? xcd * (per + 1) + slot : rem * (per + 1) + (xcd - rem) * per + slot;
}

// One slab tile: 64 x rows x TC inner columns of pair logical / per_pair.
// Wave w owns rows 16w..16w+15 and all TC/16 column blocks.
template <int TC>
__device__ void slab_tile(const SlabF64& a, long logical, double (*A1)[BK][LD],
                          double (*A2)[BK][LD], double (*B1)[BK][LD], double (*B2)[BK][LD]) {
  constexpr int CB = TC / 16;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int per_pair = a.tiles_x * a.tiles_c;
  const int P = a.pair0 + (int)(logical / per_pair);
  const int rem = (int)(logical % per_pair);
  const int xt = rem % a.tiles_x, ct = rem / a.tiles_x;
  const int p = a.pi[P], q = a.pj[P];
  const bool diag = (p == q);
  const int x0 = xt * TB, c0 = ct * TC;
  const double* Rp = a.R + (long)p * a.sRp;
  const double* Rq = a.R + (long)q * a.sRp;
  const double* Sq = a.S + (long)q * a.sSp;
  const double* Sp = a.S + (long)p * a.sSp;

  // loader: thread -> k = tid % 16, rows tid/16 + 16 i. Rows past N and
  // columns past nc read the last row / column instead (their outputs are
  // not stored), so the loads carry no condition and run ahead of the MFMAs.
  const int lk = tid & 15, lr = tid >> 4;
  long orow[4], ocol[CB];
#pragma unroll
  for (int i = 0; i < 4; ++i) orow[i] = (long)min(x0 + lr + 16 * i, a.N - 1) * a.sRx + lk;
#pragma unroll
  for (int i = 0; i < CB; ++i) ocol[i] = (long)min(c0 + lr + 16 * i, a.nc - 1) * a.sSc + lk;
  double r1[4], r2[4], s1[CB], s2[CB];
  auto load = [&](int kb) {
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      r1[i] = Rp[orow[i] + kb];
      r2[i] = Rq[orow[i] + kb];
    }
#pragma unroll
    for (int i = 0; i < CB; ++i) {
      s1[i] = Sq[ocol[i] + kb];
      s2[i] = Sp[ocol[i] + kb];
    }
  };
  auto store = [&](int buf) {
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      A1[buf][lk][lr + 16 * i] = r1[i];
      A2[buf][lk][lr + 16 * i] = r2[i];
    }
#pragma unroll
    for (int i = 0; i < CB; ++i) {
      B1[buf][lk][lr + 16 * i] = s1[i];
      B2[buf][lk][lr + 16 * i] = s2[i];
    }
  };

  const int fr = lane & 15, fk = lane >> 4;
  const int wr = 16 * wave;
  d4 c1[CB], c2[CB];
#pragma unroll
  for (int j = 0; j < CB; ++j) {
    c1[j] = d4{0.0, 0.0, 0.0, 0.0};
    c2[j] = d4{0.0, 0.0, 0.0, 0.0};
  }
  const int nsteps = a.Qp / BK;
  __syncthreads();   // the LDS may still be read by the previous item
  load(0);
  store(0);
  __syncthreads();
  // The mirrored product runs for diagonal pairs too (its inputs are then the
  // same rows and its result is not used), so the MFMA loop has no branch.
  for (int step = 0; step < nsteps; ++step) {
    const int buf = step & 1;
    load(min(step + 1, nsteps - 1) * BK);
    __builtin_amdgcn_sched_barrier(0);
#pragma unroll
    for (int kk = 0; kk < BK; kk += 4) {
      const double x1 = A1[buf][kk + fk][wr + fr];
      const double x2 = A2[buf][kk + fk][wr + fr];
#pragma unroll
      for (int j = 0; j < CB; ++j) {
        c1[j] = __builtin_amdgcn_mfma_f64_16x16x4f64(x1, B1[buf][kk + fk][16 * j + fr], c1[j],
                                                     0, 0, 0);
        c2[j] = __builtin_amdgcn_mfma_f64_16x16x4f64(x2, B2[buf][kk + fk][16 * j + fr], c2[j],
                                                     0, 0, 0);
      }
    }
    store(buf ^ 1);
    __syncthreads();
  }

  const long col0 = a.pcol[P] - a.col_base;
  const double cp = 0.70710678118654752440;   // sqrt(1/2)
  const double cm = 1.22474487139158904910;   // sqrt(3/2)
#pragma unroll
  for (int j = 0; j < CB; ++j)
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int x = x0 + wr + fk + 4 * r;
      const int c = c0 + 16 * j + fr;
      if (x >= a.N || c >= a.nc) continue;
      double* z = a.Z + (long)x * a.ldz + col0 + c;
      if (diag) {
        z[0] = c1[j][r];
      } else {
        const double u = c1[j][r], v = c2[j][r];
        z[0] = cp * (u + v);
        z[a.nc] = cm * (u - v);
      }
    }
  if (xt == 0 && tid < TC) {
    const int c = c0 + tid;
    if (c < a.nc) {
      const double wgt = a.ep[p] + a.ep[q] - a.ec[c];
      a.w[col0 + c] = wgt;
      if (!diag) a.w[col0 + a.nc + c] = wgt;
    }
  }
}

template <int TC>
__global__ __launch_bounds__(NT) void slab_f64_kernel(SlabF64 a) {
  __shared__ double A1[2][BK][LD], A2[2][BK][LD], B1[2][BK][LD], B2[2][BK][LD];
  const long G = (long)a.npairs * a.tiles_x * a.tiles_c;
  slab_tile<TC>(a, xcd_remap(blockIdx.x, G), A1, A2, B1, B2);
}

// Wide slab tile for one-job launches: 128 x rows by TC inner columns, eight
// waves arranged WX x (8 / WX), each owning (128 / WX) rows x (TC / (8 / WX))
// columns of both mirrored products, one workgroup per CU (double-buffered
// LDS, 107 KiB at TC = 80). Per K step it moves 2 (128 + TC) operand rows for
// 4 x 128 x TC x 16 flops: 12.3 flops per byte at TC = 80 against 5.3 for the
// 64 x 32 tile, and up to 0.83 MFMAs per LDS read against 0.67. Same epilogue
// as slab_tile.
constexpr int TBW = 128, LDW = TBW + 1, NTW = 512;
template <int TC, int WX>
__global__ __launch_bounds__(NTW) void slab_f64_wide(SlabF64 a) {
  constexpr int WC = 8 / WX;
  constexpr int RB = TBW / WX / 16;   // row blocks per wave
  constexpr int CBW = TC / WC / 16;   // column blocks per wave
  constexpr int LDC = TC + 1;
  constexpr int NA = TBW / 32;        // A rows per thread and array (32 rows per pass)
  constexpr int NBR = (TC + 31) / 32; // B passes (the last may be partial)
  static_assert(RB * WX * 16 == TBW && CBW * WC * 16 == TC, "wave tiling");
  __shared__ double A1[2][BK][LDW], A2[2][BK][LDW], B1[2][BK][LDC], B2[2][BK][LDC];
  const long G = (long)a.npairs * a.tiles_x * a.tiles_c;
  const long logical = xcd_remap(blockIdx.x, G);
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int per_pair = a.tiles_x * a.tiles_c;
  const int P = a.pair0 + (int)(logical / per_pair);
  const int rem = (int)(logical % per_pair);
  const int xt = rem % a.tiles_x, ct = rem / a.tiles_x;
  const int p = a.pi[P], q = a.pj[P];
  const bool diag = (p == q);
  const int x0 = xt * TBW, c0 = ct * TC;
  const double* Rp = a.R + (long)p * a.sRp;
  const double* Rq = a.R + (long)q * a.sRp;
  const double* Sq = a.S + (long)q * a.sSp;
  const double* Sp = a.S + (long)p * a.sSp;

  // loader: thread -> k = tid % 16, rows tid / 16 + 32 i. Rows past N and
  // columns past nc read the last row / column (their outputs are not
  // stored); B rows past TC in the last pass (a whole wave's rows) are skipped.
  const int lk = tid & 15, lr = tid >> 4;
  long orow[NA], ocol[NBR];
#pragma unroll
  for (int i = 0; i < NA; ++i) orow[i] = (long)min(x0 + lr + 32 * i, a.N - 1) * a.sRx + lk;
#pragma unroll
  for (int i = 0; i < NBR; ++i) ocol[i] = (long)min(c0 + lr + 32 * i, a.nc - 1) * a.sSc + lk;
  double r1[NA], r2[NA], s1[NBR], s2[NBR];
  auto load = [&](int kb) {
#pragma unroll
    for (int i = 0; i < NA; ++i) {
      r1[i] = Rp[orow[i] + kb];
      r2[i] = Rq[orow[i] + kb];
    }
#pragma unroll
    for (int i = 0; i < NBR; ++i) {
      if (lr + 32 * i < TC) {
        s1[i] = Sq[ocol[i] + kb];
        s2[i] = Sp[ocol[i] + kb];
      }
    }
  };
  auto store = [&](int buf) {
#pragma unroll
    for (int i = 0; i < NA; ++i) {
      A1[buf][lk][lr + 32 * i] = r1[i];
      A2[buf][lk][lr + 32 * i] = r2[i];
    }
#pragma unroll
    for (int i = 0; i < NBR; ++i) {
      if (lr + 32 * i < TC) {
        B1[buf][lk][lr + 32 * i] = s1[i];
        B2[buf][lk][lr + 32 * i] = s2[i];
      }
    }
  };

  const int fr = lane & 15, fk = lane >> 4;
  const int wr = (wave % WX) * (TBW / WX), wcol = (wave / WX) * (TC / WC);
  d4 c1[RB][CBW], c2[RB][CBW];
#pragma unroll
  for (int i = 0; i < RB; ++i)
#pragma unroll
    for (int j = 0; j < CBW; ++j) {
      c1[i][j] = d4{0.0, 0.0, 0.0, 0.0};
      c2[i][j] = d4{0.0, 0.0, 0.0, 0.0};
    }
  const int nsteps = a.Qp / BK;
  load(0);
  store(0);
  __syncthreads();
  // The mirrored product runs for diagonal pairs too (its result is unused),
  // so the MFMA loop has no branch.
  for (int step = 0; step < nsteps; ++step) {
    const int buf = step & 1;
    load(min(step + 1, nsteps - 1) * BK);
    __builtin_amdgcn_sched_barrier(0);
#pragma unroll
    for (int kk = 0; kk < BK; kk += 4) {
      double xa1[RB], xa2[RB];
#pragma unroll
      for (int i = 0; i < RB; ++i) {
        xa1[i] = A1[buf][kk + fk][wr + 16 * i + fr];
        xa2[i] = A2[buf][kk + fk][wr + 16 * i + fr];
      }
#pragma unroll
      for (int j = 0; j < CBW; ++j) {
        const double b1 = B1[buf][kk + fk][wcol + 16 * j + fr];
        const double b2 = B2[buf][kk + fk][wcol + 16 * j + fr];
#pragma unroll
        for (int i = 0; i < RB; ++i) {
          c1[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(xa1[i], b1, c1[i][j], 0, 0, 0);
          c2[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(xa2[i], b2, c2[i][j], 0, 0, 0);
        }
      }
    }
    store(buf ^ 1);
    __syncthreads();
  }

  const long col0 = a.pcol[P] - a.col_base;
  const double cp = 0.70710678118654752440;   // sqrt(1/2)
  const double cm = 1.22474487139158904910;   // sqrt(3/2)
#pragma unroll
  for (int i = 0; i < RB; ++i)
#pragma unroll
    for (int j = 0; j < CBW; ++j)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int x = x0 + wr + 16 * i + fk + 4 * r;
        const int c = c0 + wcol + 16 * j + fr;
        if (x >= a.N || c >= a.nc) continue;
        double* z = a.Z + (long)x * a.ldz + col0 + c;
        if (diag) {
          z[0] = c1[i][j][r];
        } else {
          const double u = c1[i][j][r], v = c2[i][j][r];
          z[0] = cp * (u + v);
          z[a.nc] = cm * (u - v);
        }
      }
  if (xt == 0 && tid < TC) {
    const int c = c0 + tid;
    if (c < a.nc) {
      const double wgt = a.ep[p] + a.ep[q] - a.ec[c];
      a.w[col0 + c] = wgt;
      if (!diag) a.w[col0 + a.nc + c] = wgt;
    }
  }
}

// Job owning global work index `it`: the largest j with prefix[j] <= it
// (jobs with no work share their prefix with the next job and are skipped).
__device__ __forceinline__ int find_job(const long* prefix, int njobs, long it) {
  int lo = 0, hi = njobs - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (prefix[mid] <= it) lo = mid; else hi = mid - 1;
  }
  return lo;
}

template <int TC>
__global__ __launch_bounds__(NT) void slab_f64_grouped(const SlabF64* jobs, const long* prefix,
                                                       int njobs, long total) {
  __shared__ double A1[2][BK][LD], A2[2][BK][LD], B1[2][BK][LD], B2[2][BK][LD];
  for (long it = blockIdx.x; it < total; it += gridDim.x) {
    const int j = find_job(prefix, njobs, it);
    slab_tile<TC>(jobs[j], it - prefix[j], A1, A2, B1, B2);
  }
}

// One SYRK tile: lower-triangle tile t, K split s.
// UNCOND: the loads of a K step carry no condition and run ahead of the
// MFMAs (the grouped kernel, whose items each span few K steps, gains from
// it); otherwise the loads are predicated and the last step skips the
// prefetch (faster for the one-item-per-workgroup kernel, measured).
template <bool UNCOND>
__device__ void syrk_tile(const SyrkF64& a, int t, int s, double (*X)[BK][LD],
                          double (*Y)[BK][LD], double (*W)[BK]) {
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  int xt = (int)((sqrt(8.0 * t + 1.0) - 1.0) * 0.5);
  while ((xt + 1) * (xt + 2) / 2 <= t) ++xt;
  while (xt * (xt + 1) / 2 > t) --xt;
  const int yt = t - xt * (xt + 1) / 2;
  const long k0 = (long)s * a.kper, k1 = std::min(a.K, k0 + a.kper);
  const int x0 = xt * TB, y0 = yt * TB;
  // loader: thread -> k = tid % 16, rows tid/16 + 16 i. Rows past N read row
  // N - 1 (their outputs are not stored); a column past the split's end is
  // read at the split's last column and replaced by zero, so the loads carry
  // no condition and run ahead of the MFMAs.
  const int lk = tid & 15, lr = tid >> 4;
  long ox[4], oy[4];
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    ox[i] = (long)min(x0 + lr + 16 * i, a.N - 1) * a.ldz;
    oy[i] = (long)min(y0 + lr + 16 * i, a.N - 1) * a.ldz;
  }
  double rx[4], ry[4], rw = 0.0;
  auto load = [&](long kb) {
    const long k = kb + lk;
    const bool kin = k < k1;
    if constexpr (UNCOND) {
      const long kc = kin ? k : k1 - 1;
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const double vx = a.Z[ox[i] + kc], vy = a.Z[oy[i] + kc];
        rx[i] = kin ? vx : 0.0;
        ry[i] = kin ? vy : 0.0;
      }
      const double vw = a.w[kc];
      rw = kin ? vw : 0.0;
    } else {
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        rx[i] = kin ? a.Z[ox[i] + k] : 0.0;
        ry[i] = kin ? a.Z[oy[i] + k] : 0.0;
      }
      if (tid < BK) rw = kin ? a.w[k] : 0.0;
    }
  };
  auto store = [&](int buf) {
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      X[buf][lk][lr + 16 * i] = rx[i];
      Y[buf][lk][lr + 16 * i] = ry[i];
    }
    if (tid < BK) W[buf][tid] = rw;
  };
  const int wm = (wave & 1) * 32, wn = (wave >> 1) * 32;
  const int fr = lane & 15, fk = lane >> 4;
  d4 u0[2][2], u1[2][2];
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j) {
      u0[i][j] = d4{0.0, 0.0, 0.0, 0.0};
      u1[i][j] = d4{0.0, 0.0, 0.0, 0.0};
    }
  const long nsteps = (k1 > k0) ? (k1 - k0 + BK - 1) / BK : 0;
  if (nsteps == 0) return;   // uniform over the workgroup
  __syncthreads();           // the LDS may still be read by the previous item
  load(k0);
  store(0);
  __syncthreads();
  for (long step = 0; step < nsteps; ++step) {
    const int buf = step & 1;
    if constexpr (UNCOND) {
      load(k0 + min(step + 1, nsteps - 1) * BK);
      __builtin_amdgcn_sched_barrier(0);
    } else if (step + 1 < nsteps) {
      load(k0 + (step + 1) * BK);
    }
#pragma unroll
    for (int kk = 0; kk < BK; kk += 4) {
      const double wk = W[buf][kk + fk];
      double xa[2], xw[2], yb[2];
#pragma unroll
      for (int i = 0; i < 2; ++i) {
        xa[i] = X[buf][kk + fk][wm + 16 * i + fr];
        xw[i] = xa[i] * wk;
      }
#pragma unroll
      for (int j = 0; j < 2; ++j) yb[j] = Y[buf][kk + fk][wn + 16 * j + fr];
#pragma unroll
      for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j) {
          u0[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(xa[i], yb[j], u0[i][j], 0, 0, 0);
          u1[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(xw[i], yb[j], u1[i][j], 0, 0, 0);
        }
    }
    // (UNCOND: the last step writes the idle buffer)
    if (UNCOND || step + 1 < nsteps) store(buf ^ 1);
    __syncthreads();
  }
  double* P0 = a.part + (long)s * a.part_stride;
  double* P1 = P0 + (long)a.N * a.N;
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int x = x0 + wm + 16 * i + fk + 4 * r;
        const int y = y0 + wn + 16 * j + fr;
        if (x >= a.N || y >= a.N) continue;
        const long o = (long)x * a.N + y;
        P0[o] += u0[i][j][r];
        P1[o] += u1[i][j][r];
      }
}

__global__ __launch_bounds__(NT) void syrk_f64_kernel(SyrkF64 a) {
  __shared__ double X[2][BK][LD], Y[2][BK][LD], W[2][BK];
  // split-major items dealt to XCDs in contiguous ranges (one K range per L2)
  const long item = xcd_remap(blockIdx.x, (long)a.tiles * a.nsplit);
  syrk_tile<false>(a, (int)(item % a.tiles), (int)(item / a.tiles), X, Y, W);
}

// Wide SYRK tile for one-job launches: lower-triangle 128 x 128 tiles (tile
// t of the 128-row triangle), eight waves of 32 x rows by 64 y rows with both
// moments, one workgroup per CU. A K step moves 256 operand rows for
// 2 x 2 x 128 x 128 x 16 flops (32 flops per byte, against 16 for the 64-row
// tile) and 2.3 MFMAs per LDS read. Waves whose sub-tile lies wholly above
// the diagonal skip their MFMAs and stores; only the lower triangle of the
// partial slots is read by the reduction. Loads carry no condition (rows past
// N read row N - 1, columns past the split's end read its last column and
// are replaced by zero).
constexpr int NTS = 512;
__global__ __launch_bounds__(NTS) void syrk_f64_wide(SyrkF64 a) {
  __shared__ double X[2][BK][LDW], Y[2][BK][LDW], W[2][BK];
  const long item = xcd_remap(blockIdx.x, (long)a.tiles * a.nsplit);
  const int t = (int)(item % a.tiles), s = (int)(item / a.tiles);
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  int xt = (int)((sqrt(8.0 * t + 1.0) - 1.0) * 0.5);
  while ((xt + 1) * (xt + 2) / 2 <= t) ++xt;
  while (xt * (xt + 1) / 2 > t) --xt;
  const int yt = t - xt * (xt + 1) / 2;
  const long k0 = (long)s * a.kper, k1 = std::min(a.K, k0 + a.kper);
  if (k1 <= k0) return;   // uniform over the workgroup
  const int x0 = xt * TBW, y0 = yt * TBW;
  const int lk = tid & 15, lr = tid >> 4;   // 32 rows per pass, 4 passes
  long ox[4], oy[4];
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    ox[i] = (long)min(x0 + lr + 32 * i, a.N - 1) * a.ldz;
    oy[i] = (long)min(y0 + lr + 32 * i, a.N - 1) * a.ldz;
  }
  double rx[4], ry[4], rw = 0.0;
  auto load = [&](long kb) {
    const long k = kb + lk;
    const bool kin = k < k1;
    const long kc = kin ? k : k1 - 1;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const double vx = a.Z[ox[i] + kc], vy = a.Z[oy[i] + kc];
      rx[i] = kin ? vx : 0.0;
      ry[i] = kin ? vy : 0.0;
    }
    const double vw = a.w[kc];
    rw = kin ? vw : 0.0;
  };
  auto store = [&](int buf) {
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      X[buf][lk][lr + 32 * i] = rx[i];
      Y[buf][lk][lr + 32 * i] = ry[i];
    }
    if (tid < BK) W[buf][tid] = rw;
  };
  const int wm = (wave & 3) * 32, wn = (wave >> 2) * 64;
  const bool active = x0 + wm + 31 >= y0 + wn;   // some element on or below the diagonal
  const int fr = lane & 15, fk = lane >> 4;
  d4 u0[2][4], u1[2][4];
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      u0[i][j] = d4{0.0, 0.0, 0.0, 0.0};
      u1[i][j] = d4{0.0, 0.0, 0.0, 0.0};
    }
  const long nsteps = (k1 - k0 + BK - 1) / BK;
  load(k0);
  store(0);
  __syncthreads();
  for (long step = 0; step < nsteps; ++step) {
    const int buf = step & 1;
    load(k0 + min(step + 1, nsteps - 1) * BK);
    __builtin_amdgcn_sched_barrier(0);
    if (active) {
#pragma unroll
      for (int kk = 0; kk < BK; kk += 4) {
        const double wk = W[buf][kk + fk];
        double xa[2], xw[2], yb[4];
#pragma unroll
        for (int i = 0; i < 2; ++i) {
          xa[i] = X[buf][kk + fk][wm + 16 * i + fr];
          xw[i] = xa[i] * wk;
        }
#pragma unroll
        for (int j = 0; j < 4; ++j) yb[j] = Y[buf][kk + fk][wn + 16 * j + fr];
#pragma unroll
        for (int i = 0; i < 2; ++i)
#pragma unroll
          for (int j = 0; j < 4; ++j) {
            u0[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(xa[i], yb[j], u0[i][j], 0, 0, 0);
            u1[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(xw[i], yb[j], u1[i][j], 0, 0, 0);
          }
      }
    }
    store(buf ^ 1);   // the last step writes the idle buffer
    __syncthreads();
  }
  if (!active) return;
  double* P0 = a.part + (long)s * a.part_stride;
  double* P1 = P0 + (long)a.N * a.N;
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int x = x0 + wm + 16 * i + fk + 4 * r;
        const int y = y0 + wn + 16 * j + fr;
        if (x >= a.N || y > x) continue;
        const long o = (long)x * a.N + y;
        P0[o] += u0[i][j][r];
        P1[o] += u1[i][j][r];
      }
}

__global__ __launch_bounds__(NT) void syrk_f64_grouped(const SyrkF64* jobs, const long* prefix,
                                                       int njobs, long total) {
  __shared__ double X[2][BK][LD], Y[2][BK][LD], W[2][BK];
  for (long it = blockIdx.x; it < total; it += gridDim.x) {
    const int j = find_job(prefix, njobs, it);
    const SyrkF64& a = jobs[j];
    const long l = it - prefix[j];
    syrk_tile<true>(a, (int)(l % a.tiles), (int)(l / a.tiles), X, Y, W);
  }
}

// U[x][y] = U[y][x] = sum_s part[s][m][x][y] for x >= y (fixed order).
__global__ void reduce_sym_kernel(const double* part, long part_stride, int nsplit,
                                  int N, double* U0, double* U1) {
  const long n = (long)N * N;
  for (long idx = blockIdx.x * (long)blockDim.x + threadIdx.x; idx < n;
       idx += (long)gridDim.x * blockDim.x) {
    const int x = (int)(idx / N), y = (int)(idx % N);
    if (x < y) continue;
    double s0 = 0.0, s1 = 0.0;
    for (int s = 0; s < nsplit; ++s) {
      s0 += part[s * part_stride + idx];
      s1 += part[s * part_stride + n + idx];
    }
    U0[(long)x * N + y] = s0; U0[(long)y * N + x] = s0;
    U1[(long)x * N + y] = s1; U1[(long)y * N + x] = s1;
  }
}

__global__ void fill_zero_kernel(double* p, long n) {
  for (long i = blockIdx.x * (long)blockDim.x + threadIdx.x; i < n;
       i += (long)gridDim.x * blockDim.x)
    p[i] = 0.0;
}

inline long nblocks(long n) { return std::max<long>(1, std::min<long>((n + 255) / 256, 4096)); }

}  // namespace

// Inner tile width for nc inner poles: the width whose padded tiles cost least,
// a tile of width TC counted as TC + 16 columns (its fixed per-tile work,
// mainly the 64 x-rows of both R operands); ties go to the wider tile.
int slab_f64_tc(int nc) {
  int best = 64;
  long best_cost = -1;
  for (int tc : {64, 32, 16}) {
    const long cost = (long)((nc + tc - 1) / tc) * (tc + 16);
    if (best_cost < 0 || cost < best_cost) {
      best = tc;
      best_cost = cost;
    }
  }
  return best;
}

long slab_f64_tiles(const SlabF64& a) { return (long)a.npairs * a.tiles_x * a.tiles_c; }

void launch_slab_f64(int tc, const SlabF64& a, hipStream_t st) {
  const dim3 grid((unsigned)slab_f64_tiles(a));
  if (tc == 16) hipLaunchKernelGGL(slab_f64_kernel<16>, grid, dim3(NT), 0, st, a);
  else if (tc == 32) hipLaunchKernelGGL(slab_f64_kernel<32>, grid, dim3(NT), 0, st, a);
  else hipLaunchKernelGGL(slab_f64_kernel<64>, grid, dim3(NT), 0, st, a);
  AGF2_CHECK_LAUNCH();
}

// One-job launches use the 128-row tile when the x range pads to at most 15%
// more rows than with 64-row tiles; its inner width is the cheapest of 80, 64
// and 32 in padded columns plus a fixed 16 per tile.
bool slab_f64_use_wide(int N) {
  return (long)((N + TBW - 1) / TBW) * TBW * 100 <= (long)((N + TB - 1) / TB) * TB * 115;
}

int slab_f64_wide_tc(int nc) {
  int best = 80;
  long best_cost = -1;
  for (int tc : {80, 64, 32}) {
    const long cost = (long)((nc + tc - 1) / tc) * (tc + 16);
    if (best_cost < 0 || cost < best_cost) {
      best = tc;
      best_cost = cost;
    }
  }
  return best;
}

void launch_slab_f64_wide(int tc, const SlabF64& a, hipStream_t st) {
  const dim3 grid((unsigned)slab_f64_tiles(a));
  if (tc == 80) hipLaunchKernelGGL((slab_f64_wide<80, 8>), grid, dim3(NTW), 0, st, a);
  else if (tc == 64) hipLaunchKernelGGL((slab_f64_wide<64, 4>), grid, dim3(NTW), 0, st, a);
  else hipLaunchKernelGGL((slab_f64_wide<32, 8>), grid, dim3(NTW), 0, st, a);
  AGF2_CHECK_LAUNCH();
}

void launch_syrk_f64_wide(const SyrkF64& a, hipStream_t st) {
  hipLaunchKernelGGL(syrk_f64_wide, dim3((unsigned)((long)a.tiles * a.nsplit)), dim3(NTS), 0,
                     st, a);
  AGF2_CHECK_LAUNCH();
}

void launch_syrk_f64(const SyrkF64& a, hipStream_t st) {
  hipLaunchKernelGGL(syrk_f64_kernel, dim3((unsigned)((long)a.tiles * a.nsplit)), dim3(NT), 0,
                     st, a);
  AGF2_CHECK_LAUNCH();
}

void launch_slab_f64_grouped(int tc, const SlabF64* jobs, const long* prefix, int njobs,
                             long total, int grid, hipStream_t st) {
  if (total <= 0 || njobs <= 0) return;
  const dim3 g((unsigned)std::max<long>(1, std::min<long>(grid, total)));
  if (tc == 16) hipLaunchKernelGGL(slab_f64_grouped<16>, g, dim3(NT), 0, st, jobs, prefix, njobs, total);
  else if (tc == 32) hipLaunchKernelGGL(slab_f64_grouped<32>, g, dim3(NT), 0, st, jobs, prefix, njobs, total);
  else hipLaunchKernelGGL(slab_f64_grouped<64>, g, dim3(NT), 0, st, jobs, prefix, njobs, total);
  AGF2_CHECK_LAUNCH();
}

void launch_syrk_f64_grouped(const SyrkF64* jobs, const long* prefix, int njobs, long total,
                             int grid, hipStream_t st) {
  if (total <= 0 || njobs <= 0) return;
  const dim3 g((unsigned)std::max<long>(1, std::min<long>(grid, total)));
  hipLaunchKernelGGL(syrk_f64_grouped, g, dim3(NT), 0, st, jobs, prefix, njobs, total);
  AGF2_CHECK_LAUNCH();
}

int grouped_grid_f64(int kind, int tc) {
  static int cached[4] = {0, 0, 0, 0};   // slab 16/32/64, syrk (one device type per process)
  const int slot = kind == 1 ? 3 : (tc == 16 ? 0 : tc == 32 ? 1 : 2);
  if (cached[slot] > 0) return cached[slot];
  int dev = 0, cus = 0, per = 0;
  AGF2_HIP(hipGetDevice(&dev));
  AGF2_HIP(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
  if (slot == 0) AGF2_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, slab_f64_grouped<16>, NT, 0));
  else if (slot == 1) AGF2_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, slab_f64_grouped<32>, NT, 0));
  else if (slot == 2) AGF2_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, slab_f64_grouped<64>, NT, 0));
  else AGF2_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, syrk_f64_grouped, NT, 0));
  cached[slot] = std::max(1, cus) * std::max(1, per);
  return cached[slot];
}

void fill_zero(double* p, long n, hipStream_t st) {
  if (n <= 0) return;
  hipLaunchKernelGGL(fill_zero_kernel, dim3(nblocks(n)), dim3(256), 0, st, p, n);
  AGF2_CHECK_LAUNCH();
}

void reduce_moment_partials(const double* part, long part_stride, int nsplit, int N,
                            double* U0, double* U1, hipStream_t st) {
  const long nn = (long)N * N;
  hipLaunchKernelGGL(reduce_sym_kernel, dim3(nblocks(nn)), dim3(256), 0, st, part, part_stride,
                     nsplit, N, U0, U1);
  AGF2_CHECK_LAUNCH();
}

namespace {

struct PairTable {
  std::vector<int> pi, pj;
  std::vector<long> col;   // column offset of each pair (prefix sum of widths)
};

PairTable make_pairs(int np, int nc) {
  PairTable t;
  long c = 0;
  for (int p = 0; p < np; ++p)
    for (int q = p; q < np; ++q) {
      t.pi.push_back(p); t.pj.push_back(q); t.col.push_back(c);
      c += (p == q) ? nc : 2L * nc;
    }
  t.col.push_back(c);
  return t;
}

long ndiag(const PairTable& t, int P0, int P1) {
  long n = 0;
  for (int P = P0; P < P1; ++P) n += (t.pi[P] == t.pj[P]);
  return n;
}

}  // namespace

namespace {

// Z[x][c] *= w[c] for the chunk's Kc columns (row stride ldz)
__global__ void scale_cols_kernel(int N, long Kc, long ldz, const double* w, double* Z) {
  const long tot = (long)N * Kc;
  for (long i = blockIdx.x * (long)blockDim.x + threadIdx.x; i < tot;
       i += (long)gridDim.x * blockDim.x) {
    const long x = i / Kc, c = i % Kc;
    Z[x * ldz + c] *= w[c];
  }
}

}  // namespace

// One part (lesser or greater) of the moment build: moments 0 .. 2 npm - 1
// into U[0 .. 2 npm - 1]. Each Z chunk feeds one SYRK per moment pair: pair m
// (moments 2m and 2m + 1) is the SYRK of Z diag(w)^m, whose columns are
// scaled by w in place before each further pair.
static void moments_part_f64(Handle& h, int N, int Q, int Qp, const double* R, long sRp,
                             long sRx, const double* S, long sSp, long sSc,
                             const double* ep, int np, const double* ec, int nc, int npm,
                             double* const* U) {
  hipStream_t st = h.stream;
  const long nn = (long)N * N;
  if (np == 0 || nc == 0) {
    for (int k = 0; k < 2 * npm; ++k) fill_zero(U[k], nn, st);
    return;
  }
  PairTable t = make_pairs(np, nc);
  const int npairs = (int)t.pi.size();
  int* d_pi = h.ws_moments[6].as<int>(2L * npairs);
  int* d_pj = d_pi + npairs;
  long* d_col = h.ws_moments[7].as<long>(npairs + 1);
  AGF2_HIP(hipMemcpyAsync(d_pi, t.pi.data(), npairs * sizeof(int), hipMemcpyHostToDevice, st));
  AGF2_HIP(hipMemcpyAsync(d_pj, t.pj.data(), npairs * sizeof(int), hipMemcpyHostToDevice, st));
  AGF2_HIP(hipMemcpyAsync(d_col, t.col.data(), (npairs + 1) * sizeof(long),
                          hipMemcpyHostToDevice, st));
  AGF2_HIP(hipStreamSynchronize(st));   // host tables go out of scope below

  // Z chunk capacity: whole pairs, at most ~1 GiB of Z
  const long cap_bytes = 1L << 30;
  long kcap = std::max<long>(2L * nc, cap_bytes / (8L * N));
  kcap = std::min<long>(kcap, t.col.back());
  kcap = (kcap + BK - 1) / BK * BK;
  double* Z = h.ws_moments[4].as<double>((long)N * kcap + kcap);
  double* w = Z + (long)N * kcap;

  const int tiles_n = (N + TB - 1) / TB;
  const bool wide = slab_f64_use_wide(N);   // 128-row slab and SYRK tiles
  const int tiles_w = (N + TBW - 1) / TBW;
  const int nlower = wide ? tiles_w * (tiles_w + 1) / 2 : tiles_n * (tiles_n + 1) / 2;
  const int nsplit_max = std::max(1, std::min(64, (2048 + nlower - 1) / nlower));
  const long part_stride = 2 * nn;
  const long pair_stride = part_stride * nsplit_max;
  double* part = h.ws_moments[5].as<double>(pair_stride * npm);
  fill_zero(part, pair_stride * npm, st);

  const int tc = wide ? slab_f64_wide_tc(nc) : slab_f64_tc(nc);
  int P0 = 0;
  while (P0 < npairs) {
    int P1 = P0;
    while (P1 < npairs && t.col[P1 + 1] - t.col[P0] <= kcap) ++P1;
    if (P1 == P0) P1 = P0 + 1;
    const long Kc = t.col[P1] - t.col[P0];

    SlabF64 sa;
    sa.R = R; sa.sRp = sRp; sa.sRx = sRx;
    sa.S = S; sa.sSp = sSp; sa.sSc = sSc;
    sa.ep = ep; sa.ec = ec; sa.N = N; sa.nc = nc; sa.Qp = Qp;
    sa.pi = d_pi; sa.pj = d_pj; sa.pcol = d_col;
    sa.pair0 = P0; sa.npairs = P1 - P0; sa.col_base = t.col[P0];
    sa.Z = Z; sa.ldz = kcap; sa.w = w;
    sa.tiles_x = wide ? (N + TBW - 1) / TBW : tiles_n; sa.tiles_c = (nc + tc - 1) / tc;
    {
      // algorithmic: 2 N nc Q per (p,q) slab, two slabs per off-diagonal pair;
      // bytes: the Z chunk and its weights written once
      const double slabs = (double)(2 * (P1 - P0)) - (double)ndiag(t, P0, P1);
      ProfScope ps(h, "moments.slab", slabs * 2.0 * N * nc * Q, 8.0 * (N + 1.0) * Kc);
      if (wide) launch_slab_f64_wide(tc, sa, st);
      else launch_slab_f64(tc, sa, st);
    }

    int nsplit = (int)std::min<long>(nsplit_max, std::max<long>(1, Kc / 256));
    long kper = (Kc + nsplit - 1) / nsplit;
    kper = (kper + BK - 1) / BK * BK;
    nsplit = (int)((Kc + kper - 1) / kper);
    SyrkF64 ya;
    ya.Z = Z; ya.ldz = kcap; ya.w = w; ya.N = N; ya.K = Kc; ya.kper = kper; ya.nsplit = nsplit;
    ya.part = part; ya.part_stride = part_stride; ya.tiles = nlower;
    for (int m = 0; m < npm; ++m) {
      if (m > 0) {
        hipLaunchKernelGGL(scale_cols_kernel, dim3(nblocks((long)N * Kc)), dim3(256), 0, st, N,
                           Kc, kcap, w, Z);
        AGF2_CHECK_LAUNCH();
      }
      ya.part = part + m * pair_stride;
      // algorithmic: lower triangles of two symmetric N x N products over Kc
      ProfScope ps(h, "moments.syrk", 2.0 * N * (N + 1.0) * Kc, 8.0 * (N + 1.0) * Kc);
      if (wide) launch_syrk_f64_wide(ya, st);
      else launch_syrk_f64(ya, st);
    }
    P0 = P1;
  }
  ProfScope ps(h, "moments.reduce", 0.0, 8.0 * (2.0 * nsplit_max + 2.0) * nn * npm);
  for (int m = 0; m < npm; ++m)
    reduce_moment_partials(part + m * pair_stride, part_stride, nsplit_max, N, U[2 * m],
                           U[2 * m + 1], st);
}

namespace {

// flag = 1 unless u (n x n) is exactly the identity
__global__ void identity_check_kernel(const double* u, int n, int* flag) {
  const long nn = (long)n * n;
  for (long k = blockIdx.x * (long)blockDim.x + threadIdx.x; k < nn;
       k += (long)gridDim.x * blockDim.x) {
    const long r = k / n, c = k - r * n;
    if (u[k] != (r == c ? 1.0 : 0.0)) *flag = 1;
  }
}

// T[p][x][q] = L[q][x][p0 + p] (zero for q >= Q) through 32 x 32 LDS tiles of
// (q, p) per row x: 256-byte runs of p read, 256-byte runs of q written.
// Adding +0.0 turns a -0.0 into the +0.0 that the product with the identity
// gives, so the copy equals that product bit for bit.
__global__ __launch_bounds__(256) void transpose_poles_kernel(const double* L, int N, int Q,
                                                              int Qp, int p0, int np,
                                                              int qtiles, double* T) {
  __shared__ double tile[32][33];
  const int x = (int)(blockIdx.x / qtiles);
  const int q0 = (int)(blockIdx.x % qtiles) * 32;
  const int pb = (int)blockIdx.y * 32;
  const int tx = (int)(threadIdx.x % 32), ty = (int)(threadIdx.x / 32);
  const long nn = (long)N * N;
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    const int q = q0 + ty + 8 * r, p = pb + tx;
    tile[ty + 8 * r][tx] =
        (q < Q && p < np) ? L[(long)q * nn + (long)x * N + p0 + p] + 0.0 : 0.0;
  }
  __syncthreads();
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    const int p = pb + ty + 8 * r, q = q0 + tx;
    if (p < np && q < Qp) T[((long)p * N + x) * Qp + q] = tile[tx][ty + 8 * r];
  }
}

// out[i][a][q] = in[a][i][q] for i < o, a < na, q < Qp
__global__ void select_rows_kernel(const double* in, int N, int o, int na, int Qp,
                                   double* out) {
  const long tot = (long)o * na * Qp;
  for (long k = blockIdx.x * (long)blockDim.x + threadIdx.x; k < tot;
       k += (long)gridDim.x * blockDim.x) {
    const long r = k / Qp;
    const int q = (int)(k - r * Qp);
    const int a = (int)(r % na), i = (int)(r / na);
    out[k] = in[((long)a * N + i) * Qp + q];
  }
}

}  // namespace

// Mean-field poles (the first iteration from the mean-field reference: one
// pole per orbital with unit coefficients) make the pole-basis transform a
// relayout of L. True when npole = N and u is exactly the identity (checked
// on the device; one host synchronisation). AGF2_NO_IDENTITY_TRANSFORM=1 in
// the environment turns the check off, so every transform runs as a product
// with u (a check that both give the same bits).
bool poles_are_identity(Handle& h, int N, int npole, const double* u) {
  if (npole != N || N == 0) return false;
  const char* env = std::getenv("AGF2_NO_IDENTITY_TRANSFORM");
  if (env && env[0] == '1') return false;
  int* flag = reinterpret_cast<int*>(h.ws_red.as<double>(4096) + 4004);
  AGF2_HIP(hipMemsetAsync(flag, 0, sizeof(int), h.stream));
  const long nn = (long)N * N;
  const unsigned blocks = (unsigned)std::min<long>((nn + 255) / 256, 4096);
  hipLaunchKernelGGL(identity_check_kernel, dim3(blocks), dim3(256), 0, h.stream, u, N, flag);
  AGF2_CHECK_LAUNCH();
  int hf = 1;
  AGF2_HIP(hipMemcpyAsync(&hf, flag, sizeof(int), hipMemcpyDeviceToHost, h.stream));
  AGF2_HIP(hipStreamSynchronize(h.stream));
  return hf == 0;
}

// Pole-basis DF tensors, Q padded to Qp (a multiple of 16) with zeros:
//   T[p][x][Q] = sum_r u[r][p0+p] L[Q][x][r]          (p in [0, np))
// u = nullptr: identity coefficients, T[p][x][Q] = L[Q][x][p0+p].
void pole_transform_f64(int N, int Q, int Qp, const double* L, const double* u, int npole,
                        int p0, int np, double* T, hipStream_t st) {
  if (np == 0) return;
  if (!u) {
    const long qtiles = (Qp + 31) / 32, ptiles = (np + 31) / 32;
    AGF2_REQUIRE((long)N * qtiles < (1L << 31) && ptiles <= 65535,
                 "pole transform: grid too large");
    hipLaunchKernelGGL(transpose_poles_kernel, dim3((unsigned)(N * qtiles), (unsigned)ptiles),
                       dim3(256), 0, st, L, N, Q, Qp, p0, np, (int)qtiles, T);
    AGF2_CHECK_LAUNCH();
    return;
  }
  Gemm g;
  g.M = np; g.N = Q; g.K = N; g.batch = N;
  g.A = u + p0; g.sAm = 1; g.sAk = npole;              // A(p, r) = u[r][p0+p]
  g.B = L; g.sBb = N; g.sBk = 1; g.sBn = (long)N * N;  // B(r, Q) = L[Q][x][r]
  g.C = T; g.sCb = Qp; g.sCm = (long)N * Qp; g.sCn = 1;
  gemm_f64_padded(g, Qp, st);
}

// Lov[i][a][Q] = sum_x u[x][i] Lxv[a][x][Q]
// u = nullptr: identity coefficients, Lov[i][a][Q] = Lxv[a][i][Q].
void lov_transform_f64(int N, int Q, int Qp, const double* u, int npole, int o, int v,
                       const double* Lxv, double* Lov, hipStream_t st) {
  if (o == 0 || v == 0) return;
  if (!u) {
    const long tot = (long)o * v * Qp;
    hipLaunchKernelGGL(select_rows_kernel,
                       dim3((unsigned)std::min<long>((tot + 255) / 256, 16384)), dim3(256), 0,
                       st, Lxv, N, o, v, Qp, Lov);
    AGF2_CHECK_LAUNCH();
    return;
  }
  Gemm g;
  g.M = o; g.N = Q; g.K = N; g.batch = v;
  g.A = u; g.sAm = 1; g.sAk = npole;
  g.B = Lxv; g.sBb = (long)N * Qp; g.sBk = Qp; g.sBn = 1;
  g.C = Lov; g.sCb = Qp; g.sCm = (long)v * Qp; g.sCn = 1;
  gemm_f64_padded(g, Qp, st);
}

void build_moments_f64_n(Handle& h, int N, int Q, const double* L, int npole, int nocc,
                         const double* e, const double* u, int npm, double* const* Uo,
                         double* const* Uv) {
  const int o = nocc, v = npole - nocc;
  const int Qp = (Q + BK - 1) / BK * BK;
  double* Lxo = h.ws_moments[0].as<double>((long)o * N * Qp);
  double* Lxv = h.ws_moments[1].as<double>((long)v * N * Qp);
  double* Lov = h.ws_moments[2].as<double>((long)o * v * Qp);
  {
    const double* ut = poles_are_identity(h, N, npole, u) ? nullptr : u;
    ProfScope ps(h, "moments.transform",
                 ut ? 2.0 * Q * (double)N * N * npole + 2.0 * Q * (double)N * o * v : 0.0,
                 8.0 * ((double)Q * N * N + (double)npole * N * Q + (double)o * v * Q));
    pole_transform_f64(N, Q, Qp, L, ut, npole, 0, o, Lxo, h.stream);
    pole_transform_f64(N, Q, Qp, L, ut, npole, o, v, Lxv, h.stream);
    lov_transform_f64(N, Q, Qp, ut, npole, o, v, Lxv, Lov, h.stream);
  }
  // lesser: pairs (i, j) occupied, inner a virtual; S[j][a][Q] = Lov[j][a][Q]
  moments_part_f64(h, N, Q, Qp, Lxo, (long)N * Qp, Qp, Lov, (long)v * Qp, Qp,
                   e, o, e + o, v, npm, Uo);
  // greater: pairs (a, b) virtual, inner i occupied; S[b][i][Q] = Lov[i][b][Q]
  moments_part_f64(h, N, Q, Qp, Lxv, (long)N * Qp, Qp, Lov, Qp, (long)v * Qp,
                   e + o, v, e, o, npm, Uv);
}

void build_moments_f64(Handle& h, int N, int Q, const double* L, int npole,
                       int nocc, const double* e, const double* u, double* m0o,
                       double* m1o, double* m0v, double* m1v) {
  double* const Uo[2] = {m0o, m1o};
  double* const Uv[2] = {m0v, m1v};
  build_moments_f64_n(h, N, Q, L, npole, nocc, e, u, 1, Uo, Uv);
}

}  // namespace agf2
