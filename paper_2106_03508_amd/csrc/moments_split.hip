// Split-precision self-energy moment build (same mathematics as the FP64
// build; see moments_f64.hip for the pairing of (p,q) with (q,p)).
//
// Precision scheme (two storage formats, same kernels):
//   - the pole-basis DF tensors are formed in float64, rounded to float32 and
//     stored as 16-bit pairs x ~ hi + lo (hi = r(x), lo = r(x - hi)) where r
//     rounds to bf16 (8 significant bits) or to fp16 (11 significant bits);
//   - fp16 operands are scaled by powers of two first (one exponent per pole
//     row of R, one per row of S, and one for all of Z and of w*Z), chosen
//     from exact maxima or a Cauchy-Schwarz bound so that nothing overflows;
//     the scales are undone exactly in float32/float64;
//   - slab products a*b are evaluated as hi*hi + hi*lo + lo*hi with
//     v_mfma_f32_16x16x32_{bf16,f16} (float32 accumulation over Q);
//   - the slab kernel writes the Z columns and their weighted copies w*Z as
//     16-bit pairs; the SYRK kernel takes all four products of Z (the lo*lo
//     term of a square is never negative, so dropping it would bias U0),
//     accumulates in float32 over chunks of KC columns and folds each chunk
//     into float64 accumulators; per-split float64 partials are summed in a
//     fixed order.
#include <algorithm>
#include <cmath>
#include <cstdlib>
#include <cstring>

#include "agf2_internal.h"

namespace agf2 {

void reduce_moment_partials(const double* part, long part_stride, int nsplit, int N,
                            double* U0, double* U1, hipStream_t st);

namespace {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef _Float16 f16x8 __attribute__((ext_vector_type(8)));
typedef unsigned short u16;
typedef u16 u16x8 __attribute__((ext_vector_type(8)));
typedef float f4 __attribute__((ext_vector_type(4)));

constexpr int KS = 32;        // k depth of one MFMA step
constexpr int KV = KS / 8;    // 16-byte vectors per row per step
// LDS rows hold KV 16-byte vectors with no padding; vector kv of row r sits
// in slot kv ^ ((r >> 1) & 3). Of the layouts timed on gfx950 (plain rows,
// rows padded to five vectors, and several XOR and rotation schemes) this is
// the one whose fragment reads (16 consecutive rows, one vector each) run at
// the speed of contiguous 16-byte reads; its loader stores (4 whole rows per
// 16 lanes) do too. The padded rows and the other schemes take ~1.55x longer
// per fragment read.
__device__ __forceinline__ int swz(int r) { return (r >> 1) & (KV - 1); }
constexpr int NT = 256;
constexpr int KC_STEPS = 8;   // float32 accumulation chunk of the SYRK (8 x 32 columns)

// v_mfma_f32_16x16x32_{bf16,f16} (gfx950): lane l supplies A[l % 16][8 (l / 16) + t]
// and B[8 (l / 16) + t][l % 16], t = 0..7; accumulator register r of lane l
// holds D[4 (l / 16) + r][l % 16].
__device__ __forceinline__ int crow(int lane, int r) { return 4 * (lane >> 4) + r; }

template <bool F16>
__device__ __forceinline__ f4 mfma(const u16x8& a, const u16x8& b, const f4& c) {
  if constexpr (F16)
    return __builtin_amdgcn_mfma_f32_16x16x32_f16(__builtin_bit_cast(f16x8, a),
                                                  __builtin_bit_cast(f16x8, b), c, 0, 0, 0);
  else
    return __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(bf16x8, a),
                                                   __builtin_bit_cast(bf16x8, b), c, 0, 0, 0);
}

// float -> bf16 bits, round to nearest even
__device__ __forceinline__ u16 f2bf(float f) {
  const unsigned u = __float_as_uint(f);
  return (u16)((u + 0x7fffu + ((u >> 16) & 1u)) >> 16);
}
__device__ __forceinline__ float bf2f(u16 b) { return __uint_as_float((unsigned)b << 16); }

template <bool F16>
__device__ __forceinline__ void split(float x, u16& hi, u16& lo) {
  if constexpr (F16) {
    const _Float16 h = (_Float16)x;
    const _Float16 l = (_Float16)(x - (float)h);
    hi = __builtin_bit_cast(u16, h);
    lo = __builtin_bit_cast(u16, l);
  } else {
    hi = f2bf(x);
    lo = f2bf(x - bf2f(hi));
  }
}

__device__ __forceinline__ long xcd_remap(long w, long G) {
  const long per = G / 8, rem = G % 8;
  const long xcd = w % 8, slot = w / 8;
  return xcd < rem ? xcd * (per + 1) + slot : rem * (per + 1) + (xcd - rem) * per + slot;
}

// Largest exponent any scaled operand may reach: |x| * 2^scale < 2^EMAX
// keeps fp16 hi (max 65504) finite with headroom.
constexpr int EMAX = 13;

// Per-row statistics of float64 rows of length Q. Row r = (ia, ib), ib
// fastest; its group is g = ia * gsa + ib * gsb. gexp[g] receives the
// largest exponent e with |x| < 2^e over the group (integer atomicMax); nrm2
// receives the largest squared row 2-norm (as the ordered bit pattern of a
// non-negative double).
__global__ void row_stats_kernel(const double* in, long s_in_a, long s_in_b, int nb, int Q,
                                 long rows, long gsa, long gsb, int* gexp,
                                 unsigned long long* nrm2) {
  const int lane = threadIdx.x & 63;
  const long wave0 = (blockIdx.x * (long)blockDim.x + threadIdx.x) >> 6;
  const long nwaves = ((long)gridDim.x * blockDim.x) >> 6;
  for (long r = wave0; r < rows; r += nwaves) {
    const long ia = r / nb, ib = r % nb;
    const double* row = in + ia * s_in_a + ib * s_in_b;
    double mx = 0.0, ss = 0.0;
    for (int q = lane; q < Q; q += 64) {
      const double x = row[q];
      mx = fmax(mx, fabs(x));
      ss += x * x;
    }
    for (int off = 32; off > 0; off >>= 1) {
      mx = fmax(mx, __shfl_down(mx, off, 64));
      ss += __shfl_down(ss, off, 64);
    }
    if (lane == 0) {
      int e = 0;
      if (mx > 0.0) frexp(mx, &e);
      else e = -1000;
      atomicMax(&gexp[ia * gsa + ib * gsb], e);
      atomicMax(nrm2, (unsigned long long)__double_as_longlong(ss));
    }
  }
}

// float64 rows -> 16-bit hi/lo rows, zero padded from Q to Qs, scaled by
// 2^(EMAX - gexp[ia * gsa + ib * gsb]) when gexp is given (fp16 format).
// Column qq of the output holds input column perm[qq] (perm[qq] < 0: zero).
template <bool F16>
__global__ void split_rows_kernel(const double* in, long s_in_a, long s_in_b, int nb,
                                  const int* perm, u16* hi, u16* lo, long s_out_a,
                                  long s_out_b, long kblk, int Qs, long rows, const int* gexp,
                                  long gsa, long gsb) {
  const long tot = rows * Qs;
  for (long idx = blockIdx.x * (long)blockDim.x + threadIdx.x; idx < tot;
       idx += (long)gridDim.x * blockDim.x) {
    const long r = idx / Qs;
    const int q = (int)(idx % Qs);
    const long ia = r / nb, ib = r % nb;
    const int src = perm[q];
    double x = src >= 0 ? in[ia * s_in_a + ib * s_in_b + src] : 0.0;
    if (gexp) x = ldexp(x, EMAX - gexp[ia * gsa + ib * gsb]);
    u16 h, l;
    split<F16>((float)x, h, l);
    const long o = (q / KS) * kblk + (ia * s_out_a + ib * s_out_b) * KS + (q % KS);
    hi[o] = h;
    lo[o] = l;
  }
}

// Slab as a plain tiled GEMM over blocks of poles:
//   X[(p, x)][(q, c)] = sum_Q R[p][x][Q] S[q][c][Q]
// for p in a row block and q in a column block, with rows and columns
// addressed through (pole, index) pairs. 256x320 output tiles, eight waves of
// 128x80 (8x5 MFMA blocks each, two waves per SIMD), float32 accumulators.
// The 16-bit operand arrays are K-blocked: element (row r, Q index k) sits at
// (k / KS) kblk + r KS + k % KS, kblk = KS x (rows of the whole array), so the
// KS columns of consecutive rows that one step reads are contiguous.
struct XgemmArgs {
  const u16* Ah; const u16* Al; long sAp, sAx; int mA;   // row m: (m / mA) sAp + (m % mA) sAx
  const u16* Bh; const u16* Bl; long sBq, sBc; int nB;   // row n: (n / nB) sBq + (n % nB) sBc
  long kblkA, kblkB;                                      // K-block strides (elements)
  int M, Nn, Qs;
  float* C; long ldc;
  int tiles_m, tiles_n;
};

constexpr int GT = 256;    // slab tile rows: two waves of 128
constexpr int GTN = 320;   // slab tile columns: four waves of 80

// One launch carries up to XB problems of the same inner size (the mirrored
// slabs of several block pairs): problem k owns workgroups [start[k],
// start[k+1]), so the device does not idle between partly filled rounds.
constexpr int XB = 8;
struct XgemmBatch {
  XgemmArgs p[XB];
  int start[XB + 1];
  int n;
};

// Eight waves (two per SIMD) share one 256 x 320 output tile, each wave a
// 128 x 80 block of 8 x 5 MFMA tiles, so a SIMD can issue one wave's MFMAs
// while the other waits on LDS or global memory.
constexpr int XNT = 512;

template <bool F16>
__global__ __launch_bounds__(XNT) void xgemm_split_kernel(XgemmBatch b) {
  // two stages, each its own LDS arrays (hi, lo planes of A and of B): 144 KiB.
  // Separate arrays let the compiler see that the stage being read is not the
  // one the direct loads are filling, so it waits for those loads only where
  // the code says so (before the barrier that ends a step).
  __shared__ u16x8 sA0[2][GT][KV], sB0[2][GTN][KV], sA1[2][GT][KV], sB1[2][GTN][KV];
  const int tid = threadIdx.x, lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const long G = (long)gridDim.x;
  long logical = xcd_remap(blockIdx.x, G);
  int k = 0;
  while (k + 1 < b.n && logical >= b.start[k + 1]) ++k;
  const XgemmArgs& a = b.p[k];
  logical -= b.start[k];
  const int tm = (int)(logical / a.tiles_n), tn = (int)(logical % a.tiles_n);
  const int m0 = tm * GT, n0 = tn * GTN;
  // direct-to-LDS loader: a stage is 72 blocks of 16 rows (blocks 0-31: A
  // plane bl / 16 of Ah, Al, rows 16 (bl % 16) ..; blocks 32-71: B plane
  // (bl - 32) / 20 of Bh, Bl, rows 16 ((bl - 32) % 20) ..); wave w fills
  // blocks 9w .. 9w + 8. Lane l lands in LDS slot l % 4 of row l / 4 of its
  // block, so it loads global vector (l % 4) ^ swz(row) of that row (the
  // conflict-free layout of the fragment reads). Rows past M (N) read row
  // M - 1 (N - 1): they only feed outputs that are not stored.
  const u16* src[9];
#pragma unroll
  for (int j = 0; j < 9; ++j) {
    const int bl = 9 * wave + j;
    const bool isa = bl < 32;
    const int b2 = isa ? bl : bl - 32;
    const int plane = isa ? b2 >> 4 : b2 / 20, rb = isa ? b2 & 15 : b2 % 20;
    const int r = 16 * rb + (lane >> 2);
    const int kvg = (lane & 3) ^ swz(r);
    if (isa) {
      const int m = min(m0 + r, a.M - 1);
      src[j] = (plane == 0 ? a.Ah : a.Al) +
               ((long)(m / a.mA) * a.sAp + (long)(m % a.mA) * a.sAx) * KS + 8 * kvg;
    } else {
      const int n = min(n0 + r, a.Nn - 1);
      src[j] = (plane == 0 ? a.Bh : a.Bl) +
               ((long)(n / a.nB) * a.sBq + (long)(n % a.nB) * a.sBc) * KS + 8 * kvg;
    }
  }
  typedef u16x8 StageA[2][GT][KV];
  typedef u16x8 StageB[2][GTN][KV];
  auto issue = [&](int kb, StageA& dA, StageB& dB) {
#pragma unroll
    for (int j = 0; j < 9; ++j) {
      const int bl = 9 * wave + j;
      const bool isa = bl < 32;
      const int b2 = isa ? bl : bl - 32;
      const int plane = isa ? b2 >> 4 : b2 / 20, row0 = 16 * (isa ? b2 & 15 : b2 % 20);
      u16x8* dst = isa ? &dA[plane][row0][0] : &dB[plane][row0][0];
      const long kofs = (long)(kb / KS) * (isa ? a.kblkA : a.kblkB);
      __builtin_amdgcn_global_load_lds((const void*)(src[j] + kofs),
                                       (__attribute__((address_space(3))) void*)dst, 16, 0, 0);
    }
  };
  const int fr = lane & 15, fk = lane >> 4;
  const int wm = (wave & 1) * 128, wn = (wave >> 1) * 80;
  f4 acc[8][5];
#pragma unroll
  for (int i = 0; i < 8; ++i)
#pragma unroll
    for (int j = 0; j < 5; ++j) acc[i][j] = f4{0.f, 0.f, 0.f, 0.f};
  const int nsteps = a.Qs / KS;
  // step s reads stage s & 1 and first starts the direct loads of step s + 1
  // (the last step re-loads itself) into the other stage, whose last readers
  // (step s - 1) the previous barrier has passed; every wave waits for its
  // own loads before the barrier that ends the step
  auto body = [&](int step, StageA& cA, StageB& cB, StageA& nA, StageB& nB) {
    issue(min(step + 1, nsteps - 1) * KS, nA, nB);
    __builtin_amdgcn_sched_barrier(0);
    u16x8 bh[5], bl[5];
#pragma unroll
    for (int j = 0; j < 5; ++j) {
      const int r = wn + 16 * j + fr;
      bh[j] = cB[0][r][fk ^ swz(r)];
      bl[j] = cB[1][r][fk ^ swz(r)];
    }
#pragma unroll
    for (int i = 0; i < 8; ++i) {
      const int r = wm + 16 * i + fr;
      const u16x8 ah = cA[0][r][fk ^ swz(r)], al = cA[1][r][fk ^ swz(r)];
#pragma unroll
      for (int j = 0; j < 5; ++j) {
        acc[i][j] = mfma<F16>(ah, bh[j], acc[i][j]);
        acc[i][j] = mfma<F16>(ah, bl[j], acc[i][j]);
        acc[i][j] = mfma<F16>(al, bh[j], acc[i][j]);
      }
    }
    __builtin_amdgcn_s_waitcnt(0);
    __syncthreads();
  };
  issue(0, sA0, sB0);
  __builtin_amdgcn_s_waitcnt(0);
  __syncthreads();
  int step = 0;
  for (; step + 2 <= nsteps; step += 2) {
    body(step, sA0, sB0, sA1, sB1);
    body(step + 1, sA1, sB1, sA0, sB0);
  }
  if (step < nsteps) body(step, sA0, sB0, sA1, sB1);
  float* const C = a.C;
  const long ldc = a.ldc;
  const int M = a.M, Nn = a.Nn;
#pragma unroll
  for (int i = 0; i < 8; ++i)
#pragma unroll
    for (int j = 0; j < 5; ++j)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int m = m0 + wm + 16 * i + crow(lane, r);
        const int n = n0 + wn + 16 * j + fr;
        if (m < M && n < Nn) C[(long)m * ldc + n] = acc[i][j][r];
      }
}

// Pairs the slabs of a block pair into Z columns. For pole pair (p, q) of the
// chunk, X^{pq}[x][c] = (xp|qc) and X^{qp}[x][c] = (xq|pc) are read from the
// GEMM outputs (X1: rows of block P0, columns of block P1; X2: the mirrored
// block, or X1 itself when P0 == P1); the Z columns are
// sqrt(1/2)(X^{pq}+X^{qp}) and sqrt(3/2)(X^{pq}-X^{qp}) (X^{pp} for p = q),
// each with its weighted copy, stored as 16-bit pairs.
struct PairArgs {
  const float* X1; const float* X2; long ld1, ld2;
  int N, nc, P0, P1;
  const int* pa; const int* pb; const long* pcol; long col_base; int npairs;
  const int* eR; const int* eS; long sEp, sEc;
  float zscale, wscale;
  const double* ep; const double* ec;
  u16* Zh; u16* Zl; u16* Wh; u16* Wl; long zblk;
};

// The Z arrays (Z and wZ, hi and lo) are stored K-blocked: column k of row x
// sits at (k / KS) zblk + x KS + k % KS with zblk = KS N, so the KS columns of
// a run of rows that one SYRK step reads are one contiguous block.
__device__ __forceinline__ long zaddr(long zblk, int x, long k) {
  return (k / KS) * zblk + (long)x * KS + (k % KS);
}

// Z column values of one (pair, x, c): the P column sqrt(1/2)(x1 + x2) and
// the M column sqrt(3/2)(x1 - x2) (only x1 for p = q), each with its weighted
// copy, as 16-bit pairs: out = {Zh, Zl, Wh, Wl} of P, then of M.
template <bool F16>
__device__ __forceinline__ void pair_values(float x1, float x2, bool diag, float wgt,
                                            float zscale, float wscale, u16 out[8]) {
  // sqrt(1/2) and sqrt(3/2) as float pairs: every column is multiplied with
  // one rounding (fma), so the constants' own float rounding does not bias
  // all P or all M columns alike
  const float cp_hi = 0.707106769084930419921875f, cp_lo = 1.2101617485882343e-08f;
  const float cm_hi = 1.22474491596221923828125f, cm_lo = -4.4570629853524224e-08f;
  float zp = x1, zm = 0.f;
  if (!diag) {
    const float sp = x1 + x2, sm = x1 - x2;
    zp = fmaf(sp, cp_hi, sp * cp_lo);
    zm = fmaf(sm, cm_hi, sm * cm_lo);
  }
  split<F16>(zscale * zp, out[0], out[1]);
  split<F16>(wscale * (wgt * zp), out[2], out[3]);
  split<F16>(zscale * zm, out[4], out[5]);
  split<F16>(wscale * (wgt * zm), out[6], out[7]);
}

// Grid: one workgroup per (element block, pair), numbered block-major with
// the pairs inner and dealt to XCDs in contiguous ranges, so the workgroups
// writing neighbouring pairs' columns of one Z row (which share cache lines)
// run on one XCD at about the same time. A thread takes PU elements (all
// slab loads first, then the arithmetic and stores; PU = 8 for long inner
// pole ranges, where the per-pair table fill is amortised over fewer rows,
// else 4); with V = 2 an element
// is two adjacent inner poles c, c+1 (nc even: the slab reads are 8-byte and
// the Z stores 4-byte aligned, since pair column offsets are multiples of nc,
// so both columns of an element fall in one K block).
template <bool F16, int V, int PU>
__global__ __launch_bounds__(256) void pair_split_kernel(PairArgs a) {
  const long logical = xcd_remap(blockIdx.x, (long)gridDim.x);
  const int xb = (int)(logical / a.npairs), pr = (int)(logical % a.npairs);
  const int p = a.pa[pr], q = a.pb[pr];
  const bool diag = (p == q);
  const long colbase = a.pcol[pr] - a.col_base;
  const int ncv = a.nc / V;
  const int per = a.N * ncv;
  const float* r1 = a.X1 + (long)(p - a.P0) * a.N * a.ld1 + (long)(q - a.P1) * a.nc;
  const float* r2 = (a.P0 == a.P1)
                        ? a.X1 + (long)(q - a.P0) * a.N * a.ld1 + (long)(p - a.P1) * a.nc
                        : a.X2 + (long)(q - a.P1) * a.N * a.ld2 + (long)(p - a.P0) * a.nc;
  const long ld2 = (a.P0 == a.P1) ? a.ld1 : a.ld2;
  // per inner pole c of this pair: the two fp16 scale exponents and the
  // weight, gathered once per workgroup (the exponent tables can be strided
  // in c) instead of once per element
  extern __shared__ int ptab[];
  int* t1 = ptab;
  int* t2 = ptab + a.nc;
  float* tw = reinterpret_cast<float*>(ptab + 2 * a.nc);
  for (int cc = threadIdx.x; cc < a.nc; cc += 256) {
    if constexpr (F16) {
      t1[cc] = a.eR[p] + a.eS[(long)q * a.sEp + (long)cc * a.sEc] - 2 * EMAX;
      t2[cc] = diag ? 0 : a.eR[q] + a.eS[(long)p * a.sEp + (long)cc * a.sEc] - 2 * EMAX;
    }
    tw[cc] = (float)(a.ep[p] + a.ep[q] - a.ec[cc]);
  }
  const int e0 = xb * (256 * PU) + threadIdx.x;
  float x1[PU][V], x2[PU][V];
#pragma unroll
  for (int u = 0; u < PU; ++u) {
    const int e = e0 + 256 * u;
#pragma unroll
    for (int t = 0; t < V; ++t) x1[u][t] = x2[u][t] = 0.f;
    if (e >= per) continue;
    const int x = e / ncv, c = V * (e - x * ncv);
    if constexpr (V == 2) {
      const float2 v1 = *reinterpret_cast<const float2*>(r1 + (long)x * a.ld1 + c);
      x1[u][0] = v1.x; x1[u][1] = v1.y;
      if (!diag) {
        const float2 v2 = *reinterpret_cast<const float2*>(r2 + (long)x * ld2 + c);
        x2[u][0] = v2.x; x2[u][1] = v2.y;
      }
    } else {
      x1[u][0] = r1[(long)x * a.ld1 + c];
      if (!diag) x2[u][0] = r2[(long)x * ld2 + c];
    }
  }
  __syncthreads();
#pragma unroll
  for (int u = 0; u < PU; ++u) {
    const int e = e0 + 256 * u;
    if (e >= per) continue;
    const int x = e / ncv, c = V * (e - x * ncv);
    const long o = zaddr(a.zblk, x, colbase + c);          // P column
    const long om = zaddr(a.zblk, x, colbase + a.nc + c);  // M column
    u16 v[V][8];
#pragma unroll
    for (int t = 0; t < V; ++t) {
      const int cc = c + t;
      float y1 = x1[u][t], y2 = x2[u][t];
      if constexpr (F16) {
        y1 = ldexpf(y1, t1[cc]);
        if (!diag) y2 = ldexpf(y2, t2[cc]);
      }
      pair_values<F16>(y1, y2, diag, tw[cc], a.zscale, a.wscale, v[t]);
    }
    u16* dst[4] = {a.Zh, a.Zl, a.Wh, a.Wl};
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      if constexpr (V == 2) {
        *reinterpret_cast<unsigned*>(dst[k] + o) = (unsigned)v[0][k] | ((unsigned)v[1][k] << 16);
        if (!diag)
          *reinterpret_cast<unsigned*>(dst[k] + om) =
              (unsigned)v[0][4 + k] | ((unsigned)v[1][4 + k] << 16);
      } else {
        dst[k][o] = v[0][k];
        if (!diag) dst[k][om] = v[0][4 + k];
      }
    }
  }
}

// Pairing where every pair's P and M column blocks are ncp columns long, ncp a
// multiple of KS (the last ncp - nc columns of each block are zero), so that
// each K block of Z lies in one block of one pair. A workgroup takes one pair
// and 16 rows x; thread t owns row x0 + t / 16 and the columns 2 (t % 16) and
// 2 (t % 16) + 1 of every K block of the pair, walking the K blocks UK at a
// time. A wave then stores four consecutive rows of one K block, 256
// contiguous bytes per plane, and reads 128 contiguous bytes of each of its
// four slab rows. V2: nc even, so the slab reads are 8-byte aligned float2.
template <bool F16, bool V2>
__global__ __launch_bounds__(256) void pair_split_blk_kernel(PairArgs a, int ncp) {
  constexpr int UK = 4;
  const long logical = xcd_remap(blockIdx.x, (long)gridDim.x);
  const int xg = (int)(logical / a.npairs), pr = (int)(logical % a.npairs);
  const int p = a.pa[pr], q = a.pb[pr];
  const bool diag = (p == q);
  const long kb0 = (a.pcol[pr] - a.col_base) / KS;   // first K block of the P columns
  const int nkb = ncp / KS;
  const float* r1 = a.X1 + (long)(p - a.P0) * a.N * a.ld1 + (long)(q - a.P1) * a.nc;
  const float* r2 = (a.P0 == a.P1)
                        ? a.X1 + (long)(q - a.P0) * a.N * a.ld1 + (long)(p - a.P1) * a.nc
                        : a.X2 + (long)(q - a.P1) * a.N * a.ld2 + (long)(p - a.P0) * a.nc;
  const long ld2 = (a.P0 == a.P1) ? a.ld1 : a.ld2;
  extern __shared__ int ptab[];
  int* t1 = ptab;
  int* t2 = ptab + a.nc;
  float* tw = reinterpret_cast<float*>(ptab + 2 * a.nc);
  for (int cc = threadIdx.x; cc < a.nc; cc += 256) {
    if constexpr (F16) {
      t1[cc] = a.eR[p] + a.eS[(long)q * a.sEp + (long)cc * a.sEc] - 2 * EMAX;
      t2[cc] = diag ? 0 : a.eR[q] + a.eS[(long)p * a.sEp + (long)cc * a.sEc] - 2 * EMAX;
    }
    tw[cc] = (float)(a.ep[p] + a.ep[q] - a.ec[cc]);
  }
  __syncthreads();
  const int x = xg * 16 + (int)(threadIdx.x / 16);
  if (x >= a.N) return;   // no barrier follows
  const int cl = 2 * (int)(threadIdx.x % 16);
  const float* row1 = r1 + (long)x * a.ld1;
  const float* row2 = r2 + (long)x * ld2;
  const long zrow = (long)x * KS + cl;
  u16* dst[4] = {a.Zh, a.Zl, a.Wh, a.Wl};
  for (int kb = 0; kb < nkb; kb += UK) {
    float x1[UK][2], x2[UK][2];
#pragma unroll
    for (int u = 0; u < UK; ++u) {
      const int c = (kb + u) * KS + cl;
      x1[u][0] = x1[u][1] = x2[u][0] = x2[u][1] = 0.f;
      if constexpr (V2) {
        if (c < a.nc) {   // nc even: c + 1 < nc too
          const float2 v1 = *reinterpret_cast<const float2*>(row1 + c);
          x1[u][0] = v1.x; x1[u][1] = v1.y;
          if (!diag) {
            const float2 v2 = *reinterpret_cast<const float2*>(row2 + c);
            x2[u][0] = v2.x; x2[u][1] = v2.y;
          }
        }
      } else {
#pragma unroll
        for (int t = 0; t < 2; ++t)
          if (c + t < a.nc) {
            x1[u][t] = row1[c + t];
            if (!diag) x2[u][t] = row2[c + t];
          }
      }
    }
#pragma unroll
    for (int u = 0; u < UK; ++u) {
      if (kb + u >= nkb) break;
      const int c = (kb + u) * KS + cl;
      u16 v[2][8];
#pragma unroll
      for (int t = 0; t < 2; ++t) {
        const int cc = c + t;
        if (cc < a.nc) {
          float y1 = x1[u][t], y2 = x2[u][t];
          if constexpr (F16) {
            y1 = ldexpf(y1, t1[cc]);
            if (!diag) y2 = ldexpf(y2, t2[cc]);
          }
          pair_values<F16>(y1, y2, diag, tw[cc], a.zscale, a.wscale, v[t]);
        } else {
#pragma unroll
          for (int k = 0; k < 8; ++k) v[t][k] = 0;   // padding column
        }
      }
      const long o = (kb0 + kb + u) * a.zblk + zrow;          // P column block
      const long om = (kb0 + nkb + kb + u) * a.zblk + zrow;   // M column block
#pragma unroll
      for (int k = 0; k < 4; ++k) {
        *reinterpret_cast<unsigned*>(dst[k] + o) = (unsigned)v[0][k] | ((unsigned)v[1][k] << 16);
        if (!diag)
          *reinterpret_cast<unsigned*>(dst[k] + om) =
              (unsigned)v[0][4 + k] | ((unsigned)v[1][4 + k] << 16);
      }
    }
  }
}

// out[a][i] = in[i][a] (o x v ints)
__global__ void transpose_int_kernel(int o, int v, const int* in, int* out) {
  const long n = (long)o * v;
  for (long k = blockIdx.x * (long)blockDim.x + threadIdx.x; k < n;
       k += (long)gridDim.x * blockDim.x)
    out[k] = in[(k % o) * v + k / o];
}

struct SyrkArgs {
  const u16* Zh; const u16* Zl; const u16* Wh; const u16* Wl; long zblk;  // K-blocked
  int N; long K; long kper;
  double u0scale, u1scale;   // 2^-2fZ, 2^-(fZ+fW)
  double* part; long part_stride;
  int tiles, nsplit, nxt;    // lower-triangle tiles, K splits (grid = tiles * nsplit), x blocks
  int lolo_all;              // 1: lo*lo products on every sub-tile
};

constexpr int SX = 64, SY = 128;   // SYRK output tile: 64 x rows by 128 y rows
constexpr int SNT = 512;           // eight waves, two per SIMD

// Lower-triangle tiles of U0 += Z Z^T and U1 += (wZ) Z^T from the 16-bit
// pairs, K split into float64 partials. Tile t is numbered y block major: y
// block yt (128 rows) holds x blocks (64 rows) 2 yt .. nxt - 1, the x blocks
// that reach the diagonal or below it. Each wave owns a 32 x 32 sub-tile and
// both moments; a wave whose sub-tile lies above the diagonal skips its
// MFMAs. A 64 x 128 tile moves a third fewer operand bytes per output element
// than a 64 x 64 one.
// Products: hi*hi into one float32 sum, hi*lo + lo*hi (+ lo*lo) into another;
// every KC_STEPS steps both are folded into float64. lo*lo is taken only on
// sub-tiles holding diagonal elements (or on all with lolo_all): there it is
// a non-negative square that dropping would bias, elsewhere a term of random
// sign ~2^-22 times the summand (measured: no change of the moment errors).
template <bool F16>
__global__ __launch_bounds__(SNT) void syrk_split_kernel(SyrkArgs a) {
  // two stages (double buffer) of: Z hi, Z lo, wZ hi, wZ lo (x rows) and
  // Z hi, Z lo (y rows); 64 KiB
  __shared__ u16x8 sX[2][4][SX][KV];
  __shared__ u16x8 sY[2][2][SY][KV];
  const int tid = threadIdx.x, lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  // (split, tile) work items numbered split-major and dealt to XCDs in
  // contiguous ranges, so the tiles reading one K range share an L2
  const long item = xcd_remap(blockIdx.x, (long)a.tiles * a.nsplit);
  const int t = (int)(item % a.tiles);
  const int s = (int)(item / a.tiles);
  int yt = 0, toff = 0;
  while (toff + (a.nxt - 2 * yt) <= t) {
    toff += a.nxt - 2 * yt;
    ++yt;
  }
  const int xt = 2 * yt + (t - toff);
  const long k0 = (long)s * a.kper, k1 = std::min(a.K, k0 + a.kper);
  if (k1 <= k0) return;   // uniform over the workgroup
  const int x0 = xt * SX, y0 = yt * SY;

  // Loader: a step is 2048 16-byte vectors (x: 4 arrays x 64 rows x KV; y: 2
  // arrays x 128 rows x KV); thread tid moves vectors tid + 512 i, i = 0..3
  // (i = 0, 1: x arrays 2i, 2i + 1; i = 2, 3: y arrays), with global row
  // pointers and LDS slots fixed for the whole K range. A step reads one K
  // block (the K range starts on a block boundary), in which the tile's rows
  // are contiguous: 64 or 128 rows of 64 bytes. Rows past N read row N - 1
  // (their outputs are not stored) and the blocks read lie below kcap, so
  // every load is unconditional and in bounds.
  const u16* gp[4];
  int lo[4];
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    const int idx = tid + SNT * i;
    const int kv = idx % KV;
    if (i < 2) {
      const int arr = idx / (SX * KV), rr = (idx / KV) % SX;
      const u16* base = arr == 0 ? a.Zh : arr == 1 ? a.Zl : arr == 2 ? a.Wh : a.Wl;
      gp[i] = base + (long)min(x0 + rr, a.N - 1) * KS + 8 * kv;
      lo[i] = (arr * SX + rr) * KV + (kv ^ swz(rr));
    } else {
      const int j = idx - 2 * SNT;
      const int arr = j / (SY * KV), rr = (j / KV) % SY;
      const u16* base = arr == 0 ? a.Zh : a.Zl;
      gp[i] = base + (long)min(y0 + rr, a.N - 1) * KS + 8 * kv;
      lo[i] = (arr * SY + rr) * KV + (kv ^ swz(rr));
    }
  }
  // register stages: the global loads run two k steps ahead of the MFMAs;
  // steps past the end re-read the last one (unused), columns >= k1 of the
  // last step are zeroed at store time
  const long nsteps = (k1 - k0 + KS - 1) / KS;
  const long kb_last = k0 + (nsteps - 1) * KS;
  auto load = [&](long kb, u16x8 (&r)[4]) {
    kb = min(kb, kb_last);
#pragma unroll
    for (int i = 0; i < 4; ++i) r[i] = *reinterpret_cast<const u16x8*>(gp[i] + (kb / KS) * a.zblk);
  };
  auto store = [&](int buf, long kb, u16x8 (&r)[4]) {
    if (kb + KS > k1) {
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const long k = kb + 8 * ((tid + SNT * i) % KV);
#pragma unroll
        for (int e = 0; e < 8; ++e)
          if (k + e >= k1) r[i][e] = 0;
      }
    }
    u16x8* bx = &sX[buf][0][0][0];
    u16x8* by = &sY[buf][0][0][0];
#pragma unroll
    for (int i = 0; i < 2; ++i) bx[lo[i]] = r[i];
#pragma unroll
    for (int i = 2; i < 4; ++i) by[lo[i]] = r[i];
  };

  const int fr = lane & 15, fk = lane >> 4;
  const int wm = (wave & 1) * 32, wn = (wave >> 1) * 32;
  const int gx = x0 + wm, gy = y0 + wn;
  const bool active = gx + 31 >= gy;          // some element on or below the diagonal
  const bool lolo = a.lolo_all || gx == gy;    // sub-tile holds diagonal elements
  f4 u0[2][2], u1[2][2], v0[2][2], v1[2][2];
  double s0[2][2][4], s1[2][2][4];
  const f4 z4 = f4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j) {
      u0[i][j] = u1[i][j] = v0[i][j] = v1[i][j] = z4;
#pragma unroll
      for (int r = 0; r < 4; ++r) s0[i][j][r] = s1[i][j][r] = 0.0;
    }
  auto flush = [&]() {
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
      for (int j = 0; j < 2; ++j) {
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          s0[i][j][r] += a.u0scale * ((double)u0[i][j][r] + (double)v0[i][j][r]);
          s1[i][j][r] += a.u1scale * ((double)u1[i][j][r] + (double)v1[i][j][r]);
        }
        u0[i][j] = u1[i][j] = v0[i][j] = v1[i][j] = z4;
      }
  };

  // Step s reads LDS stage s & 1. Its body first reloads the register stage
  // that held step s (already in LDS) with step s + 2, then runs the MFMAs,
  // then writes step s + 1 (loaded during step s - 1) into the other LDS
  // stage, whose last readers (step s - 1) the previous barrier has passed.
  // Steps run in pairs with no branch around loads or stores; for odd nsteps
  // the last body multiplies the zeroed data of step nsteps (all its columns
  // are >= k1), which adds exact zeros.
  auto body = [&](long step, int buf, u16x8 (&cur)[4], u16x8 (&nxt)[4]) {
    load(k0 + (step + 2) * KS, cur);
    if (active) {
      u16x8 xh[2], xl[2], wh[2], wl[2], yh[2], yl[2];
#pragma unroll
      for (int i = 0; i < 2; ++i) {
        const int rx_ = wm + 16 * i + fr, ry_ = wn + 16 * i + fr;
        const int sx = fk ^ swz(rx_), sy = fk ^ swz(ry_);
        xh[i] = sX[buf][0][rx_][sx];
        xl[i] = sX[buf][1][rx_][sx];
        wh[i] = sX[buf][2][rx_][sx];
        wl[i] = sX[buf][3][rx_][sx];
        yh[i] = sY[buf][0][ry_][sy];
        yl[i] = sY[buf][1][ry_][sy];
      }
#pragma unroll
      for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j) {
          u0[i][j] = mfma<F16>(xh[i], yh[j], u0[i][j]);
          v0[i][j] = mfma<F16>(xh[i], yl[j], v0[i][j]);
          v0[i][j] = mfma<F16>(xl[i], yh[j], v0[i][j]);
          u1[i][j] = mfma<F16>(wh[i], yh[j], u1[i][j]);
          v1[i][j] = mfma<F16>(wh[i], yl[j], v1[i][j]);
          v1[i][j] = mfma<F16>(wl[i], yh[j], v1[i][j]);
          if (lolo) {
            v0[i][j] = mfma<F16>(xl[i], yl[j], v0[i][j]);
            v1[i][j] = mfma<F16>(wl[i], yl[j], v1[i][j]);
          }
        }
      if ((step + 1) % KC_STEPS == 0) flush();
    }
    store(buf ^ 1, k0 + (step + 1) * KS, nxt);
    __syncthreads();
  };
  u16x8 ra[4], rb[4];
  load(k0, ra);
  load(k0 + KS, rb);
  store(0, k0, ra);
  __syncthreads();
  for (long step = 0; step < nsteps; step += 2) {
    body(step, 0, ra, rb);
    body(step + 1, 1, rb, ra);
  }
  if (!active) return;
  flush();

  double* P0 = a.part + (long)s * a.part_stride;
  double* P1 = P0 + (long)a.N * a.N;
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int x = gx + 16 * i + crow(lane, r);
        const int y = gy + 16 * j + fr;
        if (x >= a.N || y > x) continue;
        const long o = (long)x * a.N + y;
        P0[o] += s0[i][j][r];
        P1[o] += s1[i][j][r];
      }
}

// Rows (ia, ib) of `in` (float64, Q index permuted by perm) as 16-bit pairs
// in the K-blocked layout: output row ia s_out_a + ib s_out_b (in rows) of an
// array whose K blocks are kblk elements apart; hi and lo point at this
// chunk's first row.
template <bool F16>
void split_rows(const double* in, long s_in_a, long s_in_b, int na, int nb, const int* perm,
                u16* hi, u16* lo, long s_out_a, long s_out_b, long kblk, int Qs,
                const int* gexp, long gsa, long gsb, hipStream_t st) {
  const long rows = (long)na * nb;
  const long tot = rows * Qs;
  if (tot == 0) return;
  const long blocks = std::min<long>((tot + 255) / 256, 16384);
  hipLaunchKernelGGL((split_rows_kernel<F16>), dim3(blocks), dim3(256), 0, st, in, s_in_a,
                     s_in_b, nb, perm, hi, lo, s_out_a, s_out_b, kblk, Qs, rows, gexp, gsa,
                     gsb);
  AGF2_CHECK_LAUNCH();
}

// sq[Q] = sum_pq L[Q][p][q]^2 (one workgroup per Q)
__global__ __launch_bounds__(256) void slice_norm_kernel(const double* L, long nn, double* sq) {
  __shared__ double red[256];
  const double* LQ = L + blockIdx.x * nn;
  double acc = 0.0;
  for (long i = threadIdx.x; i < nn; i += 256) acc += LQ[i] * LQ[i];
  red[threadIdx.x] = acc;
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if (threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
    __syncthreads();
  }
  if (threadIdx.x == 0) sq[blockIdx.x] = red[0];
}

void row_stats(const double* in, long s_in_a, long s_in_b, int na, int nb, int Q, long gsa,
               long gsb, int* gexp, unsigned long long* nrm2, hipStream_t st) {
  const long rows = (long)na * nb;
  if (rows == 0) return;
  const long blocks = std::min<long>((rows + 3) / 4, 8192);
  hipLaunchKernelGGL(row_stats_kernel, dim3(blocks), dim3(256), 0, st, in, s_in_a, s_in_b, nb,
                     Q, rows, gsa, gsb, gexp, nrm2);
  AGF2_CHECK_LAUNCH();
}

// binary exponent e with |x| < 2^e (x > 0)
int exponent_above(double x) {
  int e = 0;
  if (x > 0.0) std::frexp(x, &e);
  return e;
}

// 1 when AGF2_SYRK_LOLO_ALL=1 is set in the environment: lo*lo products on
// every contraction sub-tile instead of the diagonal ones only (a precision
// check of the default)
int lolo_all() {
  static int v = -1;
  if (v < 0) {
    const char* e = std::getenv("AGF2_SYRK_LOLO_ALL");
    v = (e && e[0] == '1') ? 1 : 0;
  }
  return v;
}

struct PartScales {
  const int* eR = nullptr;
  const int* eS = nullptr;
  long sEp = 0, sEc = 0;
  float zscale = 1.f, wscale = 1.f;
  double u0scale = 1.0, u1scale = 1.0;
};

}  // namespace

// Workgroups resident on the whole device for a kernel (compute units x
// resident workgroups per unit), queried once per kernel.
template <class K>
int device_slots(K kernel, int& cache, int threads = NT) {
  if (cache > 0) return cache;
  int dev = 0, cus = 0, per = 0;
  AGF2_HIP(hipGetDevice(&dev));
  AGF2_HIP(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
  AGF2_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, kernel, threads, 0));
  cache = std::max(1, cus) * std::max(1, per);
  return cache;
}

// K splits of one SYRK launch: up to nmax (and about Kc / 512), chosen so that
// tiles x splits fills whole rounds of the device's resident workgroups.
int choose_splits(long Kc, int tiles, int nmax, int slots) {
  const int hi = (int)std::max<long>(1, std::min<long>(nmax, Kc / 512));
  int best = hi;
  double best_eff = -1.0;
  for (int ns = hi; ns >= std::max(1, hi / 2); --ns) {
    const long items = (long)tiles * ns;
    const double eff = (double)items / (double)(((items + slots - 1) / slots) * slots);
    if (eff > best_eff + 1e-9) {
      best_eff = eff;
      best = ns;
    }
  }
  return best;
}

template <bool F16>
static void moments_part_split(Handle& h, int N, int Q, int Qs, const u16* Rh, const u16* Rl,
                               long sRp, long sRx, long kblkR, const u16* Sh, const u16* Sl,
                               long sSp, long sSc, long kblkS, const double* ep, int np,
                               const double* ec, int nc,
                               const PartScales& sc, double* U0, double* U1) {
  hipStream_t st = h.stream;
  const long nn = (long)N * N;
  if (np == 0 || nc == 0) {
    AGF2_HIP(hipMemsetAsync(U0, 0, nn * sizeof(double), st));
    AGF2_HIP(hipMemsetAsync(U1, 0, nn * sizeof(double), st));
    return;
  }
  // blocks of kb poles; a chunk is one block pair (ib <= jb), whose slabs
  // X1 = R[block ib] S[block jb]^T and X2 = R[block jb] S[block ib]^T are
  // float32 buffers of kb N x kb nc each (<= ~256 MiB)
  static int syrk_slots = 0;
  int kb = (int)std::floor(std::sqrt((double)(1L << 26) / ((double)N * nc)));
  kb = std::max(1, std::min({kb, np, 255}));   // <= 255^2 pairs per chunk (grid y limit)
  const int nblk = (np + kb - 1) / kb;
  // Each pair's P and M column blocks are padded with zero columns to a
  // multiple of KS when that adds at most 1/32 of the columns: a K block of Z
  // then lies in one block of one pair, and the pairing kernel stores whole
  // K-block rows (pair_split_blk_kernel) instead of pieces shared by
  // neighbouring pairs. The zero columns add nothing to the sums.
  const int ncp_full = (nc + KS - 1) / KS * KS;
  const bool padded = 32L * (ncp_full - nc) <= nc;
  const int ncp = padded ? ncp_full : nc;
  // pair list ordered by block pair, with chunk-local column offsets
  std::vector<int> hpa, hpb;
  std::vector<long> hcol;
  std::vector<long> chunk_first, chunk_cols, chunk_cols_alg;
  for (int ib = 0; ib < nblk; ++ib)
    for (int jb = ib; jb < nblk; ++jb) {
      chunk_first.push_back((long)hpa.size());
      long c0 = 0, calg = 0;
      for (int p = ib * kb; p < std::min(np, (ib + 1) * kb); ++p)
        for (int q = jb * kb; q < std::min(np, (jb + 1) * kb); ++q) {
          if (ib == jb && q < p) continue;
          hpa.push_back(p); hpb.push_back(q); hcol.push_back(c0);
          c0 += (p == q) ? ncp : 2L * ncp;
          calg += (p == q) ? nc : 2L * nc;
        }
      chunk_cols.push_back(c0);
      chunk_cols_alg.push_back(calg);
    }
  const long npairs = (long)hpa.size();
  int* d_pa = h.ws_moments[6].as<int>(2 * npairs);
  int* d_pb = d_pa + npairs;
  long* d_col = h.ws_moments[7].as<long>(npairs);
  AGF2_HIP(hipMemcpyAsync(d_pa, hpa.data(), npairs * sizeof(int), hipMemcpyHostToDevice, st));
  AGF2_HIP(hipMemcpyAsync(d_pb, hpb.data(), npairs * sizeof(int), hipMemcpyHostToDevice, st));
  AGF2_HIP(hipMemcpyAsync(d_col, hcol.data(), npairs * sizeof(long), hipMemcpyHostToDevice, st));
  AGF2_HIP(hipStreamSynchronize(st));   // host tables go out of scope below

  long kcap = 0;
  for (long c : chunk_cols) kcap = std::max(kcap, c);
  kcap = (kcap + KS - 1) / KS * KS;
  u16* Z = h.ws_moments[4].as<u16>(4L * N * kcap);
  u16 *Zh = Z, *Zl = Z + (long)N * kcap, *Wh = Z + 2L * N * kcap, *Wl = Z + 3L * N * kcap;
  // slab buffers: the two mirrored slabs of each of CB block pairs per launch
  constexpr int CB = XB / 2;
  const long xel = (long)kb * N * (long)kb * nc;
  float* X = reinterpret_cast<float*>(h.ws_moments[3].as<double>(CB * xel + 8));

  const int nxt = (N + SX - 1) / SX, nyt = (N + SY - 1) / SY;
  int ntiles = 0;
  for (int yt = 0; yt < nyt; ++yt) ntiles += std::max(0, nxt - 2 * yt);
  const int slots = device_slots(syrk_split_kernel<F16>, syrk_slots, SNT);
  // K splits for about two rounds of resident workgroups per launch: each
  // item's float64 partial-slot update (a read-modify-write of its tile) is
  // amortised over a longer K range than with eight rounds (measured at
  // nmo=1000: launches 4.6% faster), and there are fewer partial slots
  const int nsplit_max = std::max(1, std::min(64, (2 * slots + ntiles - 1) / ntiles));
  const long part_stride = 2 * nn;
  double* part = h.ws_moments[5].as<double>(part_stride * nsplit_max);
  AGF2_HIP(hipMemsetAsync(part, 0, part_stride * nsplit_max * sizeof(double), st));

  auto problem = [&](int prow, int nrow, int pcol, int ncol, float* C) {
    XgemmArgs g;
    g.Ah = Rh + (long)prow * sRp * KS; g.Al = Rl + (long)prow * sRp * KS;
    g.sAp = sRp; g.sAx = sRx; g.mA = N; g.kblkA = kblkR;
    g.Bh = Sh + (long)pcol * sSp * KS; g.Bl = Sl + (long)pcol * sSp * KS;
    g.sBq = sSp; g.sBc = sSc; g.kblkB = kblkS;
    g.nB = nc;
    g.M = nrow * N; g.Nn = ncol * nc; g.Qs = Qs;
    g.C = C; g.ldc = (long)ncol * nc;
    g.tiles_m = (g.M + GT - 1) / GT; g.tiles_n = (g.Nn + GTN - 1) / GTN;
    return g;
  };
  // one launch for the problems collected in b
  auto gemm = [&](XgemmBatch& b) {
    double fl = 0.0, by = 0.0;
    b.start[0] = 0;
    for (int k = 0; k < b.n; ++k) {
      const XgemmArgs& g = b.p[k];
      b.start[k + 1] = b.start[k] + g.tiles_m * g.tiles_n;
      fl += 2.0 * g.M * (double)g.Nn * Q;
      by += 4.0 * ((double)g.M + g.Nn) * Qs + 4.0 * (double)g.M * g.Nn;
    }
    for (int k = b.n; k < XB; ++k) {
      b.p[k] = b.p[0];
      b.start[k + 1] = b.start[b.n];
    }
    ProfScope ps(h, "moments.slab", fl, by);
    hipLaunchKernelGGL((xgemm_split_kernel<F16>), dim3((unsigned)b.start[b.n]), dim3(XNT), 0, st,
                       b);
    AGF2_CHECK_LAUNCH();
  };

  std::vector<std::pair<int, int>> blocks;   // (ib, jb) in chunk order
  for (int ib = 0; ib < nblk; ++ib)
    for (int jb = ib; jb < nblk; ++jb) blocks.push_back({ib, jb});
  const int nchunks = (int)blocks.size();
  for (int c0 = 0; c0 < nchunks; c0 += CB) {
    const int c1 = std::min(nchunks, c0 + CB);
    XgemmBatch b;
    b.n = 0;
    for (int chunk = c0; chunk < c1; ++chunk) {
      const int ib = blocks[chunk].first, jb = blocks[chunk].second;
      const int P0 = ib * kb, na = std::min(kb, np - P0);
      const int P1 = jb * kb, nb = std::min(kb, np - P1);
      float* X1 = X + 2L * (chunk - c0) * xel;
      b.p[b.n++] = problem(P0, na, P1, nb, X1);
      if (ib != jb) b.p[b.n++] = problem(P1, nb, P0, na, X1 + xel);
    }
    gemm(b);
    for (int chunk = c0; chunk < c1; ++chunk) {
      const int ib = blocks[chunk].first, jb = blocks[chunk].second;
      const int P0 = ib * kb, na = std::min(kb, np - P0);
      const int P1 = jb * kb, nb = std::min(kb, np - P1);
      const float* X1 = X + 2L * (chunk - c0) * xel;
      const float* X2 = X1 + xel;
      const long first = chunk_first[chunk];
      const long last = (chunk + 1 < (int)chunk_first.size()) ? chunk_first[chunk + 1] : npairs;
      const long Kc = chunk_cols[chunk];
      PairArgs pa;
      pa.X1 = X1; pa.X2 = X2; pa.ld1 = (long)nb * nc; pa.ld2 = (long)na * nc;
      pa.N = N; pa.nc = nc; pa.P0 = P0; pa.P1 = P1;
      pa.pa = d_pa + first; pa.pb = d_pb + first; pa.pcol = d_col + first; pa.col_base = 0;
      pa.npairs = (int)(last - first);
      pa.eR = sc.eR; pa.eS = sc.eS; pa.sEp = sc.sEp; pa.sEc = sc.sEc;
      pa.zscale = sc.zscale; pa.wscale = sc.wscale;
      pa.ep = ep; pa.ec = ec;
      pa.Zh = Zh; pa.Zl = Zl; pa.Wh = Wh; pa.Wl = Wl; pa.zblk = (long)KS * N;
      if (padded) {
        const long tot = (long)pa.npairs * N * nc;
        ProfScope ps(h, "moments.pair", 0.0, 4.0 * 2.0 * tot + 8.0 * N * (double)Kc);
        const long nxg = (N + 15) / 16;
        AGF2_REQUIRE(nxg * pa.npairs < (1L << 31), "pair chunk too large");
        const dim3 grid((unsigned)(nxg * pa.npairs));
        const size_t tab = 3 * sizeof(int) * (size_t)nc;
        AGF2_REQUIRE(tab <= 64 * 1024, "pair chunk: inner pole count too large");
        if (nc % 2 == 0)
          hipLaunchKernelGGL((pair_split_blk_kernel<F16, true>), grid, dim3(256), tab, st, pa, ncp);
        else
          hipLaunchKernelGGL((pair_split_blk_kernel<F16, false>), grid, dim3(256), tab, st, pa,
                             ncp);
        AGF2_CHECK_LAUNCH();
      } else {
        const long tot = (long)pa.npairs * N * nc;
        ProfScope ps(h, "moments.pair", 0.0, 4.0 * 2.0 * tot + 8.0 * N * (double)Kc);
        const bool two = (nc % 2 == 0) && (kcap % 2 == 0);
        const long per = (long)N * nc / (two ? 2 : 1);
        const int pu = nc >= 256 ? 8 : 4;
        const long nxb = (per + 256L * pu - 1) / (256L * pu);
        AGF2_REQUIRE((long)N * nc < (1L << 31) - 256 * pu && nxb * pa.npairs < (1L << 31),
                     "pair chunk too large");
        const dim3 grid((unsigned)(nxb * pa.npairs));
        const size_t tab = 3 * sizeof(int) * (size_t)nc;   // per-c table (LDS)
        AGF2_REQUIRE(tab <= 64 * 1024, "pair chunk: inner pole count too large");
        if (pu == 8) {
          if (two) hipLaunchKernelGGL((pair_split_kernel<F16, 2, 8>), grid, dim3(256), tab, st, pa);
          else hipLaunchKernelGGL((pair_split_kernel<F16, 1, 8>), grid, dim3(256), tab, st, pa);
        } else {
          if (two) hipLaunchKernelGGL((pair_split_kernel<F16, 2, 4>), grid, dim3(256), tab, st, pa);
          else hipLaunchKernelGGL((pair_split_kernel<F16, 1, 4>), grid, dim3(256), tab, st, pa);
        }
        AGF2_CHECK_LAUNCH();
      }
      int nsplit = choose_splits(Kc, ntiles, nsplit_max, slots);
      long kper = (Kc + nsplit - 1) / nsplit;
      kper = (kper + KS - 1) / KS * KS;
      nsplit = (int)((Kc + kper - 1) / kper);
      SyrkArgs ya;
      ya.Zh = Zh; ya.Zl = Zl; ya.Wh = Wh; ya.Wl = Wl; ya.zblk = (long)KS * N;
      ya.N = N; ya.K = Kc; ya.kper = kper;
      ya.u0scale = sc.u0scale; ya.u1scale = sc.u1scale;
      ya.part = part; ya.part_stride = part_stride;
      {
        const double Ka = (double)chunk_cols_alg[chunk];   // without padding columns
        ProfScope ps(h, "moments.syrk", 2.0 * N * (N + 1.0) * Ka, 8.0 * (N + 0.0) * Ka);
        ya.tiles = ntiles; ya.nsplit = nsplit; ya.nxt = nxt;
        ya.lolo_all = lolo_all();
        hipLaunchKernelGGL((syrk_split_kernel<F16>), dim3((unsigned)(ntiles * nsplit)),
                           dim3(SNT), 0, st, ya);
        AGF2_CHECK_LAUNCH();
      }
    }
  }
  ProfScope ps(h, "moments.reduce", 0.0, 8.0 * (2.0 * nsplit_max + 2.0) * nn);
  reduce_moment_partials(part, part_stride, nsplit_max, N, U0, U1, st);
}

template <bool F16>
static void build_split(Handle& h, int N, int Q, const double* L, int npole, int nocc,
                        const double* e, const double* u, double* m0o, double* m1o,
                        double* m0v, double* m1v) {
  hipStream_t st = h.stream;
  const int o = nocc, v = npole - nocc;
  const int Qp = (Q + 15) / 16 * 16;   // float64 staging (transform) padding
  const int Qs = (Q + KS - 1) / KS * KS;
  u16* Sxo = h.ws_moments[0].as<u16>(2L * o * N * Qs);
  u16* Sxv = h.ws_moments[1].as<u16>(2L * v * N * Qs);
  u16* Sov = h.ws_moments[2].as<u16>(2L * o * v * Qs);
  u16 *Rxo_h = Sxo, *Rxo_l = Sxo + (long)o * N * Qs;
  u16 *Rxv_h = Sxv, *Rxv_l = Sxv + (long)v * N * Qs;
  u16 *Rov_h = Sov, *Rov_l = Sov + (long)o * v * Qs;
  // the same tensor with rows (a, i): the greater part's inner pole i is then
  // the contiguous row index of its B operand
  u16* Svo = h.ws_moments[8].as<u16>(2L * o * v * Qs);
  u16 *Rvo_h = Svo, *Rvo_l = Svo + (long)o * v * Qs;
  // fp16 scale exponents: per occupied pole, per virtual pole, per (i, a) row;
  // then the squared-norm maxima of the three tensors' Q rows
  int* ex = h.ws_misc[7].as<int>((long)npole + 2L * o * v + 8);
  int* eRo = ex;
  int* eRv = ex + o;
  int* eOV = ex + npole;
  int* eVO = eOV + (long)o * v;   // the same exponents as [a][i] (greater part: inner i contiguous)
  unsigned long long* nrm = reinterpret_cast<unsigned long long*>(
      h.ws_red.as<double>(4096) + 4000);   // 3 slots
  if (F16) {
    AGF2_HIP(hipMemsetAsync(ex, 0x80, ((long)npole + (long)o * v) * sizeof(int), st));
    AGF2_HIP(hipMemsetAsync(nrm, 0, 3 * sizeof(unsigned long long), st));
  }
  // Summation order of the Q index: ascending Frobenius norm of the DF
  // slices, so float32 accumulation adds small contributions before large
  // ones (a relabelling of the summed index; the result is unchanged in exact
  // arithmetic).
  int* perm = h.ws_misc[6].as<int>(Qs);
  {
    double* sq = h.ws_misc[5].as<double>(Q);
    hipLaunchKernelGGL(slice_norm_kernel, dim3(Q), dim3(256), 0, st, L, (long)N * N, sq);
    AGF2_CHECK_LAUNCH();
    std::vector<double> hsq(Q);
    AGF2_HIP(hipMemcpyAsync(hsq.data(), sq, Q * sizeof(double), hipMemcpyDeviceToHost, st));
    AGF2_HIP(hipStreamSynchronize(st));
    std::vector<int> hp(Qs, -1);
    std::vector<int> idx(Q);
    for (int q = 0; q < Q; ++q) idx[q] = q;
    std::stable_sort(idx.begin(), idx.end(), [&](int a, int b) { return hsq[a] < hsq[b]; });
    // padding first (zeros), then ascending slices
    for (int q = 0; q < Q; ++q) hp[Qs - Q + q] = idx[q];
    AGF2_HIP(hipMemcpyAsync(perm, hp.data(), Qs * sizeof(int), hipMemcpyHostToDevice, st));
    AGF2_HIP(hipStreamSynchronize(st));
  }
  {
    const double* ut = poles_are_identity(h, N, npole, u) ? nullptr : u;
    ProfScope ps(h, "moments.transform",
                 ut ? 2.0 * Q * (double)N * N * npole + 2.0 * Q * (double)N * o * v : 0.0,
                 8.0 * ((double)Q * N * N + (double)npole * N * Q + (double)o * v * Q));
    // float64 staging in chunks of poles (<= ~4 GiB each), a multiple of 64
    // poles where possible (whole GEMM tiles)
    const long per_pole = (long)N * Qp;
    long pcl = std::max<long>(1, std::min<long>(npole, (1L << 29) / per_pole));
    if (pcl > 64 && pcl < npole) pcl = pcl / 64 * 64;
    const int pc = (int)pcl;
    double* T = h.ws_moments[3].as<double>((long)pc * per_pole + (long)o * pc * Qp);
    double* Tov = T + (long)pc * per_pole;
    for (int p0 = 0; p0 < o; p0 += pc) {
      const int np = std::min(pc, o - p0);
      pole_transform_f64(N, Q, Qp, L, ut, npole, p0, np, T, st);
      // rows (p, x); one exponent per pole p
      if (F16) row_stats(T, per_pole, Qp, np, N, Q, 1, 0, eRo + p0, nrm + 0, st);
      split_rows<F16>(T, per_pole, Qp, np, N, perm, Rxo_h + (long)p0 * N * KS,
                      Rxo_l + (long)p0 * N * KS, N, 1, (long)o * N * KS, Qs,
                      F16 ? eRo + p0 : nullptr, 1, 0, st);
    }
    for (int a0 = 0; a0 < v; a0 += pc) {
      const int na = std::min(pc, v - a0);
      pole_transform_f64(N, Q, Qp, L, ut, npole, o + a0, na, T, st);
      if (F16) row_stats(T, per_pole, Qp, na, N, Q, 1, 0, eRv + a0, nrm + 1, st);
      split_rows<F16>(T, per_pole, Qp, na, N, perm, Rxv_h + (long)a0 * N * KS,
                      Rxv_l + (long)a0 * N * KS, N, 1, (long)v * N * KS, Qs,
                      F16 ? eRv + a0 : nullptr, 1, 0, st);
      // Lov[i][a][Q] = sum_x u[x][i] Lxv[a][x][Q] for this chunk of a
      lov_transform_f64(N, Q, Qp, ut, npole, o, na, T, Tov, st);
      // rows (i, a); one exponent per row, stored at i * v + a
      if (F16) row_stats(Tov, (long)na * Qp, Qp, o, na, Q, v, 1, eOV + a0, nrm + 2, st);
      split_rows<F16>(Tov, (long)na * Qp, Qp, o, na, perm, Rov_h + (long)a0 * KS,
                      Rov_l + (long)a0 * KS, v, 1, (long)o * v * KS, Qs,
                      F16 ? eOV + a0 : nullptr, v, 1, st);
      split_rows<F16>(Tov, (long)na * Qp, Qp, o, na, perm, Rvo_h + (long)a0 * o * KS,
                      Rvo_l + (long)a0 * o * KS, 1, o, (long)o * v * KS, Qs,
                      F16 ? eOV + a0 : nullptr, v, 1, st);
    }
  }
  PartScales lesser, greater;
  if (F16) {
    if ((long)o * v > 0) {
      hipLaunchKernelGGL(transpose_int_kernel, dim3((unsigned)std::min<long>(((long)o * v + 255) / 256, 4096)),
                         dim3(256), 0, st, o, v, eOV, eVO);
      AGF2_CHECK_LAUNCH();
    }
    // Cauchy-Schwarz: |(xp|qc)| <= |R[p][x]| |S[q][c]| (Q-space norms), so
    // |Z|, |wZ| <= sqrt(6) * max|R| max|S| (* max|w|)
    unsigned long long hn[3];
    AGF2_HIP(hipMemcpyAsync(hn, nrm, sizeof hn, hipMemcpyDeviceToHost, st));
    std::vector<double> he(npole);
    AGF2_HIP(hipMemcpyAsync(he.data(), e, npole * sizeof(double), hipMemcpyDeviceToHost, st));
    AGF2_HIP(hipStreamSynchronize(st));
    double n2[3];
    for (int k = 0; k < 3; ++k) std::memcpy(&n2[k], &hn[k], sizeof(double));
    double eo_max = 0.0, ev_max = 0.0;
    for (int i = 0; i < o; ++i) eo_max = std::max(eo_max, std::fabs(he[i]));
    for (int a = o; a < npole; ++a) ev_max = std::max(ev_max, std::fabs(he[a]));
    auto make = [&](const int* eR, const int* eS, double nR2, double wmax, long sEp, long sEc) {
      PartScales sc;
      sc.eR = eR; sc.eS = eS; sc.sEp = sEp; sc.sEc = sEc;
      const double zb = std::sqrt(6.0 * nR2 * n2[2]);
      const double wb = zb * wmax;
      const int fZ = EMAX - exponent_above(zb), fW = EMAX - exponent_above(wb);
      sc.zscale = std::ldexp(1.0f, fZ);
      sc.wscale = std::ldexp(1.0f, fW);
      sc.u0scale = std::ldexp(1.0, -2 * fZ);
      sc.u1scale = std::ldexp(1.0, -fZ - fW);
      return sc;
    };
    lesser = make(eRo, eOV, n2[0], 2.0 * eo_max + ev_max, (long)v, 1L);
    greater = make(eRv, eVO, n2[1], 2.0 * ev_max + eo_max, (long)o, 1L);
  }
  // strides in rows of the K-blocked arrays
  moments_part_split<F16>(h, N, Q, Qs, Rxo_h, Rxo_l, N, 1, (long)o * N * KS, Rov_h, Rov_l, v,
                          1, (long)o * v * KS, e, o, e + o, v, lesser, m0o, m1o);
  moments_part_split<F16>(h, N, Q, Qs, Rxv_h, Rxv_l, N, 1, (long)v * N * KS, Rvo_h, Rvo_l, o,
                          1, (long)o * v * KS, e + o, v, e, o, greater, m0v, m1v);
}

void build_moments_split(Handle& h, int N, int Q, const double* L, int npole, int nocc,
                         const double* e, const double* u, double* m0o, double* m1o,
                         double* m0v, double* m1v, bool fp16) {
  if (fp16)
    build_split<true>(h, N, Q, L, npole, nocc, e, u, m0o, m1o, m0v, m1v);
  else
    build_split<false>(h, N, Q, L, npole, nocc, e, u, m0o, m1o, m0v, m1v);
}

}  // namespace agf2
