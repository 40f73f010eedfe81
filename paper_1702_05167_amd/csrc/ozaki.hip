// Complex double-double block products on the integer matrix cores.
//
// The double-double solve forms every block product of Algorithms 1 and 2
// (multipliers, Schur updates, extraction and lesser-channel products) as
// D = (-1)^negate op(A) op(B) + beta C with ~106-bit operands.  Instead of
// emulating double-double arithmetic on the FP64 vector units, each operand is
// rewritten as a sum of S signed 8-bit slices times a power of two per row (of
// op(A)) or per column (of op(B)) -- the error-free splitting of Ozaki, Ogita,
// Oishi and Rump (Numer. Algorithms 59, 2012) in the integer form of Ootomo,
// Ozaki and Yokota (IJHPCA 2024):
//
//   x / 2^e_r = sum_{s=0}^{S-1} d_s 2^(-6-7s) + rem,   d_s in [-64, 64],
//   |rem| <= 2^(-6-7(S-1)-1),   e_r = exponent with max_k (|Re x_rk| + |Im x_rk|) < 2^e_r.
//
// A product of slices s and t weighs 2^(-12-7(s+t)); sums over k of int8 x int8
// products are exact in int32 (v_mfma_i32_16x16x64_i8), and only the pairs with
// s + t <= S - 1 are formed (S (S + 1) / 2 of S^2).  Complex products use three
// real products (Gauss: T1 = Ar Br, T2 = Ai Bi, T3 = (Ar + Ai)(Br + Bi)); their
// integer sums combine exactly into Re = T1 - T2 and Im = T3 - T1 - T2, and the
// S weighted partial sums of each are added in double-double only at the end.
//
// Error (S = 16): the dropped pairs (weights 2^-124 and below, at most 64^2 K
// per pair and slice) and the slice remainders (2^-113 of the row scale) give,
// for each output, at most about K 2^-106 * 2^(e_i + f_j) <= K 2^-104 max_k
// |op(A)_ik| max_k |op(B)_kj| (row scale of op(A) times column scale of op(B)),
// plus the double-double rounding of the final sums and of beta C (2^-104
// relative); with digits of random sign it is typically far smaller.  Unlike an emulated double-double product, the
// bound is relative to the largest entries of the row and column, not to
// sum_k |a_ik| |b_kj|.
//
// Layout: the slices of one operand are planes [3][S][Rp][Kp] of int8 (operand
// part 0 = Re, 1 = Im, 2 = Re + Im; rows padded to the 32-row tile, K padded to
// 64 with zeros), row scales int32 [Rp].  The GEMM kernel stages the slices of
// a 32 x 32 output tile through LDS with direct global-to-LDS loads laid out in
// the matrix-core operand order, and each of its four waves holds the 3 x S
// integer accumulators of one 16 x 16 block.
#include <hip/hip_runtime.h>

#include "dd.h"
#include "kern.h"

namespace hsc {

namespace {

typedef int v4i __attribute__((ext_vector_type(4)));

constexpr int OZ_TILE = 32;   // rows and columns of the output tile of one workgroup
constexpr int OZ_KC = 64;     // k depth of one matrix-core step (v_mfma_i32_16x16x64_i8)

// ---------------------------------------------------------------------------------------------
// splitting: rows [r0, r0 + 64) of one operand per workgroup

// element (r, k) of the operand as stored: X[r * ldr + k * ldk]; zero outside R x K
__device__ inline zdd oz_elem(const OzSplitJob& jb, int r, int k) {
  if (r >= jb.R || k >= jb.K) return zdd_zero();
  return jb.X[(int64_t)r * jb.ldr + (int64_t)k * jb.ldk];
}

// digits of x (|x| < 2^6 after scaling, x exact as a double-double) into d[0..S)
template <int S>
__device__ inline void oz_digits(dd y, int* d) {
#pragma clang fp contract(off)
#pragma unroll
  for (int s = 0; s < S; ++s) {
    const double q = rint(y.hi);
    d[s] = (int)q;
    const dd r = two_sum(y.hi - q, y.lo);   // y.hi - q is exact (|y.hi - q| <= 1/2)
    y = dd{r.hi * 128.0, r.lo * 128.0};
  }
}

template <int S, bool KFAST>
__global__ __launch_bounds__(256) void k_oz_split(const OzSplitJob* __restrict__ jobs,
                                                  const int32_t* __restrict__ blk_job) {
  const OzSplitJob& jb = jobs[blk_job[blockIdx.x]];
  const int r0 = (blockIdx.x - jb.blk_off) * 64;
  const int t = threadIdx.x;
  __shared__ double red[4][64];
  __shared__ int ex[64];
  // pass 1: row scales (max over k of |Re| + |Im|, hi and lo parts)
  {
    const int rr = t & 63, kq = t >> 6;
    double m = 0.0;
    for (int k = kq; k < jb.K; k += 4) {
      const zdd v = oz_elem(jb, r0 + rr, k);
      m = fmax(m, (fabs(v.re.hi) + fabs(v.re.lo)) + (fabs(v.im.hi) + fabs(v.im.lo)));
    }
    red[kq][rr] = m;
    __syncthreads();
    if (t < 64) {
      const double mx = fmax(fmax(red[0][t], red[1][t]), fmax(red[2][t], red[3][t]));
      int e = 0;
      if (mx > 0.0 && isfinite(mx)) (void)frexp(mx, &e);   // mx < 2^e
      ex[t] = e;
      if (r0 + t < jb.Rp) jb.ex[r0 + t] = e;
    }
    __syncthreads();
  }
  // pass 2: digits, four consecutive k per thread, packed into one int32 per (part, slice)
  const int nq = jb.Kp / 4;
  const int64_t plane = (int64_t)jb.Rp * jb.Kp;
  for (int q = t; q < 64 * nq; q += 256) {
    const int rr = KFAST ? q / nq : q % 64;
    const int kq = KFAST ? q % nq : q / 64;
    const int r = r0 + rr;
    if (r >= jb.Rp) continue;
    const int e = ex[rr];
    uint32_t packed[3][S];
#pragma unroll
    for (int p = 0; p < 3; ++p)
#pragma unroll
      for (int s = 0; s < S; ++s) packed[p][s] = 0;
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const zdd v = oz_elem(jb, r, 4 * kq + u);
      // scale by 2^(6 - e): exact
      const int sh = 6 - e;
      const dd xr{ldexp(v.re.hi, sh), ldexp(v.re.lo, sh)};
      const dd xi{ldexp(v.im.hi, sh), ldexp(v.im.lo, sh)};
      const dd xs = dd_add(xr, xi);
      int d[S];
      oz_digits<S>(xr, d);
#pragma unroll
      for (int s = 0; s < S; ++s) packed[0][s] |= (uint32_t)(d[s] & 0xff) << (8 * u);
      oz_digits<S>(xi, d);
#pragma unroll
      for (int s = 0; s < S; ++s) packed[1][s] |= (uint32_t)(d[s] & 0xff) << (8 * u);
      oz_digits<S>(xs, d);
#pragma unroll
      for (int s = 0; s < S; ++s) packed[2][s] |= (uint32_t)(d[s] & 0xff) << (8 * u);
    }
    uint32_t* out = reinterpret_cast<uint32_t*>(jb.out);
#pragma unroll
    for (int p = 0; p < 3; ++p)
#pragma unroll
      for (int s = 0; s < S; ++s)
        out[((p * S + s) * plane + (int64_t)r * jb.Kp) / 4 + kq] = packed[p][s];
  }
}

// ---------------------------------------------------------------------------------------------
// products of the slices

typedef __attribute__((address_space(3))) void* lds_ptr;

// stage the slices of operand part p, k step kc: 4 * S fragments of 1 KB (A rows m0 + [0, 16),
// A rows m0 + [16, 32), B columns n0 + [0, 16), n0 + [16, 32)); fragment (g, s) holds, at byte
// 16 l + b, slice s of row 16 (g & 1) + (l & 15), k = 64 kc + 16 (l >> 4) + b -- the order in which
// v_mfma_i32_16x16x64_i8 takes its operands (lane l: row l & 15, k group l >> 4)
template <int S>
__device__ inline void oz_stage(const GemmProbOZ& pr, v4i* buf, int m0, int n0, int p, int kc, int w, int lane) {
  const int64_t planeA = (int64_t)pr.Mp * pr.Kp, planeB = (int64_t)pr.Np * pr.Kp;
  const int64_t koff = (int64_t)kc * OZ_KC + 16 * (lane >> 4);
#pragma unroll
  for (int q = 0; q < S; ++q) {
    const int f = w * S + q;           // fragment index, 4 S per stage, S per wave
    const int g = f / S, s = f % S;
    const int8_t* src;
    if (g < 2)
      src = pr.A8 + (p * S + s) * planeA + (int64_t)(m0 + 16 * g + (lane & 15)) * pr.Kp + koff;
    else
      src = pr.B8 + (p * S + s) * planeB + (int64_t)(n0 + 16 * (g - 2) + (lane & 15)) * pr.Kp + koff;
    __builtin_amdgcn_global_load_lds(src, (lds_ptr)(buf + (size_t)f * 64), 16, 0, 0);
  }
}

template <int S>
__device__ inline void oz_mma(const v4i* __restrict__ buf, int wm, int wn, int lane, v4i (&acc)[S]) {
  v4i b[S];
#pragma unroll
  for (int t = 0; t < S; ++t) b[t] = buf[(size_t)((2 + wn) * S + t) * 64 + lane];
#pragma unroll
  for (int s = 0; s < S; ++s) {
    const v4i a = buf[(size_t)(wm * S + s) * 64 + lane];
#pragma unroll
    for (int t = 0; t < S - s; ++t) acc[s + t] = __builtin_amdgcn_mfma_i32_16x16x64_i8(a, b[t], acc[s + t], 0, 0, 0);
  }
}

// sum_d x_d 2^(-12 - 7 d) in double-double, smallest terms first (every term is exact)
template <int S>
__device__ inline dd oz_sum(const int (&x)[S]) {
  dd v{0.0, 0.0};
#pragma unroll
  for (int d = S - 1; d >= 0; --d) v = dd_add(v, dd{ldexp((double)x[d], -12 - 7 * d), 0.0});
  return v;
}

template <int S>
__global__ __launch_bounds__(256) void k_oz_gemm(const GemmProbOZ* __restrict__ probs,
                                                 const int32_t* __restrict__ tile_prob, int total_tiles, int negate,
                                                 int beta) {
  __shared__ v4i lds[2][4 * S * 64];
  const int per = (total_tiles + 7) >> 3;
  const int tile = (blockIdx.x & 7) * per + (blockIdx.x >> 3);   // XCD-aware order
  if (tile >= total_tiles) return;
  const GemmProbOZ& pr = probs[tile_prob[tile]];
  const int local = tile - pr.tile_off;
  const int m0 = (local / pr.tiles_n) * OZ_TILE, n0 = (local % pr.tiles_n) * OZ_TILE;
  const int t = threadIdx.x, lane = t & 63, w = t >> 6;
  const int wm = w >> 1, wn = w & 1;

  v4i acc0[S], acc1[S], acc2[S];
#pragma unroll
  for (int d = 0; d < S; ++d) acc0[d] = acc1[d] = acc2[d] = v4i{0, 0, 0, 0};

  const int nkc = pr.Kp / OZ_KC;
  if (nkc > 0) oz_stage<S>(pr, lds[0], m0, n0, 0, 0, w, lane);
  for (int kc = 0; kc < nkc; ++kc) {
#pragma unroll
    for (int p = 0; p < 3; ++p) {
      const int it = 3 * kc + p;
      __builtin_amdgcn_s_waitcnt(0);   // this wave's loads into the current buffer are in LDS
      __syncthreads();                 // ... and every wave's; the other buffer is no longer read
      if (p < 2) oz_stage<S>(pr, lds[(it + 1) & 1], m0, n0, p + 1, kc, w, lane);
      else if (kc + 1 < nkc) oz_stage<S>(pr, lds[(it + 1) & 1], m0, n0, 0, kc + 1, w, lane);
      const v4i* buf = lds[it & 1];
      if (p == 0) oz_mma<S>(buf, wm, wn, lane, acc0);
      else if (p == 1) oz_mma<S>(buf, wm, wn, lane, acc1);
      else oz_mma<S>(buf, wm, wn, lane, acc2);
    }
  }

  // epilogue: lane l, register r holds output row 4 (l >> 4) + r, column l & 15 of the wave's block
  const int col = n0 + 16 * wn + (lane & 15);
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    const int row = m0 + 16 * wm + 4 * (lane >> 4) + r;
    if (row >= pr.M || col >= pr.N) continue;
    int xr[S], xi[S];
#pragma unroll
    for (int d = 0; d < S; ++d) {
      const int t1 = acc0[d][r], t2 = acc1[d][r], t3 = acc2[d][r];
      xr[d] = t1 - t2;
      xi[d] = t3 - t1 - t2;
    }
    const int sc = pr.ea[row] + pr.eb[col];
    dd re = oz_sum<S>(xr), im = oz_sum<S>(xi);
    re = dd{ldexp(re.hi, sc), ldexp(re.lo, sc)};
    im = dd{ldexp(im.hi, sc), ldexp(im.lo, sc)};
    zdd o{re, im};
    if (negate) o = zdd_neg(o);
    if (beta) o = zdd_add(o, pr.C[(int64_t)row * pr.ldc + col]);
    pr.D[(int64_t)row * pr.ldd + col] = o;
    if (pr.D64) pr.D64[(int64_t)row * pr.ldd64 + col] = zdd_round(o);
  }
}

}  // namespace

void launch_oz_split(hipStream_t st, const OzSplitJob* jobs, const int32_t* blk_job, int total_blocks, int kfast) {
  if (total_blocks <= 0) return;
  if (kfast)
    hipLaunchKernelGGL((k_oz_split<kOzSlices, true>), dim3(total_blocks), dim3(256), 0, st, jobs, blk_job);
  else
    hipLaunchKernelGGL((k_oz_split<kOzSlices, false>), dim3(total_blocks), dim3(256), 0, st, jobs, blk_job);
}

void launch_oz_gemm(hipStream_t st, const GemmProbOZ* probs, const int32_t* tile_prob, int total_tiles, int negate,
                    int beta) {
  if (total_tiles <= 0) return;
  const dim3 g(((total_tiles + 7) / 8) * 8), b(256);
  hipLaunchKernelGGL((k_oz_gemm<kOzSlices>), g, b, 0, st, probs, tile_prob, total_tiles, negate, beta);
}

}  // namespace hsc
