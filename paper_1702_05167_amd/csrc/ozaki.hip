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
// Error: per k and real part product, the dropped pairs (S - 1 of weight
// 2^(-12-7S), fewer below, each at most 64^2) and the slice remainders
// (2^-7S of the scale) miss at most about (S + 1) 2^-7S of 2^(e_i + f_j);
// Im = T3 - T1 - T2 sums three such products, so each output is off by at most
// about 3 (S + 1) K 2^-7S * 2^(e_i + f_j), i.e. K 2^-104 (S = 16) or K 2^-97
// (S = 15) times max_k (|Re| + |Im|) of row i of op(A) times the same of
// column j of op(B) (2^e <= twice that maximum), plus the double-double
// rounding of the final sums and of beta C (2^-104 relative); with digits of
// random sign it is typically far smaller.  Unlike an emulated double-double
// product, the bound is relative to the largest entries of the row and column,
// not to sum_k |a_ik| |b_kj|: entries far below their row's largest keep fewer
// bits, which is why 16 slices are the default (15 save 16 of 136 pairs).
//
// Layout: the slices of one operand are 3 x S planes of int8 (operand part
// 0 = Re, 1 = Im, 2 = Re + Im; rows padded to the 32-row tile, K padded to 64
// with zeros), each stored as 1 KB fragments of 16 rows x 64 k in the order in
// which the matrix cores take an operand; row scales int32 [Rp].  The GEMM
// kernel stages the fragments of a 32 x 32 output tile into LDS with direct
// global-to-LDS loads (one contiguous kilobyte per wave instruction), and each
// of its four waves holds the 3 x S integer accumulators of one 16 x 16 block.
#include <hip/hip_runtime.h>

#include "dd.h"
#include "kern.h"

namespace hsc {

namespace {

typedef int v4i __attribute__((ext_vector_type(4)));

constexpr int OZ_TILE = 32;   // rows and columns of the output tile of one workgroup
constexpr int OZ_KC = 64;     // k depth of one matrix-core step (v_mfma_i32_16x16x64_i8)
constexpr int OZ_GROUP = 8;   // tile rows per group of the tile order

// ---------------------------------------------------------------------------------------------
// splitting, in two launches: row scales (64 rows per workgroup), then digits (tiles of 64 rows x
// 32 k per workgroup, written through LDS in the operand order of the matrix cores)

// element (r, k) of the operand as stored: X[r * ldr + k * ldk]; zero outside R x K
__device__ inline zdd oz_elem(const OzSplitJob& jb, int r, int k) {
  if (r >= jb.R || k >= jb.K) return zdd_zero();
  return jb.X[(int64_t)r * jb.ldr + (int64_t)k * jb.ldk];
}

__device__ inline double oz_mag(const zdd& v) {
  return (fabs(v.re.hi) + fabs(v.re.lo)) + (fabs(v.im.hi) + fabs(v.im.lo));
}

// ex[r] = e with max_k (|Re| + |Im|) of row r < 2^e (0 for a zero row)
__global__ __launch_bounds__(256) void k_oz_scale(const OzSplitJob* __restrict__ jobs,
                                                  const int32_t* __restrict__ blk_job) {
  const OzSplitJob& jb = jobs[blk_job[blockIdx.x]];
  const int r0 = (blockIdx.x - jb.blk_off) * 64;
  const int t = threadIdx.x, lane = t & 63, w = t >> 6;
  __shared__ double red[4][64];
  if (jb.ldk == 1) {
    // k contiguous: one wave per row, lanes along k
    for (int rr = w; rr < 64; rr += 4) {
      double m = 0.0;
      for (int k = lane; k < jb.K; k += 64) m = fmax(m, oz_mag(oz_elem(jb, r0 + rr, k)));
#pragma unroll
      for (int off = 32; off > 0; off >>= 1) m = fmax(m, __shfl_xor(m, off, 64));
      if (lane == 0) red[0][rr] = m;
    }
    __syncthreads();
    if (t < 64) {
      int e = 0;
      const double mx = red[0][t];
      if (mx > 0.0 && isfinite(mx)) (void)frexp(mx, &e);
      if (r0 + t < jb.Rp) jb.ex[r0 + t] = e;
    }
  } else {
    // rows contiguous (or general strides): lanes along rows, four k phases
    double m = 0.0;
    for (int k = w; k < jb.K; k += 4) m = fmax(m, oz_mag(oz_elem(jb, r0 + lane, k)));
    red[w][lane] = m;
    __syncthreads();
    if (t < 64) {
      int e = 0;
      const double mx = fmax(fmax(red[0][t], red[1][t]), fmax(red[2][t], red[3][t]));
      if (mx > 0.0 && isfinite(mx)) (void)frexp(mx, &e);
      if (r0 + t < jb.Rp) jb.ex[r0 + t] = e;
    }
  }
}

// S digits of y (a double-double with |y.lo| <= ulp(y.hi) / 2 and |y| < 2^6 + 2^-40), digit s of
// weight 2^(-7 s), in blocks of m <= 4 digits b0 .. b0 + m - 1: the block's integer
// v = rint(y.hi 2^(7 (b0 + m - 1))) (|v| <= 2^27 + 1, exact in int32), and the remainder
// y - v 2^(-7 (b0 + m - 1)) (exact: y.hi minus v's value is a multiple of ulp(y.hi), so at least
// twice |y.lo| unless zero) feeds the next block (|remainder| <= (2^6 + 2^-20) 2^(-7 (b0 + m))).  The
// remainder keeps the input's scale and the powers of two move into the constants: every step is
// the one at the block's own scale times an exact power of two, so the digits are the same.  v
// splits into balanced base-128 digits in integer arithmetic, the lower ones in [-64, 63] and the
// leading one in [-64, 64] (|v| <= 64.5 2^(7 (m - 1)) after the lower digits are taken off).  Four
// FP64 steps per block instead of one per digit.  Digit s goes to byte `shift` of word[s].
template <int S>
__device__ inline void oz_digits(dd y, uint32_t* word, int shift) {
#pragma clang fp contract(off)
#pragma unroll
  for (int b0 = 0; b0 < S; b0 += 4) {
    const int m = S - b0 < 4 ? S - b0 : 4;
    const double up = ldexp(1.0, 7 * (b0 + m - 1)), down = ldexp(1.0, -7 * (b0 + m - 1));
    const double q = rint(y.hi * up);
    int v = (int)q;
    const double t = fma(-q, down, y.hi);   // exact (representable), as the unfused difference is
    const double hi = t + y.lo;
    const double lo = y.lo - (hi - t);
    y = dd{hi, lo};
#pragma unroll
    for (int j = m - 1; j >= 1; --j) {
      const int d = ((v + 64) & 127) - 64;
      word[b0 + j] |= (uint32_t)(d & 0xff) << shift;
      v = (v - d) >> 7;
    }
    word[b0] |= (uint32_t)(v & 0xff) << shift;
  }
}

// Tile (64 rows from r0, 32 k from k0) of one job: each thread holds two quads of four
// consecutive k; for each operand part in turn it packs each quad's digits into one word per
// slice, the words go to LDS in the order of the global planes, and the block writes them out 16
// bytes per thread.  Global layout of a part / slice plane: fragments of 16 rows x 64 k (1 KB),
// row blocks of the plane in order, each row block's 64-k steps in order; inside a fragment,
// byte 16 l + b holds row l & 15, k = 16 (l >> 4) + b (the operand order of
// v_mfma_i32_16x16x64_i8).
template <int S>
__global__ __launch_bounds__(256) void k_oz_digits(const OzSplitJob* __restrict__ jobs,
                                                   const int32_t* __restrict__ tile_job) {
  // [slice][row block of 16][lane 0..31 of the half fragment][4 words] of one part
  __shared__ uint32_t lw[S * 4 * 32 * 4];
  const OzSplitJob& jb = jobs[tile_job[blockIdx.x]];
  const int local = blockIdx.x - jb.tile_off;
  const int nk = jb.Kp / 32;
  const int r0 = (local / nk) * 64, k0 = (local % nk) * 32;
  const int t = threadIdx.x;
  const bool kfast = jb.ldk == 1;
  // the thread's elements, scaled by 2^(6 - e) (exact) and normalised: quad j, element u
  dd xr[2][4], xi[2][4];
  int rr[2], kq[2];
#pragma unroll
  for (int j = 0; j < 2; ++j) {
    rr[j] = kfast ? (t >> 3) + 32 * j : (t & 63);
    kq[j] = kfast ? (t & 7) : (t >> 6) + 4 * j;
    const int r = r0 + rr[j];
    const int sh = 6 - (r < jb.Rp ? jb.ex[r] : 0);
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const zdd v = oz_elem(jb, r, k0 + 4 * kq[j] + u);
      const dd nr = two_sum(v.re.hi, v.re.lo), ni = two_sum(v.im.hi, v.im.lo);
      xr[j][u] = dd{ldexp(nr.hi, sh), ldexp(nr.lo, sh)};
      xi[j][u] = dd{ldexp(ni.hi, sh), ldexp(ni.lo, sh)};
    }
  }
  const int rbs = jb.Rp / 16, kcs = jb.Kp / 64, half = (k0 >> 5) & 1, kc = k0 >> 6;
  const uint4* src = reinterpret_cast<const uint4*>(lw);
#pragma unroll
  for (int p = 0; p < 3; ++p) {
#pragma unroll
    for (int j = 0; j < 2; ++j) {
      uint32_t wd[S];
#pragma unroll
      for (int q = 0; q < S; ++q) wd[q] = 0;
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const dd x = p == 0 ? xr[j][u] : p == 1 ? xi[j][u] : dd_add(xr[j][u], xi[j][u]);
        oz_digits<S>(x, wd, 8 * u);
      }
      // word (k % 16) / 4 of half-fragment lane (row & 15) + 16 ((k % 32) / 16), row block row / 16
      const int kk = 4 * kq[j];
      const int l = (rr[j] & 15) + 16 * (kk >> 4), wq = (kk & 15) >> 2, rb = rr[j] >> 4;
#pragma unroll
      for (int q = 0; q < S; ++q) lw[(((q * 4 + rb) * 32 + l) * 4) + wq] = wd[q];
    }
    __syncthreads();
    // write out: 16 bytes per (slice, row block, half-fragment lane)
    for (int c = t; c < S * 4 * 32; c += 256) {
      const int l = c & 31, rb = (c >> 5) & 3, q = c >> 7;
      const int rbg = r0 / 16 + rb;
      if (rbg >= rbs) continue;
      uint4* dst = reinterpret_cast<uint4*>(jb.out + (((int64_t)(p * S + q) * rbs + rbg) * kcs + kc) * 1024) +
                   32 * half + l;
      *dst = src[c];
    }
    __syncthreads();
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
  const int kcs = pr.Kp / OZ_KC;
  const int rbsA = pr.Mp / 16, rbsB = pr.Np / 16;
#pragma unroll
  for (int q = 0; q < S; ++q) {
    const int f = w * S + q;           // fragment index, 4 S per stage, S per wave
    const int g = f / S, s = f % S;
    const int8_t* src;
    if (g < 2)
      src = pr.A8 + (((int64_t)(p * S + s) * rbsA + m0 / 16 + g) * kcs + kc) * 1024 + 16 * lane;
    else
      src = pr.B8 + (((int64_t)(p * S + s) * rbsB + n0 / 16 + (g - 2)) * kcs + kc) * 1024 + 16 * lane;
    __builtin_amdgcn_global_load_lds(src, (lds_ptr)(buf + (size_t)f * 64), 16, 0, 0);
  }
}

// the slice pairs s + t <= S - 1 of one staged operand part: the B slices in two halves held in
// registers, the A slices read from LDS for each half
template <int S>
__device__ inline void oz_mma(const v4i* __restrict__ buf, int wm, int wn, int lane, v4i (&acc)[S]) {
  constexpr int H = (S + 1) / 2;
#pragma unroll
  for (int h = 0; h < 2; ++h) {
    v4i b[H];
#pragma unroll
    for (int t = 0; t < H; ++t)
      if (h * H + t < S) b[t] = buf[(size_t)((2 + wn) * S + h * H + t) * 64 + lane];
#pragma unroll
    for (int s = 0; s < S - h * H; ++s) {
      const v4i a = buf[(size_t)(wm * S + s) * 64 + lane];
#pragma unroll
      for (int t = 0; t < H; ++t)
        if (h * H + t < S && s + h * H + t <= S - 1)
          acc[s + h * H + t] = __builtin_amdgcn_mfma_i32_16x16x64_i8(a, b[t], acc[s + h * H + t], 0, 0, 0);
    }
  }
}

// sum_d x_d 2^(-12 - 7 d) in double-double.  |x_d| < 2^31, so up to four consecutive weights summed
// as x_d 2^21 + x_(d+1) 2^14 + x_(d+2) 2^7 + x_(d+3) stay integers below 2^53: each group is formed
// exactly in FP64 by exact fused multiply-adds, scaled exactly by its power of two, and the groups
// are added in double-double, smallest first
template <int S>
__device__ inline dd oz_sum(const int (&x)[S]) {
  dd v{0.0, 0.0};
#pragma unroll
  for (int g1 = S - 1; g1 >= 0; g1 -= 4) {
    const int g0 = g1 >= 3 ? g1 - 3 : 0;
    double acc = (double)x[g0];
#pragma unroll
    for (int d = g0 + 1; d <= g1; ++d) acc = fma(acc, 128.0, (double)x[d]);
    v = dd_add(v, dd{ldexp(acc, -12 - 7 * g1), 0.0});
  }
  return v;
}

// One 32 x 32 output tile per workgroup of four waves (a 16 x 16 block each), one staged operand
// part (64 KB) at a time and two workgroups per CU, so that one computes while the other waits for
// its loads.  The parts run one after the other with two accumulator sets: T1 = Re A Re B into acc0,
// T2 = Im A Im B into acc1; then acc0 = T1 - T2 (the real part) and acc1 = -(T1 + T2), onto which
// part 2 adds T3 = (Re A + Im A)(Re B + Im B) (the imaginary part); integer sums are exact.
template <int S>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(2, 2))) void k_oz_gemm(
    const GemmProbOZ* __restrict__ probs, const int32_t* __restrict__ tile_prob, int total_tiles, int negate,
    int beta) {
  __shared__ v4i lds[4 * S * 64];
  const int per = (total_tiles + 7) >> 3;
  const int tile = (blockIdx.x & 7) * per + (blockIdx.x >> 3);   // XCD-aware order
  if (tile >= total_tiles) return;
  const GemmProbOZ& pr = probs[tile_prob[tile]];
  const int local = tile - pr.tile_off;
  // tiles of a problem in groups of OZ_GROUP tile rows, column by column inside a group: the tiles
  // an XCD runs at once share a few row and column blocks of the slices in its L2
  const int tm = pr.Mp / OZ_TILE, tn = pr.tiles_n;
  const int grp = local / (OZ_GROUP * tn), idx = local % (OZ_GROUP * tn);
  const int rows = min(OZ_GROUP, tm - grp * OZ_GROUP);
  const int m0 = (grp * OZ_GROUP + idx % rows) * OZ_TILE, n0 = (idx / rows) * OZ_TILE;
  // the wave index is uniform across the wave: kept in scalar registers, so that every address but
  // the lane's own offset is scalar arithmetic
  const int t = threadIdx.x, lane = t & 63, w = __builtin_amdgcn_readfirstlane(t >> 6);
  const int wm = w >> 1, wn = w & 1;

  v4i acc0[S], acc1[S];
#pragma unroll
  for (int d = 0; d < S; ++d) acc0[d] = acc1[d] = v4i{0, 0, 0, 0};

  const int nkc = pr.Kp / OZ_KC;
#pragma unroll
  for (int p = 0; p < 3; ++p) {
    if (p == 2) {
#pragma unroll
      for (int d = 0; d < S; ++d) {
        const v4i t1 = acc0[d], t2 = acc1[d];
        acc0[d] = t1 - t2;
        acc1[d] = -(t1 + t2);
      }
    }
    for (int kc = 0; kc < nkc; ++kc) {
      oz_stage<S>(pr, lds, m0, n0, p, kc, w, lane);
      __builtin_amdgcn_s_waitcnt(0);   // this wave's loads are in LDS
      __syncthreads();                 // ... and every wave's
      if (p == 0) oz_mma<S>(lds, wm, wn, lane, acc0);
      else oz_mma<S>(lds, wm, wn, lane, acc1);
      __syncthreads();                 // every wave has read the stage before the next overwrites it
    }
  }
  if (nkc == 0) {
#pragma unroll
    for (int d = 0; d < S; ++d) acc0[d] = acc1[d] = v4i{0, 0, 0, 0};
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
      xr[d] = acc0[d][r];
      xi[d] = acc1[d][r];
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

// ---------------------------------------------------------------------------------------------
// the allocation-free product: descriptors and maps of one problem written on the device

// jobs A, B at ws (an array of two), the product at ws + 256, maps at ws + 1024: scale blocks (ba of job 0,
// bb of job 1), digit tiles (ta, tb), product tiles (all 0); slices and exponents at the given
// offsets
__global__ __launch_bounds__(256) void k_oz_setup(char* ws, OzSplitJob ja, OzSplitJob jb, GemmProbOZ p, int ba,
                                                  int bb, int ta, int tb, int tiles) {
  if (threadIdx.x == 0) {
    *reinterpret_cast<OzSplitJob*>(ws) = ja;
    reinterpret_cast<OzSplitJob*>(ws)[1] = jb;
    *reinterpret_cast<GemmProbOZ*>(ws + 256) = p;
  }
  int32_t* m = reinterpret_cast<int32_t*>(ws + 1024);
  const int n = ba + bb + ta + tb + tiles;
  for (int i = threadIdx.x; i < n; i += 256) {
    int v = 0;
    if (i < ba + bb) v = i < ba ? 0 : 1;
    else if (i < ba + bb + ta + tb) v = i - ba - bb < ta ? 0 : 1;
    m[i] = v;
  }
}

// Scratch of the allocation-free product: one array per device, allocated with the code object;
// host code uses the address obtained from hipGetSymbolAddress, never the array's name.
__device__ __align__(256) char scratch[kOzNoAllocScratch];

}  // namespace

// Device address of `scratch` on the current device (looked up once per device by the caller and
// kept); nullptr if the runtime cannot resolve it.
void* oz_noalloc_scratch_address() {
  void* ptr = nullptr;
  if (hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)) != hipSuccess) {
    (void)hipGetLastError();
    return nullptr;
  }
  return ptr;
}

size_t oz_noalloc_bytes(int M, int N, int K) {
  const size_t Mp = (M + 31) / 32 * 32, Np = (N + 31) / 32 * 32, Kp = (K + 63) / 64 * 64;
  const size_t ba = (Mp + 63) / 64, bb = (Np + 63) / 64, ta = ba * (Kp / 32), tb = bb * (Kp / 32);
  const size_t tiles = (Mp / 32) * (Np / 32);
  auto pad = [](size_t v) { return (v + 255) / 256 * 256; };
  return pad(1024 + 4 * (ba + bb + ta + tb + tiles)) + pad(3 * kOzSlices * Mp * Kp) + pad(3 * kOzSlices * Np * Kp) +
         pad(4 * Mp) + pad(4 * Np);
}

int launch_oz_gemm_noalloc(hipStream_t st, char* ws, int opA, int opB, int M, int N, int K, int negate,
                           const void* A, int lda, const void* B, int ldb, int beta, const void* C, int ldc, void* D,
                           int ldd) {
  const int Mp = (M + 31) / 32 * 32, Np = (N + 31) / 32 * 32, Kp = (K + 63) / 64 * 64;
  const int ba = (Mp + 63) / 64, bb = (Np + 63) / 64, ta = ba * (Kp / 32), tb = bb * (Kp / 32);
  const int tiles = (Mp / 32) * (Np / 32);
  auto pad = [](size_t v) { return (v + 255) / 256 * 256; };
  const size_t o_a8 = pad(1024 + 4 * (size_t)(ba + bb + ta + tb + tiles));
  const size_t o_b8 = o_a8 + pad((size_t)3 * kOzSlices * Mp * Kp);
  const size_t o_ea = o_b8 + pad((size_t)3 * kOzSlices * Np * Kp);
  const size_t o_eb = o_ea + pad(4 * (size_t)Mp);
  OzSplitJob ja{}, jb{};
  ja.X = (const zdd*)A; ja.R = M; ja.K = K; ja.Rp = Mp; ja.Kp = Kp;
  if (opA == 0) { ja.ldr = lda; ja.ldk = 1; } else { ja.ldr = 1; ja.ldk = lda; }
  ja.out = (int8_t*)(ws + o_a8); ja.ex = (int32_t*)(ws + o_ea);
  ja.blk_off = 0; ja.tile_off = 0;
  jb.X = (const zdd*)B; jb.R = N; jb.K = K; jb.Rp = Np; jb.Kp = Kp;
  if (opB == 0) { jb.ldr = 1; jb.ldk = ldb; } else { jb.ldr = ldb; jb.ldk = 1; }
  jb.out = (int8_t*)(ws + o_b8); jb.ex = (int32_t*)(ws + o_eb);
  jb.blk_off = ba; jb.tile_off = ta;
  GemmProbOZ p{};
  p.A8 = ja.out; p.B8 = jb.out; p.ea = ja.ex; p.eb = jb.ex;
  p.C = (const zdd*)C; p.D = (zdd*)D; p.D64 = nullptr;
  p.M = M; p.N = N; p.Mp = Mp; p.Np = Np; p.Kp = Kp; p.ldc = ldc; p.ldd = ldd; p.ldd64 = 0;
  p.tiles_n = Np / 32; p.tile_off = 0;
  hipLaunchKernelGGL(k_oz_setup, dim3(1), dim3(256), 0, st, ws, ja, jb, p, ba, bb, ta, tb, tiles);
  const int32_t* m = reinterpret_cast<const int32_t*>(ws + 1024);
  launch_oz_split(st, kOzSlices, reinterpret_cast<const OzSplitJob*>(ws), m, ba + bb, m + ba + bb, ta + tb);
  launch_oz_gemm(st, kOzSlices, reinterpret_cast<const GemmProbOZ*>(ws + 256), m + ba + bb + ta + tb, tiles, negate,
                 beta);
  return hipGetLastError() == hipSuccess ? 0 : -1;
}

void launch_oz_split(hipStream_t st, int slices, const OzSplitJob* jobs, const int32_t* blk_job, int total_blocks,
                     const int32_t* tile_job, int total_tiles) {
  if (total_blocks <= 0) return;
  hipLaunchKernelGGL(k_oz_scale, dim3(total_blocks), dim3(256), 0, st, jobs, blk_job);
  if (total_tiles <= 0) return;   // none when K = 0
  if (slices == 15) hipLaunchKernelGGL((k_oz_digits<15>), dim3(total_tiles), dim3(256), 0, st, jobs, tile_job);
  else hipLaunchKernelGGL((k_oz_digits<16>), dim3(total_tiles), dim3(256), 0, st, jobs, tile_job);
}

void launch_oz_gemm(hipStream_t st, int slices, const GemmProbOZ* probs, const int32_t* tile_prob, int total_tiles,
                    int negate, int beta) {
  if (total_tiles <= 0) return;
  const dim3 g(((total_tiles + 7) / 8) * 8), b(256);
  if (slices == 15) hipLaunchKernelGGL((k_oz_gemm<15>), g, b, 0, st, probs, tile_prob, total_tiles, negate, beta);
  else hipLaunchKernelGGL((k_oz_gemm<16>), g, b, 0, st, probs, tile_prob, total_tiles, negate, beta);
}

}  // namespace hsc
