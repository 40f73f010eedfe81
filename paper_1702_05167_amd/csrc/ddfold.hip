// Algorithms 1 and 2 in double-double: frontal assembly, blocked Gauss-Jordan
// inversion of the pivot blocks, the multiplier / Schur-update products, and the
// row kernels of the extraction (gathers, lesser-channel seeds, diagonals).  Same
// structure as the FP64 kernels (inverse.hip, gemm.hip, kernels.hip); every value
// is a complex double-double (dd.h) and the products run on the FP64 vector units
// (on this chip their peak equals the FP64 matrix cores', and double-double needs
// the error-free fused multiply-add).
#include <hip/hip_runtime.h>

#include "dd.h"
#include "kern.h"

namespace hsc {

namespace {

constexpr int RB = 256;

// ---------------------------------------------------------------------------------------------
// assembly: F[a][b] = sum_children U_k[invrel_k[a]][invrel_k[b]] + (-H)[a][b] + delta_ab (z - Sigma_a - U_a)
__global__ __launch_bounds__(RB) void k_dd_assemble(const RowJob* __restrict__ jobs,
                                                    const int32_t* __restrict__ row_job,
                                                    const EnergyScalars* __restrict__ es) {
  const int g = blockIdx.x;
  const RowJob& jb = jobs[row_job[g]];
  const int a = g - jb.row_off;
  const int cols = jb.cols;
  const ChildRef* kids = reinterpret_cast<const ChildRef*>(jb.p0);
  const FrontSparse* fs = reinterpret_cast<const FrontSparse*>(jb.p1);
  const int nk = jb.aux0, n = jb.aux1, nL = jb.aux2, nR = jb.aux3;
  __shared__ int s_col[64];
  __shared__ double2 s_val[64];
  const int q0 = fs->ptr[a], q1 = fs->ptr[a + 1];
  const int nq = min(q1 - q0, 64);
  if (threadIdx.x < nq) {
    s_col[threadIdx.x] = fs->col[q0 + threadIdx.x];
    s_val[threadIdx.x] = fs->val[q0 + threadIdx.x];
  }
  __syncthreads();
  zdd diag_add = zdd_zero();
  if (a < n) {   // z - Sigma_a, as the exact sum of the two FP64 inputs
    const EnergyScalars& s = es[jb.e];
    if (a < nL + nR) {
      const double2 sg = a < nL ? s.sig[0] : s.sig[1];
      diag_add = zdd{two_sum(s.z.x, -sg.x), two_sum(s.z.y, -sg.y)};
    } else {
      diag_add = zdd_from(s.z);
    }
    if (fs->pot) diag_add.re = dd_add(diag_add.re, dd{-fs->pot[a], 0.0});
  }
  zdd* out = reinterpret_cast<zdd*>(jb.dst) + (int64_t)a * jb.ldd;
  // whole-face contact cluster: minus its dense self-energy block (rows and columns < nface)
  const int nface = jb.aux4;
  const double2* dsig = a < nface ? reinterpret_cast<const double2*>(jb.p2) : nullptr;
  for (int b = threadIdx.x; b < cols; b += RB) {
    zdd v = zdd_zero();
    for (int k = 0; k < nk; ++k) {
      const int ia = kids[k].invrel[a];
      if (ia < 0) continue;
      const int ib = kids[k].invrel[b];
      if (ib < 0) continue;
      v = zdd_add(v, reinterpret_cast<const zdd*>(kids[k].U)[(int64_t)ia * kids[k].ldU + ib]);
    }
    for (int q = 0; q < nq; ++q)
      if (s_col[q] == b) v = zdd_add(v, zdd_from(s_val[q]));
    for (int q = q0 + 64; q < q1; ++q)
      if (fs->col[q] == b) v = zdd_add(v, zdd_from(fs->val[q]));
    if (b == a) v = zdd_add(v, diag_add);
    if (dsig && b < nface) {
      const double2 sv = dsig[(int64_t)a * nface + b];
      v = zdd_sub(v, zdd_from(sv));
    }
    out[b] = v;
  }
}

// ---------------------------------------------------------------------------------------------
// Gauss-Jordan panel in double-double (same algorithm as k_inv_panel)
constexpr int PT = 512;

template <int RPT, int NB>
__global__ __launch_bounds__(PT) __attribute__((amdgpu_waves_per_eu(1, 2))) void k_dd_inv_panel(
    const InvJobDD* __restrict__ jobs, int k0, int nbw, int32_t* __restrict__ status) {
  const InvJobDD jb = jobs[blockIdx.x];
  const int n = jb.n;
  if (k0 >= n) return;
  const int nb = min(nbw, n - k0);
  const int t = threadIdx.x, lane = t & 63, w = t >> 6;
  __shared__ double red_v[PT / 64];
  __shared__ int red_i[PT / 64];
  __shared__ zdd rowp[NB], rowc[NB], srow[NB];
  __shared__ int bad;
  if (t == 0) bad = 0;

  zdd P[RPT][NB];
#pragma unroll
  for (int q = 0; q < RPT; ++q) {
    const int r = t + q * PT;
#pragma unroll
    for (int j = 0; j < NB; ++j) P[q][j] = (r < n && j < nb) ? jb.X[(int64_t)r * jb.ld + k0 + j] : zdd_zero();
  }
  __syncthreads();

#pragma unroll
  for (int j = 0; j < NB; ++j) {
    if (j < nb) {
      const int c = k0 + j;
      double bv = -1.0;
      int bi = n;
#pragma unroll
      for (int q = 0; q < RPT; ++q) {
        const int r = t + q * PT;
        if (r >= c && r < n) {
          const double v = zdd_cabs1(P[q][j]);
          if (v > bv) { bv = v; bi = r; }
        }
      }
#pragma unroll
      for (int off = 32; off > 0; off >>= 1) {
        const double ov = __shfl_xor(bv, off, 64);
        const int oi = __shfl_xor(bi, off, 64);
        if (ov > bv || (ov == bv && oi < bi)) { bv = ov; bi = oi; }
      }
      if (lane == 0) { red_v[w] = bv; red_i[w] = bi; }
      __syncthreads();
      double pv = red_v[0];
      int prow = red_i[0];
#pragma unroll
      for (int k = 1; k < PT / 64; ++k) {
        const double ov = red_v[k];
        const int oi = red_i[k];
        if (ov > pv || (ov == pv && oi < prow)) { pv = ov; prow = oi; }
      }
      if (prow >= n) { prow = c; pv = 0.0; }
#pragma unroll
      for (int q = 0; q < RPT; ++q) {
        const int r = t + q * PT;
        if (r == prow) {
#pragma unroll
          for (int jj = 0; jj < NB; ++jj) rowp[jj] = P[q][jj];
        }
        if (r == c && prow != c) {
#pragma unroll
          for (int jj = 0; jj < NB; ++jj) rowc[jj] = P[q][jj];
        }
      }
      if (t == 0) jb.piv[c] = prow;
      __syncthreads();
      if (t < NB) {
        const zdd pivv = rowp[j];
        const zdd inv = zdd_rcp(pivv);
        srow[t] = (t == j) ? inv : zdd_mul(rowp[t], inv);
        if (t == 0 && (!(pv > 0.0) || !isfinite(pivv.re.hi) || !isfinite(pivv.im.hi))) bad = 1;
      }
      __syncthreads();
      const zdd inv = srow[j];
#pragma unroll
      for (int q = 0; q < RPT; ++q) {
        const int r = t + q * PT;
        if (r == c) {
#pragma unroll
          for (int jj = 0; jj < NB; ++jj) P[q][jj] = srow[jj];
        } else {
          if (r == prow) {
#pragma unroll
            for (int jj = 0; jj < NB; ++jj) P[q][jj] = rowc[jj];
          }
          const zdd m = P[q][j];
#pragma unroll
          for (int jj = 0; jj < NB; ++jj)
            if (jj != j) P[q][jj] = zdd_sub(P[q][jj], zdd_mul(m, srow[jj]));
          P[q][j] = zdd_neg(zdd_mul(m, inv));
        }
      }
    }
  }
#pragma unroll
  for (int q = 0; q < RPT; ++q) {
    const int r = t + q * PT;
    if (r < n) {
#pragma unroll
      for (int j = 0; j < NB; ++j) {
        if (j < nb) {
          jb.X[(int64_t)r * jb.ld + k0 + j] = P[q][j];
          zdd v = P[q][j];
          if (r == k0 + j) v.re = dd_add(v.re, dd_from(-1.0));
          jb.T[(int64_t)r * nb + j] = v;
        }
      }
    }
  }
  __syncthreads();
  if (t == 0 && bad && status) atomicMin(&status[jb.e], (int32_t)HSC_E_SINGULAR);
}

__global__ __launch_bounds__(256) void k_dd_inv_swap(const InvJobDD* __restrict__ jobs, int k0, int nbw,
                                                     int chunks) {
  const InvJobDD jb = jobs[blockIdx.x / chunks];
  const int n = jb.n;
  if (k0 >= n) return;
  const int nb = min(nbw, n - k0);
  const int col = (blockIdx.x % chunks) * 256 + threadIdx.x;
  if (col >= n) return;
  const bool in_panel = col >= k0 && col < k0 + nb;
  if (!in_panel) {
    for (int j = 0; j < nb; ++j) {
      const int c = k0 + j, p = jb.piv[c];
      if (p != c) {
        zdd* a = jb.X + (int64_t)c * jb.ld + col;
        zdd* b = jb.X + (int64_t)p * jb.ld + col;
        const zdd x = *a;
        *a = *b;
        *b = x;
      }
    }
  }
  for (int j = 0; j < nb; ++j)
    jb.R[(int64_t)j * n + col] = in_panel ? zdd_zero() : jb.X[(int64_t)(k0 + j) * jb.ld + col];
}

// After the panels of a super-panel [s0, s0 + ws) (two-level Gauss-Jordan, as inverse.hip):
//   U[r][c] = X[r][s0 + c] - (r == s0 + c)   (n x ws, row stride W; the T workspace)
//   R[c][j] = X[s0 + c][j]                     (ws x n; the R workspace)
__global__ __launch_bounds__(64) void k_dd_inv_super_u(const InvJobDD* __restrict__ jobs, int s0, int W, int chunks) {
  const InvJobDD jb = jobs[blockIdx.x / chunks];
  const int n = jb.n;
  if (s0 >= n) return;
  const int ws = min(W, n - s0);
  const int c = threadIdx.x;
  const int r0 = (blockIdx.x % chunks) * 16;
  if (c >= ws) return;
  for (int r = r0; r < min(n, r0 + 16); ++r) {
    zdd v = jb.X[(int64_t)r * jb.ld + s0 + c];
    if (r == s0 + c) v.re = dd_add(v.re, dd_from(-1.0));
    jb.T[(int64_t)r * W + c] = v;
  }
}

__global__ __launch_bounds__(256) void k_dd_inv_super_r(const InvJobDD* __restrict__ jobs, int s0, int W, int chunks) {
  const InvJobDD jb = jobs[blockIdx.x / (W * chunks)];
  const int n = jb.n;
  if (s0 >= n) return;
  const int ws = min(W, n - s0);
  const int rem = blockIdx.x % (W * chunks);
  const int c = rem / chunks;
  const int j = (rem % chunks) * 256 + threadIdx.x;
  if (c >= ws || j >= n) return;
  jb.R[(int64_t)c * n + j] = jb.X[(int64_t)(s0 + c) * jb.ld + j];
}

__global__ __launch_bounds__(256) void k_dd_inv_unscramble(const InvJobDD* __restrict__ jobs, int rows_per_block,
                                                           int chunks) {
  extern __shared__ int idx[];
  const InvJobDD jb = jobs[blockIdx.x / chunks];
  const int n = jb.n;
  const int r0 = (blockIdx.x % chunks) * rows_per_block;
  if (r0 >= n) return;
  for (int j = threadIdx.x; j < n; j += blockDim.x) idx[j] = j;
  __syncthreads();
  if (threadIdx.x == 0) {
    for (int c = n - 1; c >= 0; --c) {
      const int p = jb.piv[c];
      const int a = idx[c];
      idx[c] = idx[p];
      idx[p] = a;
    }
  }
  __syncthreads();
  const int r1 = min(n, r0 + rows_per_block);
  for (int r = r0; r < r1; ++r)
    for (int j = threadIdx.x; j < n; j += blockDim.x) {
      const zdd v = jb.X[(int64_t)r * jb.ld + idx[j]];
      jb.Y[(int64_t)r * jb.ldy + j] = v;
      jb.Y64[(int64_t)r * jb.ldy64 + j] = zdd_round(v);
    }
}

// ---------------------------------------------------------------------------------------------
// grouped complex double-double GEMM: 256 threads as 16 x 16, each with an RM x RN block of outputs
// (tile BM x BN = 16 RM x 16 RN: 32x32, 64x32 or 64x64), three real products per complex
// multiply-add (Gauss; the sums re + im of both operands are formed once, when a tile is staged),
// lazily accumulated (dd.h: ddacc) and renormalised after every 8-deep k step.
//   OPA 0: A'(m,k) = A[m*lda + k];  OPA 1: A'(m,k) = A[k*lda + m]
//   OPB 0: B'(k,n) = B[k*ldb + n];  OPB 1: B'(k,n) = B[n*ldb + k]
constexpr int DK = 8;
constexpr int kDDConfigs = 3;
constexpr int kDDRM[kDDConfigs] = {2, 4, 4}, kDDRN[kDDConfigs] = {2, 2, 4};

template <int OPA, int OPB, int RM, int RN>
__global__ __launch_bounds__(256) void k_dd_gemm(const GemmProbDD* __restrict__ probs,
                                                 const int32_t* __restrict__ tile_prob, int total_tiles, int negate,
                                                 int beta) {
  constexpr int BM = 16 * RM, BN = 16 * RN;
  __shared__ zdd As[DK][BM + 1];
  __shared__ zdd Bs[DK][BN + 1];
  __shared__ dd Ass[DK][BM + 1];   // re + im of each staged element (the third product of the Gauss form)
  __shared__ dd Bss[DK][BN + 1];
  const int per = (total_tiles + 7) >> 3;
  const int tile = (blockIdx.x & 7) * per + (blockIdx.x >> 3);
  if (tile >= total_tiles) return;
  const GemmProbDD& pr = probs[tile_prob[tile]];
  const int local = tile - pr.tile_off;
  const int m0 = (local / pr.tiles_n) * BM, n0 = (local % pr.tiles_n) * BN;
  const int M = pr.M, N = pr.N, K = pr.K;
  const int t = threadIdx.x;
  const int tm = (t / 16) * RM, tn = (t % 16) * RN;   // this thread's RM x RN block
  // three real products per complex multiply-add (Gauss): t1 = sum ar br, t2 = sum ai bi,
  // t3 = sum (ar + ai)(br + bi); re = t1 - t2, im = t3 - t1 - t2
  ddacc t1[RM][RN], t2[RM][RN], t3[RM][RN];
#pragma unroll
  for (int i = 0; i < RM; ++i)
#pragma unroll
    for (int j = 0; j < RN; ++j) t1[i][j] = t2[i][j] = t3[i][j] = ddacc{0.0, 0.0};
  for (int k0 = 0; k0 < K; k0 += DK) {
    // stage A' (BM x DK) and B' (DK x BN), RM / 2 and RN / 2 elements per thread
#pragma unroll
    for (int u = 0; u < RM / 2; ++u) {
      const int idx = t + u * 256;
      const int mm = OPA == 0 ? idx / DK : idx % BM;
      const int kk = OPA == 0 ? idx % DK : idx / BM;
      const int gm = m0 + mm, gk = k0 + kk;
      zdd v = zdd_zero();
      if (gm < M && gk < K) v = OPA == 0 ? pr.A[(int64_t)gm * pr.lda + gk] : pr.A[(int64_t)gk * pr.lda + gm];
      As[kk][mm] = v;
      Ass[kk][mm] = dd_add(v.re, v.im);
    }
#pragma unroll
    for (int u = 0; u < RN / 2; ++u) {
      const int idx = t + u * 256;
      const int bk = OPB == 0 ? idx / BN : idx % DK;
      const int bn = OPB == 0 ? idx % BN : idx / DK;
      const int gbk = k0 + bk, gbn = n0 + bn;
      zdd v = zdd_zero();
      if (gbk < K && gbn < N) v = OPB == 0 ? pr.B[(int64_t)gbk * pr.ldb + gbn] : pr.B[(int64_t)gbn * pr.ldb + gbk];
      Bs[bk][bn] = v;
      Bss[bk][bn] = dd_add(v.re, v.im);
    }
    __syncthreads();
#pragma unroll
    for (int kk = 0; kk < DK; ++kk) {
      zdd a[RM], b[RN];
      dd sa[RM], sb[RN];
#pragma unroll
      for (int i = 0; i < RM; ++i) { a[i] = As[kk][tm + i]; sa[i] = Ass[kk][tm + i]; }
#pragma unroll
      for (int j = 0; j < RN; ++j) { b[j] = Bs[kk][tn + j]; sb[j] = Bss[kk][tn + j]; }
#pragma unroll
      for (int i = 0; i < RM; ++i)
#pragma unroll
        for (int j = 0; j < RN; ++j) {
          ddacc_add_prod(t1[i][j], a[i].re, b[j].re);
          ddacc_add_prod(t2[i][j], a[i].im, b[j].im);
          ddacc_add_prod(t3[i][j], sa[i], sb[j]);
        }
    }
#pragma unroll
    for (int i = 0; i < RM; ++i)
#pragma unroll
      for (int j = 0; j < RN; ++j) {
        ddacc_renorm(t1[i][j]);
        ddacc_renorm(t2[i][j]);
        ddacc_renorm(t3[i][j]);
      }
    __syncthreads();
  }
#pragma unroll
  for (int i = 0; i < RM; ++i)
#pragma unroll
    for (int j = 0; j < RN; ++j) {
      const int row = m0 + tm + i, col = n0 + tn + j;
      if (row < M && col < N) {
        const dd v1 = two_sum(t1[i][j].hi, t1[i][j].lo), v2 = two_sum(t2[i][j].hi, t2[i][j].lo);
        const dd v3 = two_sum(t3[i][j].hi, t3[i][j].lo);
        const zdd v{dd_sub(v1, v2), dd_sub(dd_sub(v3, v1), v2)};
        zdd o = negate ? zdd_neg(v) : v;
        if (beta) o = zdd_add(o, pr.C[(int64_t)row * pr.ldc + col]);
        pr.D[(int64_t)row * pr.ldd + col] = o;
        if (pr.D64) pr.D64[(int64_t)row * pr.ldd64 + col] = zdd_round(o);
      }
    }
}

template <int RM, int RN>
void dd_gemm_dispatch(hipStream_t st, int opA, int opB, const GemmProbDD* probs, const int32_t* tile_prob,
                      int total_tiles, int negate, int beta) {
  const dim3 g(((total_tiles + 7) / 8) * 8), b(256);
  if (opA == 0 && opB == 0)
    hipLaunchKernelGGL((k_dd_gemm<0, 0, RM, RN>), g, b, 0, st, probs, tile_prob, total_tiles, negate, beta);
  else if (opA == 1 && opB == 0)
    hipLaunchKernelGGL((k_dd_gemm<1, 0, RM, RN>), g, b, 0, st, probs, tile_prob, total_tiles, negate, beta);
  else if (opA == 0)
    hipLaunchKernelGGL((k_dd_gemm<0, 1, RM, RN>), g, b, 0, st, probs, tile_prob, total_tiles, negate, beta);
  else
    hipLaunchKernelGGL((k_dd_gemm<1, 1, RM, RN>), g, b, 0, st, probs, tile_prob, total_tiles, negate, beta);
}

// ---------------------------------------------------------------------------------------------
// extraction row kernels (Algorithm 2 and the lesser channels), as in kernels.hip

// dst[r][c] = op(trans ? src[cmap[c]][rmap[r]] : src[rmap[r]][cmap[c]]);  op 1 = -conj
template <int TRANS, int OP>
__global__ __launch_bounds__(RB) void k_dd_gather(const RowJob* __restrict__ jobs,
                                                  const int32_t* __restrict__ row_job) {
  const int g = blockIdx.x;
  const RowJob& jb = jobs[row_job[g]];
  const int r = g - jb.row_off;
  const int rr = jb.rmap ? jb.rmap[r] : r;
  const int32_t* __restrict__ cmap = jb.cmap;
  const zdd* __restrict__ src = reinterpret_cast<const zdd*>(jb.src);
  zdd* __restrict__ out = reinterpret_cast<zdd*>(jb.dst) + (int64_t)r * jb.ldd;
  for (int c = threadIdx.x; c < jb.cols; c += RB) {
    const int cc = cmap ? cmap[c] : c;
    zdd v = TRANS ? src[(int64_t)cc * jb.lds + rr] : src[(int64_t)rr * jb.lds + cc];
    if (OP == 1) v.re = dd_neg(v.re);
    out[c] = v;
  }
}

// NF[rr][b] = sum_children U_k[invrel_k[a(rr)]][b] + seed(rr, b), the seed i * w * conj(G[a][b])
// on the contact rows (argument layout of k_assemble_n)
__global__ __launch_bounds__(RB) void k_dd_assemble_n(const RowJob* __restrict__ jobs,
                                                      const int32_t* __restrict__ row_job,
                                                      const EnergyScalars* __restrict__ es, int channel) {
  const int g = blockIdx.x;
  const RowJob& jb = jobs[row_job[g]];
  const int rr = g - jb.row_off;
  const ChildRef* kids = reinterpret_cast<const ChildRef*>(jb.p0);
  const int nk = jb.aux0, r = jb.aux1, row0 = jb.aux2, n = jb.aux3, nL = jb.aux4, nR = jb.aux5;
  const int a = rr < r ? row0 + rr : n + (rr - r);
  // whole-face contact: p1 holds Gamma G (same leading dimension) and w is the occupation alone
  const zdd* gam_g = reinterpret_cast<const zdd*>(jb.p1);
  double w = 0.0;
  if (rr < r && a < nL + nR)
    w = gam_g ? channel_occ(es[jb.e], channel, a < nL ? 0 : 1) : channel_weight(es[jb.e], channel, a < nL ? 0 : 1);
  const zdd* grow = (gam_g ? gam_g : reinterpret_cast<const zdd*>(jb.src)) + (int64_t)a * jb.lds;
  zdd* out = reinterpret_cast<zdd*>(jb.dst) + (int64_t)rr * jb.ldd;
  for (int b = threadIdx.x; b < jb.cols; b += RB) {
    zdd v = zdd_zero();
    for (int k = 0; k < nk; ++k) {
      const int ia = kids[k].invrel[a];
      if (ia >= 0) v = zdd_add(v, reinterpret_cast<const zdd*>(kids[k].U)[(int64_t)ia * kids[k].ldU + b]);
    }
    if (w != 0.0) {
      const zdd gv = grow[b];
      v.re = dd_add(v.re, dd_mul(dd_from(w), gv.im));
      v.im = dd_add(v.im, dd_mul(dd_from(w), gv.re));
    }
    out[b] = v;
  }
}

__device__ __forceinline__ double shfl_xor_d(double v, int off) { return __shfl_xor(v, off, 64); }

// diagonal outputs, one wave per row, rounded to complex128 at the store (modes of k_diag)
template <int MODE>
__global__ __launch_bounds__(RB) void k_dd_diag(const RowJob* __restrict__ jobs, const int32_t* __restrict__ row_job,
                                                int total_rows, int out_kind, void* out, int64_t out_stride,
                                                int e_base, int nvalid) {
  const int g = blockIdx.x * (RB / 64) + (threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  if (g >= total_rows) return;
  const RowJob& jb = jobs[row_job[g]];
  const int k = g - jb.row_off;
  if (jb.e >= nvalid) return;
  const zdd* src = reinterpret_cast<const zdd*>(jb.src);
  zdd v = zdd_zero();
  if (MODE == DIAG_SEP) {
    v = src[(int64_t)k * jb.lds + k];
  } else {
    const int f = jb.aux0;
    const zdd* psi = reinterpret_cast<const zdd*>(jb.p0) + (int64_t)k * f;
    const zdd* x = src + (int64_t)k * jb.lds;
    zdd acc = zdd_zero();
    for (int j = lane; j < f; j += 64) {
      zdd y = x[j];
      if (MODE == DIAG_LEAF_P) y.im = dd_neg(y.im);
      acc = zdd_fma(acc, psi[j], y);
    }
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
      zdd o;
      o.re.hi = shfl_xor_d(acc.re.hi, off);
      o.re.lo = shfl_xor_d(acc.re.lo, off);
      o.im.hi = shfl_xor_d(acc.im.hi, off);
      o.im.lo = shfl_xor_d(acc.im.lo, off);
      acc = zdd_add(acc, o);
    }
    const zdd* base = reinterpret_cast<const zdd*>(jb.p1);
    const zdd d = base ? base[(int64_t)k * jb.aux1 + k] : zdd_zero();
    v = MODE == DIAG_LEAF_P ? zdd_sub(d, acc) : zdd_add(d, acc);
  }
  if (lane != 0) return;
  const double2 r = zdd_round(v);
  const int64_t site = reinterpret_cast<const int64_t*>(jb.p2)[k];
  const int64_t idx = (int64_t)(e_base + jb.e) * out_stride + site;
  if (out_kind == OUT_COMPLEX) reinterpret_cast<double2*>(out)[idx] = r;
  else reinterpret_cast<double*>(out)[idx] = r.y;
}

}  // namespace

int dd_gemm_configs() { return kDDConfigs; }
int dd_gemm_tile_m(int config) { return 16 * kDDRM[config]; }
int dd_gemm_tile_n(int config) { return 16 * kDDRN[config]; }
int dd_inv_nb(int max_n) { return max_n <= 1024 ? 8 : max_n <= 2048 ? 4 : 2; }

void launch_dd_gemm(hipStream_t st, int opA, int opB, int config, const GemmProbDD* probs,
                    const int32_t* tile_prob, int total_tiles, int negate, int beta) {
  if (total_tiles <= 0) return;
  if (config == 1) dd_gemm_dispatch<4, 2>(st, opA, opB, probs, tile_prob, total_tiles, negate, beta);
  else if (config == 2) dd_gemm_dispatch<4, 4>(st, opA, opB, probs, tile_prob, total_tiles, negate, beta);
  else dd_gemm_dispatch<2, 2>(st, opA, opB, probs, tile_prob, total_tiles, negate, beta);
}

void launch_dd_gather(hipStream_t st, const RowJob* jobs, const int32_t* row_job, int total_rows, int trans, int op) {
  if (total_rows <= 0) return;
  const dim3 g(total_rows), b(RB);
  if (trans == 0 && op == 0) hipLaunchKernelGGL((k_dd_gather<0, 0>), g, b, 0, st, jobs, row_job);
  else if (trans == 1 && op == 0) hipLaunchKernelGGL((k_dd_gather<1, 0>), g, b, 0, st, jobs, row_job);
  else if (trans == 0) hipLaunchKernelGGL((k_dd_gather<0, 1>), g, b, 0, st, jobs, row_job);
  else hipLaunchKernelGGL((k_dd_gather<1, 1>), g, b, 0, st, jobs, row_job);
}

void launch_dd_assemble_n(hipStream_t st, const RowJob* jobs, const int32_t* row_job, int total_rows,
                          const EnergyScalars* es, int channel) {
  if (total_rows <= 0) return;
  hipLaunchKernelGGL(k_dd_assemble_n, dim3(total_rows), dim3(RB), 0, st, jobs, row_job, es, channel);
}

void launch_dd_diag(hipStream_t st, const RowJob* jobs, const int32_t* row_job, int total_rows, int mode,
                    int out_kind, void* out, int64_t out_stride, int e_base, int nvalid) {
  if (total_rows <= 0) return;
  const dim3 grid((total_rows + RB / 64 - 1) / (RB / 64)), block(RB);
  if (mode == DIAG_SEP)
    hipLaunchKernelGGL(k_dd_diag<DIAG_SEP>, grid, block, 0, st, jobs, row_job, total_rows, out_kind, out,
                       out_stride, e_base, nvalid);
  else if (mode == DIAG_LEAF_G)
    hipLaunchKernelGGL(k_dd_diag<DIAG_LEAF_G>, grid, block, 0, st, jobs, row_job, total_rows, out_kind, out,
                       out_stride, e_base, nvalid);
  else
    hipLaunchKernelGGL(k_dd_diag<DIAG_LEAF_P>, grid, block, 0, st, jobs, row_job, total_rows, out_kind, out,
                       out_stride, e_base, nvalid);
}

void launch_dd_assemble(hipStream_t st, const RowJob* jobs, const int32_t* row_job, int total_rows,
                        const EnergyScalars* es) {
  if (total_rows <= 0) return;
  hipLaunchKernelGGL(k_dd_assemble, dim3(total_rows), dim3(RB), 0, st, jobs, row_job, es);
}

void launch_dd_inv_panel(hipStream_t st, const InvJobDD* jobs, int njobs, int k0, int nb, int max_n,
                         int32_t* status) {
  if (njobs <= 0 || max_n > 8 * PT) return;
  dim3 g(njobs), b(PT);
  if (max_n <= 512) hipLaunchKernelGGL((k_dd_inv_panel<1, 8>), g, b, 0, st, jobs, k0, nb, status);
  else if (max_n <= 1024) hipLaunchKernelGGL((k_dd_inv_panel<2, 8>), g, b, 0, st, jobs, k0, nb, status);
  else if (max_n <= 2048) hipLaunchKernelGGL((k_dd_inv_panel<4, 4>), g, b, 0, st, jobs, k0, nb, status);
  else hipLaunchKernelGGL((k_dd_inv_panel<8, 2>), g, b, 0, st, jobs, k0, nb, status);
}

void launch_dd_inv_swap(hipStream_t st, const InvJobDD* jobs, int njobs, int k0, int nb, int max_n) {
  if (njobs <= 0) return;
  const int chunks = (max_n + 255) / 256;
  hipLaunchKernelGGL(k_dd_inv_swap, dim3(njobs * chunks), dim3(256), 0, st, jobs, k0, nb, chunks);
}

void launch_dd_inv_super(hipStream_t st, const InvJobDD* jobs, int njobs, int s0, int W, int max_n) {
  if (njobs <= 0 || W <= 0 || W > 64) return;
  const int cu = (max_n + 15) / 16, cr = (max_n + 255) / 256;
  hipLaunchKernelGGL(k_dd_inv_super_u, dim3(njobs * cu), dim3(64), 0, st, jobs, s0, W, cu);
  hipLaunchKernelGGL(k_dd_inv_super_r, dim3(njobs * W * cr), dim3(256), 0, st, jobs, s0, W, cr);
}

void launch_dd_inv_unscramble(hipStream_t st, const InvJobDD* jobs, int njobs, int max_n) {
  if (njobs <= 0) return;
  const int rpb = 16;
  const int chunks = (max_n + rpb - 1) / rpb;
  hipLaunchKernelGGL(k_dd_inv_unscramble, dim3(njobs * chunks), dim3(256), max_n * sizeof(int), st, jobs, rpb,
                     chunks);
}

}  // namespace hsc
