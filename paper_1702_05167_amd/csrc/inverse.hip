// Batched blocked Gauss-Jordan inversion with partial pivoting (complex128).
//
// Algorithm 1 inverts each (Schur-complemented) diagonal block A_ii; pivoting
// is within the block only (the cluster order itself is fixed by the tree).
// Blocked in-place Gauss-Jordan: for each panel of NB columns,
//   1. panel kernel: unblocked Gauss-Jordan on the n x NB panel held in
//      registers (one row per thread slot), row interchanges by partial
//      pivoting; the panel then holds T[:, panel] (the transformation applied
//      to the identity columns), and T - I goes to a workspace;
//   2. swap kernel: the same row interchanges on the other columns, and a copy
//      of the (swapped) pivot rows with the panel columns zeroed;
//   3. a grouped GEMM: X += (T - I) * R  (rank-NB update of every row).
// Finally the column permutation (interchanges undone in reverse order) is
// applied while copying into the output buffer.
//
// Two levels: panels of NB columns are grouped into super-panels of W = 4 NB.
// Inside a super-panel the rank-NB updates touch only its W columns; the W
// eliminations together act on every other column as X += U R with
// U = (the super-panel columns) - I at the pivot rows and R = the W pivot
// rows before the update (interchanges are applied to all columns at once:
// each panel pivots only among rows not yet used, so they commute with the
// deferred update).  One rank-W update replaces W/NB rank-NB updates and
// reads / writes X a quarter as often.
#include <hip/hip_runtime.h>

#include "kern.h"

namespace hsc {

namespace {

constexpr int PT = 512;   // threads per panel block

__device__ inline double cabs1(double2 a) { return fabs(a.x) + fabs(a.y); }
__device__ inline double2 cmul(double2 a, double2 b) {
  return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
__device__ inline double2 crcp(double2 a) {
  // 1/a with scaling to avoid overflow in |a|^2
  double s = fmax(fabs(a.x), fabs(a.y));
  if (s == 0.0) return make_double2(0.0, 0.0);
  double ar = a.x / s, ai = a.y / s;
  double d = ar * ar + ai * ai;
  return make_double2(ar / (d * s), -ai / (d * s));
}

template <int RPT, int NB>
__global__ __launch_bounds__(PT) __attribute__((amdgpu_waves_per_eu(1, 2))) void k_inv_panel(const InvJob* __restrict__ jobs, int k0, int nbw,
                                                  int32_t* __restrict__ status) {
  const InvJob jb = jobs[blockIdx.x];
  const int n = jb.n;
  if (k0 >= n) return;
  const int nb = min(nbw, n - k0);
  const int t = threadIdx.x, lane = t & 63, w = t >> 6;
  __shared__ double red_v[PT / 64];
  __shared__ int red_i[PT / 64];
  __shared__ double2 rowp[NB], rowc[NB], srow[NB];
  __shared__ int bad;
  if (t == 0) bad = 0;

  // the panel: row t + q*PT of the n x nb block, in registers
  double2 P[RPT][NB];
#pragma unroll
  for (int q = 0; q < RPT; ++q) {
    const int r = t + q * PT;
#pragma unroll
    for (int j = 0; j < NB; ++j) {
      double2 v = make_double2(0.0, 0.0);
      if (r < n && j < nb) v = jb.X[(int64_t)r * jb.ld + k0 + j];
      P[q][j] = v;
    }
  }
  __syncthreads();

#pragma unroll
  for (int j = 0; j < NB; ++j) {
    if (j < nb) {   // uniform over the block
      const int c = k0 + j;
      // pivot: largest |re|+|im| among rows >= c, smallest row on ties
      double bv = -1.0;
      int bi = n;
#pragma unroll
      for (int q = 0; q < RPT; ++q) {
        const int r = t + q * PT;
        if (r >= c && r < n) {
          const double v = cabs1(P[q][j]);
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
      if (prow >= n) {   // no candidate row (cannot happen for n <= RPT*PT): keep row c, flag
        prow = c;
        pv = 0.0;
      }
      // rows c and prow go through LDS
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
      // scaled pivot row
      if (t < NB) {
        const double2 pivv = rowp[j];
        const double2 inv = crcp(pivv);
        srow[t] = (t == j) ? inv : cmul(rowp[t], inv);
        if (t == 0 && (!(pv > 0.0) || !isfinite(pivv.x) || !isfinite(pivv.y))) bad = 1;
      }
      __syncthreads();
      const double2 inv = srow[j];
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
          const double2 m = P[q][j];
#pragma unroll
          for (int jj = 0; jj < NB; ++jj) {
            if (jj != j) {
              const double2 u = cmul(m, srow[jj]);
              P[q][jj].x -= u.x;
              P[q][jj].y -= u.y;
            }
          }
          const double2 u = cmul(m, inv);
          P[q][j] = make_double2(-u.x, -u.y);
        }
      }
    }
  }
  // write back the panel and T - I
#pragma unroll
  for (int q = 0; q < RPT; ++q) {
    const int r = t + q * PT;
    if (r < n) {
#pragma unroll
      for (int j = 0; j < NB; ++j) {
        if (j < nb) {
          jb.X[(int64_t)r * jb.ld + k0 + j] = P[q][j];
          double2 v = P[q][j];
          if (r == k0 + j) v.x -= 1.0;
          jb.T[(int64_t)r * nb + j] = v;
        }
      }
    }
  }
  __syncthreads();
  if (t == 0 && bad && status) atomicMin(&status[jb.e], (int32_t)HSC_E_SINGULAR);
}

// Apply the panel's row interchanges to the non-panel columns and copy the
// pivot rows (panel columns zeroed) into R.
__global__ __launch_bounds__(256) void k_inv_swap(const InvJob* __restrict__ jobs, int k0, int nbw,
                                                  int chunks) {
  const InvJob jb = jobs[blockIdx.x / chunks];
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
        double2* a = jb.X + (int64_t)c * jb.ld + col;
        double2* b = jb.X + (int64_t)p * jb.ld + col;
        const double2 x = *a;
        *a = *b;
        *b = x;
      }
    }
  }
  for (int j = 0; j < nb; ++j)
    jb.R[(int64_t)j * n + col] = in_panel ? make_double2(0.0, 0.0) : jb.X[(int64_t)(k0 + j) * jb.ld + col];
}

// After the NB-panels of a super-panel [s0, s0 + ws):
//   U[r][c] = X[r][s0 + c] - (r == s0 + c)   (n x ws, row stride W; the T workspace)
//   R[c][j] = X[s0 + c][j]                     (ws x n; the R workspace)
__global__ __launch_bounds__(64) void k_inv_super_u(const InvJob* __restrict__ jobs, int s0, int W, int chunks) {
  const InvJob jb = jobs[blockIdx.x / chunks];
  const int n = jb.n;
  if (s0 >= n) return;
  const int ws = min(W, n - s0);
  const int c = threadIdx.x;
  const int r0 = (blockIdx.x % chunks) * 16;
  if (c >= ws) return;
  for (int r = r0; r < min(n, r0 + 16); ++r) {
    double2 v = jb.X[(int64_t)r * jb.ld + s0 + c];
    if (r == s0 + c) v.x -= 1.0;
    jb.T[(int64_t)r * W + c] = v;
  }
}

__global__ __launch_bounds__(256) void k_inv_super_r(const InvJob* __restrict__ jobs, int s0, int W, int chunks) {
  const InvJob jb = jobs[blockIdx.x / (W * chunks)];
  const int n = jb.n;
  if (s0 >= n) return;
  const int ws = min(W, n - s0);
  const int rem = blockIdx.x % (W * chunks);
  const int c = rem / chunks;
  const int j = (rem % chunks) * 256 + threadIdx.x;
  if (c >= ws || j >= n) return;
  jb.R[(int64_t)c * n + j] = jb.X[(int64_t)(s0 + c) * jb.ld + j];
}

// Y[r][j] = X[r][idx[j]] where idx undoes the interchanges in reverse order.
__global__ __launch_bounds__(256) void k_inv_unscramble(const InvJob* __restrict__ jobs, int rows_per_block,
                                                        int chunks) {
  extern __shared__ int idx[];
  const InvJob jb = jobs[blockIdx.x / chunks];
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
    for (int j = threadIdx.x; j < n; j += blockDim.x)
      jb.Y[(int64_t)r * jb.ldy + j] = jb.X[(int64_t)r * jb.ld + idx[j]];
}

}  // namespace

void launch_inv_panel(hipStream_t st, const InvJob* jobs, int njobs, int k0, int nb, int max_n,
                      int32_t* status) {
  if (njobs <= 0 || max_n > 8 * PT) return;   // callers validate n <= 4096
  dim3 g(njobs), b(PT);
  if (max_n <= 512 && nb <= 16)
    hipLaunchKernelGGL((k_inv_panel<1, 16>), g, b, 0, st, jobs, k0, nb, status);
  else if (max_n <= 1024 && nb <= 16)
    hipLaunchKernelGGL((k_inv_panel<2, 16>), g, b, 0, st, jobs, k0, nb, status);
  else if (max_n <= 2048 && nb <= 8)
    hipLaunchKernelGGL((k_inv_panel<4, 8>), g, b, 0, st, jobs, k0, nb, status);
  else
    hipLaunchKernelGGL((k_inv_panel<8, 4>), g, b, 0, st, jobs, k0, nb, status);
}

void launch_inv_swap(hipStream_t st, const InvJob* jobs, int njobs, int k0, int nb, int max_n) {
  if (njobs <= 0) return;
  const int chunks = (max_n + 255) / 256;
  hipLaunchKernelGGL(k_inv_swap, dim3(njobs * chunks), dim3(256), 0, st, jobs, k0, nb, chunks);
}

void launch_inv_super(hipStream_t st, const InvJob* jobs, int njobs, int s0, int W, int max_n) {
  if (njobs <= 0 || W <= 0 || W > 64) return;
  const int cu = (max_n + 15) / 16, cr = (max_n + 255) / 256;
  hipLaunchKernelGGL(k_inv_super_u, dim3(njobs * cu), dim3(64), 0, st, jobs, s0, W, cu);
  hipLaunchKernelGGL(k_inv_super_r, dim3(njobs * W * cr), dim3(256), 0, st, jobs, s0, W, cr);
}

void launch_inv_unscramble(hipStream_t st, const InvJob* jobs, int njobs, int max_n) {
  if (njobs <= 0) return;
  const int rpb = 16;
  const int chunks = (max_n + rpb - 1) / rpb;
  hipLaunchKernelGGL(k_inv_unscramble, dim3(njobs * chunks), dim3(256), max_n * sizeof(int), st, jobs, rpb,
                     chunks);
}

}  // namespace hsc
