// Bandwidth-bound kernels of the solve: per-energy scalars, frontal assembly
// (Algorithm 1 fold: A_ii, A_ij plus the Schur updates of the children),
// gathers from the parent's frontal blocks (Algorithm 1/2 extract), the
// N-frontal assembly with its seed N = Sigma^< (G^r)^dagger (Algorithm 2), and
// the diagonal / transmission outputs.
#include <hip/hip_runtime.h>

#include "dd.h"
#include "kern.h"

namespace hsc {

namespace {

__device__ inline double2 cadd(double2 a, double2 b) { return make_double2(a.x + b.x, a.y + b.y); }
__device__ inline double2 cmul(double2 a, double2 b) {
  return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}

// principal square root
__device__ inline double2 csqrt_p(double2 z) {
  const double r = hypot(z.x, z.y);
  if (r == 0.0) return make_double2(0.0, 0.0);
  if (z.x >= 0.0) {
    const double a = sqrt(0.5 * (r + z.x));
    return make_double2(a, z.y / (2.0 * a));
  }
  double b = sqrt(0.5 * (r - z.x));
  if (z.y < 0.0) b = -b;
  return make_double2(z.y / (2.0 * b), b);
}

__device__ inline double2 cdiv_real(double2 a, double s) { return make_double2(a.x / s, a.y / s); }

// Surface Green's function of a semi-infinite chain: t^2 g^2 - w g + 1 = 0,
// the decaying root (smaller modulus; the two roots multiply to 1/t^2).
__device__ inline double2 lead_sigma(double2 z, double eps0, double tl, double tc) {
  const double2 w = make_double2(z.x - eps0, z.y);
  const double2 w2 = cmul(w, w);
  const double2 disc = csqrt_p(make_double2(w2.x - 4.0 * tl * tl, w2.y));
  const double2 g1 = cdiv_real(cadd(w, disc), 2.0 * tl * tl);
  const double2 g2 = cdiv_real(make_double2(w.x - disc.x, w.y - disc.y), 2.0 * tl * tl);
  const double m1 = hypot(g1.x, g1.y), m2 = hypot(g2.x, g2.y);
  const double2 g = m1 < m2 ? g1 : g2;
  return make_double2(tc * tc * g.x, tc * tc * g.y);
}

__device__ inline double fermi_fn(double e, double mu, double kT) {
  const double x = (e - mu) / kT;
  if (x > 0.0) {
    const double ex = exp(-x);
    return ex / (1.0 + ex);
  }
  return 1.0 / (1.0 + exp(x));
}

__global__ void k_energy_setup(const double* __restrict__ energies, int nvalid, int nslots, double eta,
                               double kT, double mu_L, double mu_R, LeadParams lp,
                               EnergyScalars* __restrict__ out, int32_t* __restrict__ status) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= nslots) return;
  const double en = energies[e < nvalid ? e : nvalid - 1];   // idle slots repeat the last energy
  status[e] = isfinite(en) ? 0 : (int32_t)HSC_E_NONFINITE;
  EnergyScalars s;
  s.z = make_double2(en, eta);
  for (int c = 0; c < 2; ++c) {
    s.sig[c] = lead_sigma(s.z, lp.onsite[c], lp.hopping[c], lp.coupling[c]);
    s.gam[c] = -2.0 * s.sig[c].y;
  }
  s.fermi[0] = fermi_fn(en, mu_L, kT);
  s.fermi[1] = fermi_fn(en, mu_R, kT);
  out[e] = s;
}

constexpr int RB = 256;

// F[a][b] = sum_children U_k[invrel_k[a]][invrel_k[b]] + (-H)[a][b] + delta_ab (z - Sigma_a - U_a)
//   jobs: rows = cols = n+f; p0 = ChildRef[aux0]; p1 = FrontSparse*; aux1 = n, aux2 = nL, aux3 = nR
__global__ __launch_bounds__(RB) void k_assemble(const RowJob* __restrict__ jobs, const int32_t* __restrict__ row_job,
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
  double2 diag_add = make_double2(0.0, 0.0);
  if (a < n) {
    const EnergyScalars& s = es[jb.e];
    diag_add = s.z;
    if (a < nL) { diag_add.x -= s.sig[0].x; diag_add.y -= s.sig[0].y; }
    else if (a < nL + nR) { diag_add.x -= s.sig[1].x; diag_add.y -= s.sig[1].y; }
    if (fs->pot) diag_add.x -= fs->pot[a];
  }
  double2* out = jb.dst + (int64_t)a * jb.ldd;
  // whole-face contact cluster: minus its dense self-energy block (rows and columns < nface)
  const double2* dsig = a < jb.aux4 ? reinterpret_cast<const double2*>(jb.p2) : nullptr;
  const int nface = jb.aux4;
  // children whose update has a row for a: that row and the column map, up to four in registers
  constexpr int KMAX = 4;
  const double2* urow[KMAX];
  const int32_t* umap[KMAX];
  int nu = 0;
  for (int k = 0; k < nk && k < KMAX; ++k) {
    const int ia = kids[k].invrel[a];
    if (ia >= 0) {
      urow[nu] = kids[k].U + (int64_t)ia * kids[k].ldU;
      umap[nu++] = kids[k].invrel;
    }
  }
  for (int b = threadIdx.x; b < cols; b += RB) {
    double2 v = make_double2(0.0, 0.0);
    for (int q = 0; q < nu; ++q) {
      const int ib = umap[q][b];
      if (ib >= 0) v = cadd(v, urow[q][ib]);
    }
    for (int k = KMAX; k < nk; ++k) {
      const int ia = kids[k].invrel[a];
      if (ia < 0) continue;
      const int ib = kids[k].invrel[b];
      if (ib < 0) continue;
      v = cadd(v, kids[k].U[(int64_t)ia * kids[k].ldU + ib]);
    }
    for (int q = 0; q < nq; ++q)
      if (s_col[q] == b) v = cadd(v, s_val[q]);
    for (int q = q0 + 64; q < q1; ++q)
      if (fs->col[q] == b) v = cadd(v, fs->val[q]);
    if (b == a) v = cadd(v, diag_add);
    if (dsig && b < nface) {
      const double2 sv = dsig[(int64_t)a * nface + b];
      v.x -= sv.x;
      v.y -= sv.y;
    }
    out[b] = v;
  }
}

// dst[r][c] = op(trans ? src[cmap[c]][rmap[r]] : src[rmap[r]][cmap[c]]);  op 1 = -conj
template <int TRANS, int OP>
__global__ __launch_bounds__(RB) void k_gather(const RowJob* __restrict__ jobs, const int32_t* __restrict__ row_job) {
  const int g = blockIdx.x;
  const RowJob& jb = jobs[row_job[g]];
  const int r = g - jb.row_off;
  const int rr = jb.rmap ? jb.rmap[r] : r;
  const int cols = jb.cols;
  const int64_t lds = jb.lds;
  const int32_t* __restrict__ cmap = jb.cmap;
  const double2* __restrict__ src = jb.src;
  double2* __restrict__ out = jb.dst + (int64_t)r * jb.ldd;
  // four columns per thread and step: four independent loads in flight
  for (int c0 = threadIdx.x; c0 < cols; c0 += 4 * RB) {
    double2 v[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int c = c0 + u * RB;
      if (c < cols) {
        const int cc = cmap ? cmap[c] : c;
        v[u] = TRANS ? src[(int64_t)cc * lds + rr] : src[(int64_t)rr * lds + cc];
      }
    }
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int c = c0 + u * RB;
      if (c < cols) out[c] = OP == 1 ? make_double2(-v[u].x, v[u].y) : v[u];
    }
  }
}

// NF[rr][b] = sum_children U_k[invrel_k[a(rr)]][b] + seed(rr, b)
//   a(rr) = rr < r ? row0 + rr : n + (rr - r)
//   seed: rr < r, a < nL + nR: i * w(side) * conj(Grow[a][b])
//   jobs: p0 = ChildRef[aux0]; aux1 = r; aux2 = row0; aux3 = n; aux4 = nL; aux5 = nR; src = Grow (lds)
__global__ __launch_bounds__(RB) void k_assemble_n(const RowJob* __restrict__ jobs, const int32_t* __restrict__ row_job,
                                                   const EnergyScalars* __restrict__ es, int channel) {
  const int g = blockIdx.x;
  const RowJob& jb = jobs[row_job[g]];
  const int rr = g - jb.row_off;
  const ChildRef* kids = reinterpret_cast<const ChildRef*>(jb.p0);
  const int nk = jb.aux0, r = jb.aux1, row0 = jb.aux2, n = jb.aux3, nL = jb.aux4, nR = jb.aux5;
  const int a = rr < r ? row0 + rr : n + (rr - r);
  // seed rows: i w conj(G row a); for a whole-face contact p1 holds Gamma G (the face's Gamma
  // times its G rows, same leading dimension) and w is the occupation alone
  const double2* gam_g = reinterpret_cast<const double2*>(jb.p1);
  double w = 0.0;
  if (rr < r && a < nL + nR)
    w = gam_g ? channel_occ(es[jb.e], channel, a < nL ? 0 : 1) : channel_weight(es[jb.e], channel, a < nL ? 0 : 1);
  const double2* grow = (gam_g ? gam_g : jb.src) + (int64_t)a * jb.lds;
  double2* out = jb.dst + (int64_t)rr * jb.ldd;
  // the row of each child's update that lands on row a (same for every column): up to four
  // children in registers, more through the general loop
  constexpr int KMAX = 4;
  const double2* urow[KMAX];
  int nu = 0;
  for (int k = 0; k < nk && k < KMAX; ++k) {
    const int ia = kids[k].invrel[a];
    if (ia >= 0) urow[nu++] = kids[k].U + (int64_t)ia * kids[k].ldU;
  }
  const int cols = jb.cols;
  if (nk <= KMAX) {
    // four columns per thread and step, all loads issued before the stores
    for (int b0 = threadIdx.x; b0 < cols; b0 += 4 * RB) {
      double2 v[4];
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const int b = b0 + u * RB;
        v[u] = make_double2(0.0, 0.0);
        if (b < cols) {
          for (int q = 0; q < nu; ++q) v[u] = cadd(v[u], urow[q][b]);
          if (w != 0.0) {
            const double2 gv = grow[b];
            v[u].x += w * gv.y;
            v[u].y += w * gv.x;
          }
        }
      }
#pragma unroll
      for (int u = 0; u < 4; ++u)
        if (b0 + u * RB < cols) out[b0 + u * RB] = v[u];
    }
    return;
  }
  for (int b = threadIdx.x; b < cols; b += RB) {
    double2 v = make_double2(0.0, 0.0);
    for (int q = 0; q < nu; ++q) v = cadd(v, urow[q][b]);
    for (int k = KMAX; k < nk; ++k) {
      const int ia = kids[k].invrel[a];
      if (ia >= 0) v = cadd(v, kids[k].U[(int64_t)ia * kids[k].ldU + b]);
    }
    if (w != 0.0) {
      const double2 gv = grow[b];
      v.x += w * gv.y;
      v.y += w * gv.x;
    }
    out[b] = v;
  }
}

// Diagonal outputs, one wave per row.
//   DIAG_SEP:    v = src[k][k]
//   DIAG_LEAF_G: v = Inv[k][k] + sum_j Psi[k][j] * GT[k][j]           (p1 = Inv, aux1 = ld Inv)
//   DIAG_LEAF_P: v = M[k][k] - sum_j Psi[k][j] * conj(PT[k][j])      (p1 = M or null, aux1 = ld M)
//   p0 = Psi (ld aux0 = f), src = GT/PT (lds), p2 = int64 sites of the rows
template <int MODE>
__global__ __launch_bounds__(RB) void k_diag(const RowJob* __restrict__ jobs, const int32_t* __restrict__ row_job,
                                             int total_rows, int out_kind, void* out, int64_t out_stride,
                                             int e_base, int nvalid) {
  const int g = blockIdx.x * (RB / 64) + (threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  if (g >= total_rows) return;
  const RowJob& jb = jobs[row_job[g]];
  const int k = g - jb.row_off;
  if (jb.e >= nvalid) return;
  double2 v = make_double2(0.0, 0.0);
  if (MODE == DIAG_SEP) {
    v = jb.src[(int64_t)k * jb.lds + k];
  } else {
    const int f = jb.aux0;
    const double2* psi = reinterpret_cast<const double2*>(jb.p0) + (int64_t)k * f;
    const double2* x = jb.src + (int64_t)k * jb.lds;
    double2 acc = make_double2(0.0, 0.0);
    for (int j = lane; j < f; j += 64) {
      double2 y = x[j];
      if (MODE == DIAG_LEAF_P) y.y = -y.y;
      acc = cadd(acc, cmul(psi[j], y));
    }
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
      acc.x += __shfl_xor(acc.x, off, 64);
      acc.y += __shfl_xor(acc.y, off, 64);
    }
    const double2* base = reinterpret_cast<const double2*>(jb.p1);
    double2 d = base ? base[(int64_t)k * jb.aux1 + k] : make_double2(0.0, 0.0);
    if (MODE == DIAG_LEAF_P) v = make_double2(d.x - acc.x, d.y - acc.y);
    else v = cadd(d, acc);
  }
  if (lane != 0) return;
  const int64_t site = reinterpret_cast<const int64_t*>(jb.p2)[k];
  const int64_t idx = (int64_t)(e_base + jb.e) * out_stride + site;
  if (out_kind == OUT_COMPLEX) reinterpret_cast<double2*>(out)[idx] = v;
  else reinterpret_cast<double*>(out)[idx] = v.y;
}

__global__ __launch_bounds__(RB) void k_trans(const double* __restrict__ a_r, int64_t ld,
                                              const int64_t* __restrict__ left, int nleft, int nvalid,
                                              int e_base, const EnergyScalars* __restrict__ es,
                                              double* __restrict__ trans) {
  const int e = blockIdx.x;
  if (e >= nvalid) return;
  __shared__ double red[RB];
  double acc = 0.0;
  for (int k = threadIdx.x; k < nleft; k += RB) acc += a_r[(int64_t)e * ld + left[k]];
  red[threadIdx.x] = acc;
  __syncthreads();
  for (int s = RB / 2; s > 0; s >>= 1) {
    if (threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
    __syncthreads();
  }
  if (threadIdx.x == 0) trans[e_base + e] = es[e].gam[0] * red[0];
}

__global__ void k_combine_gl(const double* __restrict__ spec, int nvalid, int e_base, int64_t n,
                             const EnergyScalars* __restrict__ es, double2* __restrict__ gl) {
  const int e = blockIdx.y;
  if (e >= nvalid) return;
  const int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= n) return;
  const int64_t eg = e_base + e;
  const double al = spec[eg * 2 * n + s], ar = spec[eg * 2 * n + n + s];
  gl[eg * n + s] = make_double2(0.0, es[e].fermi[0] * al + es[e].fermi[1] * ar);
}

// per (cluster, slot): infinity norms (max row sum of moduli) of Inv = A_ii^-1
// and of Psi.  For the complex-symmetric Inv, ||Inv||_2 <= ||Inv||_inf.
//   jobs: src = Inv (n x n, ld lds), p0 = Psi (n x f), aux0 = n, aux1 = f, aux2 = cluster index
__global__ __launch_bounds__(RB) void k_guard(const RowJob* __restrict__ jobs, int nclusters, int e_base, int nvalid,
                                              double* __restrict__ out) {
  const RowJob& jb = jobs[blockIdx.x];
  if (jb.e >= nvalid) return;
  const int n = jb.aux0, f = jb.aux1;
  const double2* psi = reinterpret_cast<const double2*>(jb.p0);
  __shared__ double red[2][RB];
  double mi = 0.0, mp = 0.0;
  for (int r = threadIdx.x; r < n; r += RB) {
    double si = 0.0, sp = 0.0;
    const double2* row = jb.src + (int64_t)r * jb.lds;
    for (int j = 0; j < n; ++j) si += hypot(row[j].x, row[j].y);
    if (psi) {
      const double2* prow = psi + (int64_t)r * f;
      for (int j = 0; j < f; ++j) sp += hypot(prow[j].x, prow[j].y);
    }
    mi = fmax(mi, si);
    mp = fmax(mp, sp);
  }
  red[0][threadIdx.x] = mi;
  red[1][threadIdx.x] = mp;
  __syncthreads();
  for (int s = RB / 2; s > 0; s >>= 1) {
    if (threadIdx.x < s) {
      red[0][threadIdx.x] = fmax(red[0][threadIdx.x], red[0][threadIdx.x + s]);
      red[1][threadIdx.x] = fmax(red[1][threadIdx.x], red[1][threadIdx.x + s]);
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    const int64_t o = ((int64_t)(e_base + jb.e) * nclusters + jb.aux2) * 2;
    out[o] = red[0][0];
    out[o + 1] = red[1][0];
  }
}

}  // namespace

void launch_guard(hipStream_t st, const RowJob* jobs, int njobs, int nclusters, int e_base, int nvalid,
                  double* out) {
  if (njobs <= 0 || !out) return;
  hipLaunchKernelGGL(k_guard, dim3(njobs), dim3(RB), 0, st, jobs, nclusters, e_base, nvalid, out);
}

// ---- whole-face contacts: dense self-energy (Section 3.1.2's DENSE case) ----
// Each transverse mode (p, q) of the face is a semi-infinite chain with on-site
// eps + 2 tl (cos(pi (p+1) / (d1+1)) + cos(pi (q+1) / (d2+1))) and hopping tl; the face block is
// Sigma = tc^2 sum_{p,q} g_pq (phi_p x phi_q)(phi_p x phi_q)^T, summed over q first (one block per
// (job, p)), then over p (one thread per entry).
constexpr double kPi = 3.14159265358979323846;

__global__ __launch_bounds__(256) void k_face_half(const FaceJob* __restrict__ jobs,
                                                   const EnergyScalars* __restrict__ es) {
  extern __shared__ double2 s_g[];   // [d2] surface functions of the modes (p, 0..d2-1)
  const FaceJob& j = jobs[blockIdx.y];
  const int p = blockIdx.x;
  if (p >= j.d1) return;
  const int d2 = j.d2;
  const double2 z = es[j.e].z;
  const double cp = cos(kPi * (p + 1) / (j.d1 + 1));
  for (int q = threadIdx.x; q < d2; q += blockDim.x)
    s_g[q] = lead_sigma(z, j.eps + 2.0 * j.tl * (cp + cos(kPi * (q + 1) / (d2 + 1))), j.tl, 1.0);
  __syncthreads();
  double2* out = j.half + (int64_t)p * d2 * d2;
  for (int idx = threadIdx.x; idx < d2 * d2; idx += blockDim.x) {
    const int k = idx / d2, k2 = idx - k * d2;
    const double* r1 = j.tab2 + (int64_t)k * d2;
    const double* r2 = j.tab2 + (int64_t)k2 * d2;
    double re = 0.0, im = 0.0;
    for (int q = 0; q < d2; ++q) {
      const double w = r1[q] * r2[q];
      re = fma(w, s_g[q].x, re);
      im = fma(w, s_g[q].y, im);
    }
    out[idx] = make_double2(re, im);
  }
}

__global__ __launch_bounds__(256) void k_face_sigma(const FaceJob* __restrict__ jobs) {
  const FaceJob& j = jobs[blockIdx.y];
  const int64_t F = j.F;
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= F * F) return;
  const int a = (int)(idx / F), b = (int)(idx - (int64_t)a * F);
  const int d1 = j.d1, d2 = j.d2;
  const int ja = j.jk[a] / d2, ka = j.jk[a] - ja * d2;
  const int jb = j.jk[b] / d2, kb = j.jk[b] - jb * d2;
  const double* r1 = j.tab1 + (int64_t)ja * d1;
  const double* r2 = j.tab1 + (int64_t)jb * d1;
  const double2* h = j.half + (int64_t)ka * d2 + kb;
  const int64_t hs = (int64_t)d2 * d2;
  double re = 0.0, im = 0.0;
  for (int p = 0; p < d1; ++p) {
    const double w = r1[p] * r2[p];
    const double2 hv = h[p * hs];
    re = fma(w, hv.x, re);
    im = fma(w, hv.y, im);
  }
  const double t2 = j.tc * j.tc;
  const double2 sg = make_double2(t2 * re, t2 * im);
  j.sigma[idx] = sg;
  const double gam = -2.0 * sg.y;
  if (j.gamma_dd) reinterpret_cast<zdd*>(j.gamma)[idx] = zdd{dd{gam, 0.0}, dd{0.0, 0.0}};
  else reinterpret_cast<double2*>(j.gamma)[idx] = make_double2(gam, 0.0);
}

// The lesser-type block of the right channel is P = G (i Gamma_R) G^dagger = i A_R, so
// T = Tr(Gamma_L A_R) over the left face = sum_{a,b} Gamma_L[a][b] Im P[a][b].
__global__ __launch_bounds__(256) void k_face_trans(const FaceTransJob* __restrict__ jobs, int nvalid, int e_base,
                                                    double* __restrict__ trans) {
  const int e = blockIdx.x;
  if (e >= nvalid) return;
  const FaceTransJob& j = jobs[e];
  const int64_t F = j.F;
  dd acc{0.0, 0.0};
  for (int64_t idx = threadIdx.x; idx < F * F; idx += blockDim.x) {
    const int64_t a = idx / F, b = idx - a * F;
    if (j.dd) {
      const double g = reinterpret_cast<const zdd*>(j.gamma)[idx].re.hi;
      acc = dd_add(acc, dd_mul(dd_from(g), reinterpret_cast<const zdd*>(j.P)[a * j.ldp + b].im));
    } else {
      const double g = reinterpret_cast<const double2*>(j.gamma)[idx].x;
      acc = dd_add(acc, two_prod(g, reinterpret_cast<const double2*>(j.P)[a * j.ldp + b].y));
    }
  }
  __shared__ double sh[256], sl[256];
  sh[threadIdx.x] = acc.hi;
  sl[threadIdx.x] = acc.lo;
  __syncthreads();
  for (int s = blockDim.x / 2; s > 0; s >>= 1) {
    if (threadIdx.x < s) {
      const dd v = dd_add(dd{sh[threadIdx.x], sl[threadIdx.x]}, dd{sh[threadIdx.x + s], sl[threadIdx.x + s]});
      sh[threadIdx.x] = v.hi;
      sl[threadIdx.x] = v.lo;
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) trans[e_base + e] = sh[0] + sl[0];
}

void launch_energy_setup(hipStream_t st, const double* energies, int nvalid, int nslots, double eta,
                         double kT, double mu_L, double mu_R, LeadParams lp, EnergyScalars* out,
                         int32_t* status) {
  if (nslots <= 0) return;
  hipLaunchKernelGGL(k_energy_setup, dim3((nslots + 63) / 64), dim3(64), 0, st, energies, nvalid, nslots, eta,
                     kT, mu_L, mu_R, lp, out, status);
}

__global__ void k_status_out(const int32_t* __restrict__ st_slots, int nvalid, int32_t* __restrict__ out) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e < nvalid) out[e] = st_slots[e];
}

void launch_status_out(hipStream_t st, const int32_t* st_slots, int nvalid, int32_t* out) {
  if (nvalid <= 0 || !out) return;
  hipLaunchKernelGGL(k_status_out, dim3((nvalid + 63) / 64), dim3(64), 0, st, st_slots, nvalid, out);
}

void launch_assemble(hipStream_t st, const RowJob* jobs, const int32_t* row_job, int total_rows,
                     const EnergyScalars* es) {
  if (total_rows <= 0) return;
  hipLaunchKernelGGL(k_assemble, dim3(total_rows), dim3(RB), 0, st, jobs, row_job, es);
}

void launch_gather(hipStream_t st, const RowJob* jobs, const int32_t* row_job, int total_rows, int trans,
                   int op) {
  if (total_rows <= 0) return;
  if (trans && op) hipLaunchKernelGGL((k_gather<1, 1>), dim3(total_rows), dim3(RB), 0, st, jobs, row_job);
  else if (trans) hipLaunchKernelGGL((k_gather<1, 0>), dim3(total_rows), dim3(RB), 0, st, jobs, row_job);
  else if (op) hipLaunchKernelGGL((k_gather<0, 1>), dim3(total_rows), dim3(RB), 0, st, jobs, row_job);
  else hipLaunchKernelGGL((k_gather<0, 0>), dim3(total_rows), dim3(RB), 0, st, jobs, row_job);
}

void launch_assemble_n(hipStream_t st, const RowJob* jobs, const int32_t* row_job, int total_rows,
                       const EnergyScalars* es, int channel) {
  if (total_rows <= 0) return;
  hipLaunchKernelGGL(k_assemble_n, dim3(total_rows), dim3(RB), 0, st, jobs, row_job, es, channel);
}

void launch_diag(hipStream_t st, const RowJob* jobs, const int32_t* row_job, int total_rows, int mode,
                 int out_kind, void* out, int64_t out_stride, int e_base, int nvalid) {
  if (total_rows <= 0) return;
  dim3 grid((total_rows + 3) / 4), block(RB);
  if (mode == DIAG_SEP)
    hipLaunchKernelGGL(k_diag<DIAG_SEP>, grid, block, 0, st, jobs, row_job, total_rows, out_kind, out,
                       out_stride, e_base, nvalid);
  else if (mode == DIAG_LEAF_G)
    hipLaunchKernelGGL(k_diag<DIAG_LEAF_G>, grid, block, 0, st, jobs, row_job, total_rows, out_kind, out,
                       out_stride, e_base, nvalid);
  else
    hipLaunchKernelGGL(k_diag<DIAG_LEAF_P>, grid, block, 0, st, jobs, row_job, total_rows, out_kind, out,
                       out_stride, e_base, nvalid);
}

void launch_trans(hipStream_t st, const double* a_r, int64_t ld, const int64_t* left_sites, int nleft,
                  int nslots, int nvalid, int e_base, const EnergyScalars* es, double* trans) {
  if (nslots <= 0) return;
  hipLaunchKernelGGL(k_trans, dim3(nslots), dim3(RB), 0, st, a_r, ld, left_sites, nleft, nvalid, e_base, es,
                     trans);
}

// bond entries (see BondRef); one thread per (bond, slot)
__device__ inline double2 bz_mul(double2 a, double2 b) { return cmul(a, b); }
__device__ inline zdd bz_mul(zdd a, zdd b) { return zdd_mul(a, b); }
__device__ inline double2 bz_add(double2 a, double2 b) { return cadd(a, b); }
__device__ inline zdd bz_add(zdd a, zdd b) { return zdd_add(a, b); }
__device__ inline double2 bz_conj(double2 a) { return make_double2(a.x, -a.y); }
__device__ inline zdd bz_conj(zdd a) { return zdd{a.re, dd_neg(a.im)}; }
__device__ inline double2 bz_neg(double2 a) { return make_double2(-a.x, -a.y); }
__device__ inline zdd bz_neg(zdd a) { return zdd_neg(a); }
__device__ inline double2 bz_round(double2 a) { return a; }
__device__ inline double2 bz_round(zdd a) { return zdd_round(a); }
template <class T> __device__ inline T bz_zero();
template <> __device__ inline double2 bz_zero<double2>() { return make_double2(0.0, 0.0); }
template <> __device__ inline zdd bz_zero<zdd>() { return zdd_zero(); }

template <class T, int LESSER>
__global__ __launch_bounds__(256) void k_bonds(const BondRef* __restrict__ refs, int nbonds,
                                               const BondSrc* __restrict__ src, int nslots, int nvalid, int e_base,
                                               double2* __restrict__ out) {
  const int b = blockIdx.x * blockDim.x + threadIdx.x;
  const int e = blockIdx.y;
  if (b >= nbonds || e >= nvalid) return;
  const BondRef r = refs[b];
  const BondSrc& s = src[(int64_t)r.c * nslots + e];
  const int col = LESSER ? r.colp : r.colg;
  T v;
  if (r.mode == 0) {
    v = reinterpret_cast<const T*>(s.X)[(int64_t)r.a * s.ld + col];
  } else if (r.mode == 2) {
    v = reinterpret_cast<const T*>(s.xt)[(int64_t)r.a * s.f + col];
  } else {
    const T* psi = reinterpret_cast<const T*>(s.psi) + (int64_t)r.a * s.f;
    const T* xt = reinterpret_cast<const T*>(s.xt) + (int64_t)col * s.f;
    T acc = bz_zero<T>();
    for (int j = 0; j < s.f; ++j) acc = bz_add(acc, bz_mul(psi[j], LESSER ? bz_conj(xt[j]) : xt[j]));
    const T d = s.d ? reinterpret_cast<const T*>(s.d)[(int64_t)r.a * s.ldd + col] : bz_zero<T>();
    v = LESSER ? bz_add(d, bz_neg(acc)) : bz_add(d, acc);
  }
  if (LESSER && r.flip) v = bz_neg(bz_conj(v));
  out[(int64_t)(e_base + e) * nbonds + b] = bz_round(v);
}

void launch_face_half(hipStream_t st, const FaceJob* jobs, int njobs, int max_d1, int max_d2,
                      const EnergyScalars* es) {
  if (njobs <= 0 || max_d1 <= 0) return;
  hipLaunchKernelGGL(k_face_half, dim3(max_d1, njobs), dim3(256), (size_t)max_d2 * sizeof(double2), st, jobs, es);
}

void launch_face_sigma(hipStream_t st, const FaceJob* jobs, int njobs, int max_f) {
  if (njobs <= 0 || max_f <= 0) return;
  const int64_t cells = (int64_t)max_f * max_f;
  hipLaunchKernelGGL(k_face_sigma, dim3((unsigned)((cells + 255) / 256), njobs), dim3(256), 0, st, jobs);
}

void launch_face_trans(hipStream_t st, const FaceTransJob* jobs, int nvalid, int e_base, double* trans) {
  if (nvalid <= 0) return;
  hipLaunchKernelGGL(k_face_trans, dim3(nvalid), dim3(256), 0, st, jobs, nvalid, e_base, trans);
}

void launch_bonds(hipStream_t st, const BondRef* refs, int nbonds, const BondSrc* src, int nslots, int nvalid,
                  int e_base, int lesser, int dd, double2* out) {
  if (nbonds <= 0 || nvalid <= 0 || !out) return;
  const dim3 grid((unsigned)((nbonds + 255) / 256), nvalid);
  if (dd) {
    if (lesser) hipLaunchKernelGGL((k_bonds<zdd, 1>), grid, dim3(256), 0, st, refs, nbonds, src, nslots, nvalid, e_base, out);
    else hipLaunchKernelGGL((k_bonds<zdd, 0>), grid, dim3(256), 0, st, refs, nbonds, src, nslots, nvalid, e_base, out);
  } else {
    if (lesser) hipLaunchKernelGGL((k_bonds<double2, 1>), grid, dim3(256), 0, st, refs, nbonds, src, nslots, nvalid, e_base, out);
    else hipLaunchKernelGGL((k_bonds<double2, 0>), grid, dim3(256), 0, st, refs, nbonds, src, nslots, nvalid, e_base, out);
  }
}

void launch_combine_gl(hipStream_t st, const double* spec, int nvalid, int e_base, int64_t n,
                       const EnergyScalars* es, double2* gl) {
  if (nvalid <= 0) return;
  dim3 grid((unsigned)((n + 255) / 256), nvalid);
  hipLaunchKernelGGL(k_combine_gl, grid, dim3(256), 0, st, spec, nvalid, e_base, n, es, gl);
}

namespace {

// totals[e][0] = -(1/pi) sum_i Im gr[e][i]; totals[e][1] = (1/2pi) sum_i Im gl[e][i];
// totals[e][2] = (1/2pi) sum_i (A_L + A_R)[e][i] from spec ([e][2][n]);
// one workgroup per energy, fixed-order reduction
__global__ __launch_bounds__(256) void k_totals(int64_t n, const double2* __restrict__ gr,
                                                const double2* __restrict__ gl, const double* __restrict__ spec,
                                                double* __restrict__ totals) {
  __shared__ double part[3][256];
  const int e = blockIdx.x;
  double a = 0.0, b = 0.0, c = 0.0;
  for (int64_t i = threadIdx.x; i < n; i += 256) {
    if (gr) a += gr[(int64_t)e * n + i].y;
    if (gl) b += gl[(int64_t)e * n + i].y;
    if (spec) c += spec[(int64_t)e * 2 * n + i] + spec[(int64_t)e * 2 * n + n + i];
  }
  part[0][threadIdx.x] = a;
  part[1][threadIdx.x] = b;
  part[2][threadIdx.x] = c;
  __syncthreads();
  for (int h = 128; h > 0; h /= 2) {
    if ((int)threadIdx.x < h)
      for (int q = 0; q < 3; ++q) part[q][threadIdx.x] += part[q][threadIdx.x + h];
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    const double pi = 3.141592653589793;
    if (gr) totals[3 * e] = -part[0][0] / pi;
    if (gl) totals[3 * e + 1] = part[1][0] / (2.0 * pi);
    if (spec) totals[3 * e + 2] = part[2][0] / (2.0 * pi);
  }
}

}  // namespace

void launch_totals(hipStream_t st, int n_e, int64_t n, const double2* gr, const double2* gl, const double* spec,
                   double* totals) {
  hipLaunchKernelGGL(k_totals, dim3(n_e), dim3(256), 0, st, n, gr, gl, spec, totals);
}

}  // namespace hsc
