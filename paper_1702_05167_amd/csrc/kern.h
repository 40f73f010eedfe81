// Device kernel descriptors and launchers (complex128 stored as double2).
#pragma once

#include <hip/hip_runtime.h>
#include <cstdint>
#include <string>

#include "../../include/hsc.h"

namespace hsc {

// op codes for GEMM operands and gathers
enum { OP_N = 0, OP_T = 1, OP_C = 2 };   // as is, transposed, conjugate-transposed

// One problem of a grouped GEMM:  D = alpha * op(A) * op(B) + beta * C
// (row-major, leading dimensions in elements).
struct GemmProb {
  const double2* A;
  const double2* B;
  const double2* C;
  double2* D;
  int32_t M, N, K;
  int32_t lda, ldb, ldc, ldd;
  int32_t tiles_n;   // ceil(N / tile width)
  int32_t tile_off;  // first tile of this problem in the launch
};

// Row-parallel 2D job (gathers, assembly, diagonals): one block per (job, row);
// row_job[g] = job owning global row g (host-built map).
struct RowJob {
  int32_t rows, cols;
  int32_t row_off;   // first global row of this job in the launch
  int32_t e;         // energy slot
  const double2* src;
  double2* dst;
  const int32_t* rmap;   // may be null (identity)
  const int32_t* cmap;   // may be null (identity)
  int32_t lds, ldd;
  int32_t aux0, aux1, aux2, aux3, aux4, aux5;   // kernel specific
  const void* p0;        // kernel specific
  const void* p1;
  const void* p2;
};

// Batched Gauss-Jordan matrix: in place on X (n x n, ld), result gathered into Y (ld ldy).
struct InvJob {
  double2* X;
  double2* Y;
  int32_t n, ld, ldy;
  int32_t e;          // energy slot (status reporting)
  int32_t* piv;       // [n] workspace
  double2* T;         // [n][W] workspace (panel / super-panel columns minus identity)
  double2* R;         // [W][n] workspace (pivot rows)
};

// Per-energy scalars computed on the device.
struct EnergyScalars {
  double2 z;
  double2 sig[2];     // contact self-energies (left, right)
  double gam[2];      // broadenings
  double fermi[2];    // occupations
};

// weight of a contact side in a lesser-self-energy channel:
// 0 = both contacts with occupations, 1 = left only, 2 = right only
__device__ inline double channel_weight(const EnergyScalars& s, int channel, int side) {
  if (channel == 0) return s.fermi[side] * s.gam[side];
  if (channel == 1) return side == 0 ? s.gam[0] : 0.0;
  return side == 1 ? s.gam[1] : 0.0;
}

// lesser-channel weight of a contact side without its broadening (whole-face contacts carry
// Gamma as a matrix): occupation in channel 0, 1 for the channel's own side, else 0
__device__ inline double channel_occ(const EnergyScalars& s, int channel, int side) {
  if (channel == 0) return s.fermi[side];
  if (channel == 1) return side == 0 ? 1.0 : 0.0;
  return side == 1 ? 1.0 : 0.0;
}

// Child of a frontal matrix: its update block U (rows/cols = child front) and
// invrel[a] = position of the parent's frontal index a in the child front, or -1.
struct ChildRef {
  const double2* U;
  const int32_t* invrel;
  int32_t ldU;
  int32_t pad;
};

// Sparse entries of A = -H restricted to a frontal matrix, CSR over its rows; pot: the on-site
// potential of the cluster's own rows (plan workspace, cluster order), subtracted on the diagonal
// (A = z I - (H + diag U) - Sigma), or null.
struct FrontSparse {
  const int32_t* ptr;
  const int32_t* col;
  const double2* val;
  const double* pot;
};

struct LeadParams {
  double onsite[2], hopping[2], coupling[2];
};

// launchers (all asynchronous on `st`)
// tile_prob[t] = problem owning tile t (host-built map; one entry per tile)
void launch_gemm(hipStream_t st, int opA, int opB, const GemmProb* probs, const int32_t* tile_prob,
                 int total_tiles, double alpha_re, double alpha_im, int beta, int tile_kind);
int gemm_tile_kinds();
int gemm_tile_m(int tile_kind);
int gemm_tile_n(int tile_kind);

// per-slot scalars for the slots of one chunk; idle slots (>= nvalid) repeat
// the last energy; status[slot] is reset (0, or NONFINITE for a bad energy)
void launch_energy_setup(hipStream_t st, const double* energies, int nvalid, int nslots, double eta,
                         double kT, double mu_L, double mu_R, LeadParams lp, EnergyScalars* out,
                         int32_t* status);
void launch_status_out(hipStream_t st, const int32_t* st_slots, int nvalid, int32_t* out);
void launch_totals(hipStream_t st, int n_e, int64_t n, const double2* gr, const double2* gl, const double* spec,
                   double* totals);

// Frontal assembly: F = sum of children's update blocks (pull) + sparse A entries.
void launch_assemble(hipStream_t st, const RowJob* jobs, const int32_t* row_job, int total_rows,
                     const EnergyScalars* es);
// dst[r][c] = op(src[rmap[r]][cmap[c]]) (or transposed source indexing)
void launch_gather(hipStream_t st, const RowJob* jobs, const int32_t* row_job, int total_rows, int trans, int op);
// N-frontal assembly: pull children's updates + seed rows i*w*conj(G row)
void launch_assemble_n(hipStream_t st, const RowJob* jobs, const int32_t* row_job, int total_rows,
                       const EnergyScalars* es, int channel);
// diagonal outputs (mode: DIAG_*), written for energy slots < nvalid at
// out[(e_base + slot) * out_stride + site]
enum { DIAG_SEP = 0, DIAG_LEAF_G = 1, DIAG_LEAF_P = 2 };
enum { OUT_COMPLEX = 0, OUT_IMAG = 1 };
void launch_diag(hipStream_t st, const RowJob* jobs, const int32_t* row_job, int total_rows, int mode,
                 int out_kind, void* out, int64_t out_stride, int e_base, int nvalid);
// T[e_base + slot] = Gamma_L(slot) * sum over left sites of a_r[slot][site]
void launch_trans(hipStream_t st, const double* a_r, int64_t ld, const int64_t* left_sites, int nleft,
                  int nslots, int nvalid, int e_base, const EnergyScalars* es, double* trans);
// diag G^< = i (f_L A_L + f_R A_R) from spectral [e][2][n]
void launch_combine_gl(hipStream_t st, const double* spec, int nvalid, int e_base, int64_t n,
                       const EnergyScalars* es, double2* gl);

// ---- whole-face contacts (dense self-energy blocks) ----
// One (energy slot, contact) job.  The face is a d1 x d2 rectangle; its lead continues the face
// lattice (on-site eps, hopping tl inside a layer and between layers, coupling tc per site).
// Mode p of an axis of extent d: phi_p(j) = sqrt(2 / (d + 1)) sin(pi (p+1) (j+1) / (d + 1)),
// 0-based p, j; tab[j * d + p].
struct FaceJob {
  int32_t e;                 // energy slot
  int32_t d1, d2, F;         // F = d1 d2 = rows of the face cluster
  double eps, tl, tc;
  const double* tab1;        // [d1][d1]
  const double* tab2;        // [d2][d2]
  const int32_t* jk;         // [F] row of the face cluster -> j * d2 + k
  double2* half;             // [d1][d2][d2] partial mode sums
  double2* sigma;            // [F][F] self-energy, rows/cols in the face cluster's order
  void* gamma;               // [F][F] Gamma = -2 Im Sigma: double2 (re, 0) or zdd
  int32_t gamma_dd;
};
// half[p][k][k'] = sum_q phi_q(k) phi_q(k') g_pq(z)   (g_pq: surface function of mode (p, q))
void launch_face_half(hipStream_t st, const FaceJob* jobs, int njobs, int max_d1, int max_d2,
                      const EnergyScalars* es);
// sigma[a][b] = tc^2 sum_p phi_p(j_a) phi_p(j_b) half[p][k_a][k_b]; gamma = -2 Im sigma
void launch_face_sigma(hipStream_t st, const FaceJob* jobs, int njobs, int max_f);
// T[e_base + slot] = sum_{a,b} Gamma_L[a][b] Im P[a][b] over the left face block of the right
// channel's lesser block P (= i A_R there); accumulated in double-double
struct FaceTransJob {
  const void* gamma;         // Gamma_L of the slot (layout as FaceJob::gamma)
  const void* P;             // left face's diagonal block of i A_R (double2 or zdd), leading dim ldp
  int32_t F, ldp, dd;
};
void launch_face_trans(hipStream_t st, const FaceTransJob* jobs, int nvalid, int e_base, double* trans);

// ---- bond entries of G^r and G^< (off-diagonal entries on the bonds of H) ----
// Source of one bond entry, fixed per plan: cluster c, own row a, and
//   mode 0 (separator or root): X[a][col] of its G block (GX, columns colg) or lesser block
//          (PX, columns colp);
//   mode 1 (leaf, both sites its own, col = b): G = Inv_ab + sum_j Psi_aj GT_bj,
//          P = M_ab - sum_j Psi_aj conj(PT_bj)  (M absent: 0);
//   mode 2 (leaf, front site k = col): G = GT_ak, P = PT_ak.
// flip: the bond (i, j) is the transpose of the stored (row, col): G^r is symmetric (same value),
// G^< anti-Hermitian (-conj).
struct BondRef {
  int32_t c, a, colg, colp, mode, flip;
};
// blocks of one (cluster, slot) a bond entry reads (element type double2 or zdd)
struct BondSrc {
  const void* X;      // mode 0: GX / PX; leaves: unused
  const void* d;      // leaves: A_ii^-1 (G) or M (P, may be null)
  const void* psi;    // leaves: Psi (n x f)
  const void* xt;     // leaves: GT / PT (n x f)
  int32_t ld, n, f, ldd;
};
// out[(e_base + slot) * nbonds + b] for slots < nvalid; lesser = 1 applies the anti-Hermitian flip
void launch_bonds(hipStream_t st, const BondRef* refs, int nbonds, const BondSrc* src, int nslots, int nvalid,
                  int e_base, int lesser, int dd, double2* out);

// Batched blocked Gauss-Jordan inversion.
void launch_inv_panel(hipStream_t st, const InvJob* jobs, int njobs, int k0, int nb, int max_n,
                      int32_t* status);
void launch_inv_swap(hipStream_t st, const InvJob* jobs, int njobs, int k0, int nb, int max_n);
void launch_inv_unscramble(hipStream_t st, const InvJob* jobs, int njobs, int max_n);
void launch_inv_super(hipStream_t st, const InvJob* jobs, int njobs, int s0, int W, int max_n);

// guard[(e_base + slot) * nclusters + cluster][0..1] = ||Inv||_inf, ||Psi||_inf (one block per job)
void launch_guard(hipStream_t st, const RowJob* jobs, int njobs, int nclusters, int e_base, int nvalid,
                  double* out);

// ---- double-double fold (see dd.h) ----
struct zdd;
// Batched Gauss-Jordan in double-double: in place on X (zdd, ld); the inverse
// goes to Y (zdd, ldy) and, rounded, to Y64 (complex128, ldy64).
struct InvJobDD {
  zdd* X;
  zdd* Y;
  double2* Y64;
  int32_t n, ld, ldy, ldy64;
  int32_t e;
  int32_t* piv;
  zdd* T;
  zdd* R;
};
// D = sign * op(A) op(B) + beta * C in double-double; D64 (optional) = round(D).
struct GemmProbDD {
  const zdd* A;
  const zdd* B;
  const zdd* C;
  zdd* D;
  double2* D64;
  int32_t M, N, K;
  int32_t lda, ldb, ldc, ldd, ldd64;
  int32_t tiles_n;
  int32_t tile_off;
};
// tile configurations of the double-double GEMM: 0 = 32x32, 1 = 64x32, 2 = 64x64 (rows x columns)
int dd_gemm_configs();
int dd_gemm_tile_m(int config);
int dd_gemm_tile_n(int config);
void launch_dd_gemm(hipStream_t st, int opA, int opB, int config, const GemmProbDD* probs,
                    const int32_t* tile_prob, int total_tiles, int negate, int beta);
// extraction row kernels in double-double: RowJob.src / dst / p0 / p1 and ChildRef.U point to zdd;
// same arguments as launch_gather, launch_assemble_n and launch_diag (outputs rounded to complex128)
void launch_dd_gather(hipStream_t st, const RowJob* jobs, const int32_t* row_job, int total_rows, int trans, int op);
void launch_dd_assemble_n(hipStream_t st, const RowJob* jobs, const int32_t* row_job, int total_rows,
                          const EnergyScalars* es, int channel);
void launch_dd_diag(hipStream_t st, const RowJob* jobs, const int32_t* row_job, int total_rows, int mode,
                    int out_kind, void* out, int64_t out_stride, int e_base, int nvalid);
// frontal assembly in double-double (RowJob.dst and ChildRef.U point to zdd)
void launch_dd_assemble(hipStream_t st, const RowJob* jobs, const int32_t* row_job, int total_rows,
                        const EnergyScalars* es);
void launch_dd_inv_panel(hipStream_t st, const InvJobDD* jobs, int njobs, int k0, int nb, int max_n,
                         int32_t* status);
void launch_dd_inv_swap(hipStream_t st, const InvJobDD* jobs, int njobs, int k0, int nb, int max_n);
void launch_dd_inv_unscramble(hipStream_t st, const InvJobDD* jobs, int njobs, int max_n);
// two-level Gauss-Jordan: T = super-panel columns minus identity (row stride W), R = its pivot rows
void launch_dd_inv_super(hipStream_t st, const InvJobDD* jobs, int njobs, int s0, int W, int max_n);
int dd_inv_nb(int max_n);
// columns of a super-panel of the double-double Gauss-Jordan (its pivot rows update the rest at once)
constexpr int kDDSuper = 64;

// ---- double-double products from 8-bit slices on the integer matrix cores (ozaki.hip) ----
// slices per operand: S = 16 (the default) keeps each double-double operand to 2^-112 of its row's
// (or column's) largest entry, S = 15 to 2^-105
constexpr int kOzSlices = 16;
constexpr int kOzSlicesMin = 15, kOzSlicesMax = 16;
// deepest slice product: the int32 accumulator of one weight sums up to 3 Gauss parts x S pairs x
// 64^2 x Kp, which must stay below 2^31
constexpr int oz_max_depth(int slices) { return (int)(((1ll << 31) - 1) / (3ll * slices * 64 * 64) / 64 * 64); }
// One operand to split: element (r, k) = X[r * ldr + k * ldk] for r < R, k < K (complex
// double-double); out = 3 x S planes (Re, Im, Re + Im) of Rp x Kp int8 in 1 KB fragments of
// 16 rows x 64 k (matrix-core operand order), ex = [Rp] row exponents; Rp a multiple of 32 (>= R),
// Kp of 64 (>= K); zero padding.  Row-scale workgroups [blk_off, blk_off + ceil(Rp / 64)) and digit
// workgroups [tile_off, tile_off + ceil(Rp / 64) * Kp / 32) of a split launch belong to this job.
struct OzSplitJob {
  const zdd* X;
  int64_t ldr, ldk;
  int32_t R, K, Rp, Kp;
  int8_t* out;
  int32_t* ex;
  int32_t blk_off, tile_off;
};
// One product D = (-1)^negate A' B' + beta C from split operands (A8: rows of A', B8: columns of
// B'); 32 x 32 output tiles.
struct GemmProbOZ {
  const int8_t* A8;
  const int8_t* B8;
  const int32_t* ea;
  const int32_t* eb;
  const zdd* C;
  zdd* D;
  double2* D64;
  int32_t M, N, Mp, Np, Kp;
  int32_t ldc, ldd, ldd64;
  int32_t tiles_n, tile_off;
};
// slices: kOzSlicesMin..kOzSlicesMax, the same for the split and the product of one operand pair
void launch_oz_split(hipStream_t st, int slices, const OzSplitJob* jobs, const int32_t* blk_job, int total_blocks,
                     const int32_t* tile_job, int total_tiles);
void launch_oz_gemm(hipStream_t st, int slices, const GemmProbOZ* probs, const int32_t* tile_prob, int total_tiles,
                    int negate, int beta);
// the allocation-free product: a static device array of kOzNoAllocScratch bytes per device holds
// descriptors, maps, slices and exponents of one problem (oz_noalloc_bytes of them)
constexpr size_t kOzNoAllocScratch = size_t(64) << 20;
void* oz_noalloc_scratch_address();
size_t oz_noalloc_bytes(int M, int N, int K);
int launch_oz_gemm_noalloc(hipStream_t st, char* ws, int opA, int opB, int M, int N, int K, int negate,
                           const void* A, int lda, const void* B, int ldb, int beta, const void* C, int ldc, void* D,
                           int ldd);

// debug / unit-test helpers
void launch_mfma_rate(hipStream_t st, double* out, int blocks, int iters);
void launch_mfma_probe(hipStream_t st, double* out);

// ---- self-consistent NEGF-Poisson loop (poisson.hip) ----
// pot[p] = U[perm[p]] (U in site order, pot in cluster order), zeros without U
void launch_potential(hipStream_t st, int64_t n, const int64_t* perm, const double* U, double* pot);
// dens[i] = sum_e w[e] Im G^<_ii(E_e) / (2 pi); gl: complex128 [ne][n]
void launch_density(hipStream_t st, int ne, int64_t n, const double* w, const void* gl, double* dens);
// *r = max_i |u_new - u| (bits of a non-negative double), then u += beta (u_new - u)
void launch_mix(hipStream_t st, int64_t n, double* u, const double* u_new, double beta, unsigned long long* r);
// Anderson mixing: f = u_new - u with its max |f_i| in *r; the history difference (dX, dF may be null) and the
// previous (u, f); the update u = u + beta f - sum_j gamma_j (dX_j + beta dF_j) over the slots in `order`
constexpr int kScfMaxHistory = 16;
// most streams one solve call runs its batches on
constexpr int kMaxStreams = 8;
void launch_scf_resid(hipStream_t st, int64_t n, const double* u, const double* u_new, double* f,
                      unsigned long long* r);
void launch_scf_hist(hipStream_t st, int64_t n, const double* u, const double* f, double* u_prev, double* f_prev,
                     double* dX, double* dF);
void launch_scf_update(hipStream_t st, int64_t n, double* u, const double* f, double beta, int mk, const double* dX,
                       const double* dF, const int32_t* order, const double* gamma);
constexpr int kPoissonMaxSide = 1024;
// 0 when the grid is usable (sides in [1, kPoissonMaxSide], finite lead-plane values), else -1
// with the reason
int poisson_check(const hsc_grid* g, std::string* why);
// device workspace of the fast Poisson solve on one grid: two arrays of n doubles, the three
// closed-form bases and their eigenvalues
struct PoissonWork {
  hsc_grid grid{};
  int64_t n = 0;
  double* buf = nullptr;
  double *t1 = nullptr, *t2 = nullptr;
  const double* Q[3] = {};
  const double* lam[3] = {};
  int create(const hsc_grid& g);   // 0 or -1 (allocation or copy failed)
  void destroy();
  // u = the solution for the source rho, or, when dens is given, for coupling (dens - n0)
  // (n0 may be null); enqueued on st
  void run(hipStream_t st, const double* rho, const double* dens, const double* n0, double coupling, double* u) const;
};

}  // namespace hsc
