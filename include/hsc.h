/*
 * hsc.h -- C ABI of the MI355X nested-dissection NEGF solver (HSC + HSC-extension).
 *
 * For a device Hamiltonian H (sparse, complex symmetric: H^T == H) with two
 * contacts, and for each energy E, the library computes
 *
 *   diag G^r(E),  G^r = A^-1,  A = (E + i eta) I - H - Sigma_L - Sigma_R       (Eq. 1)
 *   diag G^<(E),  G^< = G^r Sigma^< (G^r)^dagger,                              (Eq. 2)
 *                 Sigma^< = i (f_L Gamma_L + f_R Gamma_R)
 *   T(E) = Tr[Gamma_L G^r Gamma_R (G^r)^dagger]
 *
 * with Algorithm 1 (HSC: fold, root inverse, extract of G^r) and Algorithm 2
 * (HSC-extension: N = Sigma^< (G^r)^dagger, fold of N, extract of P = G^<) over
 * a binary cluster tree from multilevel nested dissection (Section 2.2).
 *
 * Conventions shared by every entry point:
 *   - Every call returns hsc_status; 0 is success, negative values are errors.
 *     hsc_last_error() returns a text description of the calling thread's last
 *     error (valid until the next failing call on that thread).
 *   - "host" pointers are ordinary CPU memory, read during the call only.
 *     "device" pointers are HIP device memory owned by the caller (for example a
 *     torch tensor's data_ptr()); the library never frees them.
 *   - Complex numbers are two doubles (re, im) adjacent in memory.
 *   - Site order in every output is the caller's site order (the order of H).
 *   - Solves are asynchronous on the context's HIP stream.  Output buffers are
 *     valid after hsc_sync() or after the caller synchronises that stream.
 */
#ifndef HSC_H_
#define HSC_H_

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  HSC_OK = 0,
  HSC_E_ARG = -1,           /* invalid argument (null pointer, bad size, bad index) */
  HSC_E_NOT_SYMMETRIC = -2, /* H^T != H: the method uses transposes (Alg. 1), not adjoints */
  HSC_E_SINGULAR = -3,      /* an exactly singular pivot block was met */
  HSC_E_NONFINITE = -4,     /* NaN or Inf in the input or the factors */
  HSC_E_OOM = -5,           /* device or host allocation failed */
  HSC_E_HIP = -6,           /* a HIP runtime call failed */
  HSC_E_UNSTABLE = -7       /* growth guard still above threshold after re-planning */
} hsc_status;

/* Output selection bits for hsc_solve_opts.want. */
enum {
  HSC_DIAG_GR = 1,        /* diag G^r                                          */
  HSC_DIAG_GL = 2,        /* diag G^< for Sigma^< = i(f_L Gamma_L + f_R Gamma_R) */
  HSC_TRANS = 4,          /* transmission T(E)                                 */
  HSC_SPECTRAL_LR = 8,    /* diag of A_L = G Gamma_L G^dagger and A_R, separately */
  /* The desired off-diagonal entries (Section 3: the timed quantities are the diagonal and the
   * desired off-diagonal entries of G^r and G^<): the entries on every bond of H, i.e. every
   * pair (i, j), i < j, with H_ij != 0, in the order of hsc_tree_bonds.  Bond currents follow
   * from G^<_ij and H_ij.  Requested through hsc_solve_ex. */
  HSC_BOND_GR = 16,       /* G^r_ij on every bond                              */
  HSC_BOND_GL = 32        /* G^<_ij on every bond (G^<_ji = -conj(G^<_ij))      */
};

typedef struct hsc_ctx hsc_ctx;   /* one HIP device + one stream + workspaces; not thread-safe */
typedef struct hsc_tree hsc_tree; /* cluster tree of one device; immutable after build        */

/* One contact: a list of device sites and the parameters of its lead.
 * Per-site leads (tree option dense_contacts = 0): each site couples (hopping
 * `coupling`) to its own semi-infinite 1D lead with on-site `lead_onsite` and
 * hopping `lead_hopping` -- the diagonal contact self-energy of the paper's
 * SPARSE case (Section 3.1.1).
 * Whole-face leads (dense_contacts = 1): the sites are one whole face of the
 * device, a full rectangle of a plane normal to the transport axis, and the
 * lead is the semi-infinite continuation of that face: every lead layer is a
 * copy of the face lattice (on-site `lead_onsite`, nearest-neighbour hopping
 * `lead_hopping` inside the layer and to the next layer), each face site
 * coupled to its copy by `coupling`.  The self-energy is then a dense
 * |face| x |face| block -- the paper's DENSE case (Section 3.1.2; the
 * open-boundary caveat of Section 2.3). */
typedef struct {
  int64_t n_sites;
  const int64_t* sites;      /* host, [n_sites] site indices in [0, n) */
  double lead_onsite;
  double lead_hopping;
  double coupling;
} hsc_contact;

/* Geometric nested dissection (Section 2.2, multilevel nested dissection):
 * split the longest splittable axis of the cluster's bounding box with a
 * one-site-thick plane at lo + floor(extent / 2); stop when every splittable
 * extent is <= leaf_side (or < 3).  split_mask bit a allows axis a.
 * The separating property is verified against the graph of H. */
typedef struct {
  const int32_t* coords;     /* host, [n][3] integer site coordinates */
  int32_t split_mask;        /* e.g. 7 for x|y|z, 3 for in-plane only */
  int32_t leaf_side;         /* >= 1 */
  int32_t method;            /* 0: geometric nested dissection from coords (above);
                              * 1: graph nested dissection from the sparsity of H alone, for
                              * unstructured H (coords may be NULL): breadth-first level sets
                              * from a pseudo-peripheral site, the level that best balances the two
                              * sides is the separator; leaf_side is then the largest leaf in sites */
  int32_t dense_contacts;    /* 0: per-site leads; 1: whole-face leads (dense self-energy).
                              * With 1 the two contacts must be the two end planes of the
                              * device along one axis (every site between them), each a full
                              * rectangle in the other two axes; each face becomes a cluster of
                              * its own, above the dissection of its half: the root is the middle
                              * plane (devices at least 4 planes long), else the left face heads
                              * a chain.  Such trees are not merged or put into forests. */
} hsc_tree_opts;

typedef struct {
  int64_t n_sites;
  int32_t n_clusters;
  int32_t depth;             /* number of levels (root level is 0) */
  int32_t max_cluster;       /* max n_i */
  int32_t max_front;         /* max |front(i)| */
  int32_t max_ancestors;     /* max |P_i| (sites), over clusters on contact paths */
  int32_t n_leaves;
  double flops_per_energy;   /* real flops of one energy (complex FMA = 8), all outputs */
  double bytes_per_energy;   /* device working set of one energy */
} hsc_tree_stats;

typedef struct {
  double eta;                /* z = E + i*eta, > 0 */
  double kT;                 /* Fermi temperature, > 0 (same unit as E) */
  double mu_L, mu_R;         /* contact chemical potentials */
  uint32_t want;             /* HSC_* bits */
  int32_t batch;             /* energies per launch sequence; 0 = as many as 70 % of the free
                              * device memory holds (at most 64), spread evenly over the batches */
  /* Growth guard.  Algorithm 1 inverts each cluster block A_ii with no
   * pivoting across clusters; a nearly singular block amplifies rounding
   * errors.  When guard_tau > 0, every energy whose non-root clusters have
   * ||Psi_i||_inf > guard_tau is solved again on a tree in which those
   * clusters are merged into their parents (a delayed pivot), for up to
   * guard_rounds rounds; energies still above the threshold get status
   * HSC_E_UNSTABLE.  With guard_tau > 0 the call waits for the device. */
  double guard_tau;          /* 0 disables the guard */
  int32_t guard_rounds;      /* maximum re-planning rounds (e.g. 6) */
  /* Arithmetic of the solve:
   * 0 = complex128 throughout (Algorithms 1 and 2 as written, on the FP64
   *     matrix cores);
   * 1 = double-double fold (block inverses, multipliers Psi, Schur updates in
   *     about 106-bit significands on the FP64 vector units); the extraction
   *     of Algorithm 2 and the lesser channels stay complex128;
   * 2 = double-double fold and extraction: every block of G, of the lesser
   *     channels and their products is carried in double-double and only the
   *     returned diagonals are rounded to complex128;
   * 3 = as 2, with every double-double block product of depth K >= 32 formed
   *     on the integer matrix cores: each operand is split into 16 signed
   *     8-bit slices (`slices` below) scaled by a power of two per row (per
   *     column of the right operand), to 2^-112 of the row's largest entry,
   *     the slice products are summed exactly in 32-bit integers, and the pairs
   *     whose weight is within 2^-105 of the leading one are combined in
   *     double-double (at most about K 2^-104 times the product of the largest
   *     row and column entries; products with K < 32, the
   *     pivot-block inverse updates among them, stay on the vector units).
   *     Needs a slice scratch of up to 4 GiB besides the workspace.
   * The unpivoted cluster elimination amplifies rounding errors by up to
   * ~1/sigma_min(A_ii)^2 at energies where a cluster block A_ii is nearly
   * singular (outside the lead band, where nothing broadens it): in the fold
   * (1 removes that share) and in the extraction G_ii = A_ii^-1 + Psi G_fi, a
   * difference of large terms (2 removes that share as well).  2 needs twice
   * the workspace of 0 for G. */
  int32_t precision;
  /* 1: record the launch sequence of one batch of energies once as a HIP graph
   * (its outputs go to staging rows owned by the plan) and replay it for every
   * batch, copying the rows out; 0: launch step by step.  Ignored when the
   * guard is on or launch timing is enabled. */
  int32_t graph;
  /* 1: when the plan for (tree, batch, outputs, precision) is first built, time
   * every tile shape of the grouped GEMM (64x64, 128x64, 64x128, 32x32 and,
   * over 8 waves, 128x128 on the 16x16x4 MFMA; 64x64 on the 4x4x4 MFMA) on each
   * of its launches and keep the fastest per launch; 0: 64x64 everywhere.  With
   * complex3m = 1 the candidates are the three-product kernels plus the 128x128
   * four-product one.  Double-double products (precision >= 1) are timed with
   * 32x32, 64x32 and 64x64 tiles (untuned: 64x32).  Results agree to rounding. */
  int32_t tune;
  /* Complex block products: 0 = four real products per complex multiply-add
   * (Re = ArBr - AiBi, Im = ArBi + AiBr); 1 = three (Gauss: ArBr, AiBi,
   * (Ar+Ai)(Br+Bi)), a quarter less matrix-core work with an imaginary-part
   * error bound proportional to (|Ar| + |Ai|)(|Br| + |Bi|). */
  int32_t complex3m;
  /* precision 3: 8-bit slices per operand of the integer-matrix-core products.
   * 0 = 16 (the default), or 16 or 15: fifteen keep every operand to 2^-105
   * instead of 2^-112 of its row's largest entry (a product bound of about
   * K 2^-97 instead of K 2^-104 times the row and column maxima) for 120
   * instead of 136 slice pairs, about 6 % less solve time; entries far below
   * their row's largest (large devices out of the lead band) then lose up to
   * two more digits.  Ignored with precision 0-2.  Other values: HSC_E_ARG. */
  int32_t slices;
  /* On-site potential energy U (device, double[n], site order of the tree's H),
   * or NULL: the device Hamiltonian becomes H + diag(U) (the electrostatic
   * potential of a self-consistent NEGF-Poisson loop; the leads keep their own
   * on-site energies).  Read when the call enqueues its first launch; single-
   * device solves only (hsc_solve_batch returns HSC_E_ARG for a non-NULL U).
   * The values must be finite (they are not checked; a NaN typically ends as
   * HSC_E_SINGULAR in the energy's status). */
  const double* potential;
  /* Concurrent batches.  0 or 1: the batches of a call run one after another on
   * the context's stream.  k in [2, 8]: they run round-robin on k streams of
   * the context (created on first use, default priority), each with a plan and
   * workspace of its own (`batch` slots each, so k times the memory of one
   * plan), forked from and joined back to the context's stream: the call stays
   * ordered on that stream as before.  The drain of one batch's launches then
   * overlaps another's: on a 32^3 cube two streams of 8 energies run 3 % faster
   * than one stream of 16, four of 4 are 3 % slower.  Effective only when the
   * call has more energies than one
   * batch; one stream while launch profiling is on, with the growth guard and
   * with bond outputs.  Other values: HSC_E_ARG. */
  int32_t streams;
} hsc_solve_opts;

/* Library version string. */
const char* hsc_version(void);
const char* hsc_last_error(void);
/* The same text for callers holding a context (the message of the calling thread's last failed
 * call, on this context or not; ctx may be NULL). */
const char* hsc_ctx_last_error(const hsc_ctx* ctx);

/* Create a context on HIP device `device`.  `hip_stream` is a hipStream_t
 * (for example torch.cuda.current_stream().cuda_stream) or NULL for the null
 * stream.  Errors: HSC_E_ARG, HSC_E_HIP. */
hsc_status hsc_ctx_create(int32_t device, void* hip_stream, hsc_ctx** out);
hsc_status hsc_ctx_destroy(hsc_ctx* ctx);

/* Build the nested-dissection cluster tree of one device (host work only; the
 * device copy is made by the first solve).  H is CSR with n rows: indptr[n+1]
 * (int64), indices[nnz] (int32), values_ri[2*nnz] interleaved (re, im), all
 * host.  Exactly two contacts: contacts[0] = left, contacts[1] = right; a site
 * may belong to at most one contact.  Errors: HSC_E_ARG (bad CSR, indices,
 * contacts or opts), HSC_E_NOT_SYMMETRIC, HSC_E_NONFINITE, HSC_E_OOM. */
hsc_status hsc_tree_build(int64_t n, const int64_t* indptr, const int32_t* indices,
                          const double* values_ri, int32_t n_contacts,
                          const hsc_contact* contacts, const hsc_tree_opts* opts,
                          hsc_tree** out);

/* A tree of the caller's own partition (Section 2.2: any cluster tree whose separators separate;
 * a chain of slabs makes the method the recursive Green's function of Section 2.1; the DNA study's
 * customised partitions): cluster_of_site[s] in [0, n_clusters) and parent[c] (-1 for the one
 * root).  Clusters are renumbered children-first (hsc_tree_export gives the new order), every
 * cluster must be non-empty, and every bond of H must join a cluster and one of its ancestors
 * (checked).  Contacts as in hsc_tree_build with per-site leads.
 * Errors: HSC_E_ARG (bad partition, not a tree, not separating), HSC_E_NOT_SYMMETRIC,
 * HSC_E_NONFINITE, HSC_E_OOM. */
hsc_status hsc_tree_build_custom(int64_t n, const int64_t* indptr, const int32_t* indices,
                                 const double* values_ri, int32_t n_contacts, const hsc_contact* contacts,
                                 int32_t n_clusters, const int32_t* cluster_of_site, const int32_t* parent,
                                 hsc_tree** out);

/* A copy of `src` in which every listed cluster (ids as numbered by
 * hsc_tree_export) is merged into its parent: the parent takes its sites and
 * children.  Merging removes the unpivoted elimination of that cluster's block
 * on its own.  The root cannot be merged.  Errors: HSC_E_ARG. */
hsc_status hsc_tree_merge(const hsc_tree* src, int32_t n_ids, const int32_t* ids,
                          hsc_tree** out);

/* A forest of several devices (Section 2.2 trees side by side): the clusters of
 * trees[0], trees[1], ... in that order, sites numbered device after device.
 * Solving the forest solves every device at once, each device's clusters of a
 * level sharing the batched launches of that level.  All devices must use the
 * same lead model (HSC_E_ARG otherwise); total sites < 2^31.  The new tree
 * copies what it needs: the inputs may be destroyed afterwards. */
hsc_status hsc_tree_concat(int32_t n_trees, const hsc_tree* const* trees, hsc_tree** out);

hsc_status hsc_tree_stats_get(const hsc_tree* tree, hsc_tree_stats* out);

/* Bonds of H: every pair (i, j), i < j, with a stored entry H_ij, ordered by i then j
 * (duplicates of a pair count once).  With pairs == NULL only *count is set; otherwise pairs
 * (host, int64[count][2]) receives them and *count must hold its capacity in pairs on entry.
 * Errors: HSC_E_ARG (NULL tree or count, capacity too small). */
hsc_status hsc_tree_bonds(const hsc_tree* tree, int64_t* pairs, int64_t* count);

/* Export the tree (host buffers, sized from hsc_tree_stats_get):
 *   perm[n]            site at position p of the cluster ordering (post-order)
 *   cl_parent[nc]      parent cluster id (-1 for the root); ids are post-order
 *   cl_first[nc]       first position of the cluster's sites in perm
 *   cl_size[nc]        n_i
 *   front_ptr[nc+1]    offsets into front_sites
 *   front_sites[...]   point-level front of each cluster (original site ids),
 *                      in cluster-ordering position order.
 * Any pointer may be NULL to skip that array; front_sites needs front_ptr[nc]
 * entries.  Errors: HSC_E_ARG. */
hsc_status hsc_tree_export(const hsc_tree* tree, int64_t* perm, int32_t* cl_parent,
                           int32_t* cl_first, int32_t* cl_size, int64_t* front_ptr,
                           int64_t* front_sites);
hsc_status hsc_tree_destroy(hsc_tree* tree);

/* Solve n_e energies of one device.
 *   energies     device, double[n_e] (real energies)
 *   diag_gr      device, complex[n_e][n]   (HSC_DIAG_GR) or NULL
 *   diag_gl      device, complex[n_e][n]   (HSC_DIAG_GL) or NULL
 *   trans        device, double[n_e]       (HSC_TRANS) or NULL
 *   spectral_lr  device, double[n_e][2][n] (HSC_SPECTRAL_LR: A_L then A_R) or NULL
 *   status       device, int32[n_e] per-energy status (0 or a negative code) or NULL
 *   guard        device, double[n_e][n_clusters][2] or NULL: for every pivot block
 *                A_ii of Algorithm 1, ||(A_ii)^-1||_inf and ||Psi_i||_inf (max row
 *                sums of moduli: conditioning and growth of the unpivoted cluster
 *                elimination; clusters in hsc_tree_export order)
 * Outputs whose bit is not set in opts->want are not written.
 * Errors: HSC_E_ARG, HSC_E_OOM, HSC_E_HIP.  Numerical failures of single
 * energies are reported through `status` (see hsc_sync). */
hsc_status hsc_solve(hsc_ctx* ctx, const hsc_tree* tree, int32_t n_e, const double* energies,
                     const hsc_solve_opts* opts, void* diag_gr, void* diag_gl, double* trans,
                     double* spectral_lr, int32_t* status, double* guard);

/* Outputs of hsc_solve_ex: the buffers of hsc_solve plus the bond entries.
 *   bond_gr, bond_gl  device, complex[n_e][n_bonds] (HSC_BOND_GR / HSC_BOND_GL) or NULL; entry
 *                     b of row e belongs to bond b of hsc_tree_bonds. */
typedef struct {
  void* diag_gr;
  void* diag_gl;
  double* trans;
  double* spectral_lr;
  int32_t* status;
  double* guard;
  void* bond_gr;
  void* bond_gl;
} hsc_outputs;

/* hsc_solve with every output, the bond entries included.  Bond outputs are read from the blocks
 * the two algorithms already form: a bond inside a separator (or root) from its diagonal block
 * of G^r (Algorithm 1 extract) or of the combined lesser channel (Algorithm 2 extract); a bond
 * between a cluster and an ancestor from the cluster's (own, front) block; a bond inside a leaf
 * from A_ii^-1 + Psi G_f,i (resp. A_ii^-1 N_ii - Psi P_i,f^dagger) evaluated for that entry.
 * Bond outputs do not combine with the growth guard (HSC_E_ARG) and switch graph replay off.
 * Errors as hsc_solve. */
hsc_status hsc_solve_ex(hsc_ctx* ctx, const hsc_tree* tree, int32_t n_e, const double* energies,
                        const hsc_solve_opts* opts, const hsc_outputs* out);

/* Solve several devices in one call.  Arrays are indexed by device; entries
 * follow hsc_solve.  When every device has the same energy list, the same
 * per-site lead model and the guard is off, consecutive devices are packed into forests
 * (hsc_tree_concat) whose workspace per energy slot fits about a ninth of the
 * free device memory: one plan per forest, every level's clusters of all its
 * devices in the same launches, outputs staged in device memory and copied to
 * each device's buffers; a numerical failure at an energy is then reported in
 * the status of every device of that forest.  A device too large to share is
 * solved alone, and with differing energy lists the devices are solved one
 * after another.  Errors as hsc_solve. */
hsc_status hsc_solve_batch(hsc_ctx* ctx, int32_t n_trees, const hsc_tree* const* trees,
                           const int32_t* n_e, const double* const* energies,
                           const hsc_solve_opts* opts, void* const* diag_gr,
                           void* const* diag_gl, double* const* trans,
                           double* const* spectral_lr, int32_t* const* status,
                           double* const* guard);

/* Wait for the context's stream (and the context's streams of concurrent batches, see
 * hsc_solve_opts.streams); returns HSC_E_HIP on an asynchronous HIP error. */
hsc_status hsc_sync(hsc_ctx* ctx);

/* Per-energy sums over sites of solve outputs (Section 2: density of states from
 * G^r, electron density from G^<, hbar = 1, no spin factor):
 *   totals[e][0] = -(1/pi)  sum_i Im G^r_ii(E_e)              (DOS)
 *   totals[e][1] =  (1/2pi) sum_i Im G^<_ii(E_e)              (electrons per unit energy)
 *   totals[e][2] =  (1/2pi) sum_i (A_L + A_R)_ii(E_e)         (DOS injected by the contacts)
 * diag_gr, diag_gl: device, complex128 [n_e][n]; spectral_lr: device, double
 * [n_e][2][n]; all as written by hsc_solve.  Any of them may be NULL; its column of
 * totals (device, double [n_e][3]) is then not written.
 * Errors: HSC_E_ARG for n_e < 0, n < 0 or a NULL totals with n_e > 0. */
hsc_status hsc_totals(hsc_ctx* ctx, int32_t n_e, int64_t n, const void* diag_gr, const void* diag_gl,
                      const double* spectral_lr, double* totals);

/* ---- self-consistent NEGF-Poisson loop ----
 * The paper presents the method as the costly half of self-consistent NEGF-Poisson
 * simulations (abstract, Section 1) without fixing the electrostatics; these
 * calls supply a plain one on the device grid.
 *
 * Grid: site (x, y, z) of an nx x ny x nz cuboid has index x + nx (y + ny z) (the
 * layout of the benchmark cuboids); x is the transport axis.  Poisson operator,
 * unit spacing, 7 points: sum over the three axes of (2 U_i - U_prev - U_next);
 * the outside neighbour along x is a lead plane (x = -1 at u_left, x = nx at
 * u_right: Dirichlet), along y and z the site itself (zero normal derivative). */
typedef struct {
  int32_t nx, ny, nz;        /* each in [1, 1024] */
  double u_left, u_right;    /* potential energy of the lead planes */
} hsc_grid;

/* u = the solution of (Poisson operator) u = rho + lead-plane terms, by the
 * closed-form eigenbases of the three 1D operators (exact up to FP64 rounding).
 * rho, u: device double[nx ny nz] (may not overlap).  Synchronous.
 * Errors: HSC_E_ARG (sides out of range, non-finite lead values, NULL arrays),
 * HSC_E_OOM, HSC_E_HIP. */
hsc_status hsc_poisson_solve(hsc_ctx* ctx, const hsc_grid* grid, const double* rho, double* u);

/* Electron density per site (no spin factor, hbar = 1) from the diagonal of
 * G^< (Eq. 2): density[i] = sum_e weights[e] Im G^<_ii(E_e) / (2 pi), the
 * energies summed in order.  weights: device double[n_e] (the caller's
 * quadrature weights); diag_gl: device complex128 [n_e][n] as hsc_solve writes
 * it; density: device double[n].  Asynchronous on the context's stream.
 * Errors: HSC_E_ARG. */
hsc_status hsc_density(hsc_ctx* ctx, int32_t n_e, int64_t n, const double* weights, const void* diag_gl,
                       double* density);

typedef struct {
  double coupling;           /* c of the source rho = c (n - n0) (e^2 / epsilon in model units), >= 0 */
  const double* n0;          /* device double[n] background density, or NULL (zero) */
  double mixing;             /* beta in (0, 1]: U <- U + beta (U_new - U) */
  int32_t max_iter;          /* >= 1 */
  double tol;                /* stop after the iteration whose residual max|U_new - U| < tol; 0: max_iter */
  int32_t history;           /* 0: linear mixing; m in [1, 16]: Anderson mixing over the last m steps
                              * (Anderson 1965, in the form of Walker and Ni 2011): with f_k = U_new - U_k
                              * and the last m differences dX, dF of U and f, gamma = argmin
                              * ||f_k - dF gamma||_2 (Householder QR on the host), U_k+1 = U_k + beta f_k
                              * - (dX + beta dF) gamma; the history is cleared when R is numerically
                              * singular (a diagonal entry below 1e-12 of the largest) */
} hsc_scf_opts;

/* The loop: for each iteration, solve every energy with potential u (hsc_solve
 * with opts, diag G^< only), density as hsc_density, source c (n - n0),
 * U_new = hsc_poisson_solve(source), residual max_i |U_new - u|, then
 * u <- u + beta (U_new - u).  u: device double[n], the starting potential on
 * entry and the last mixed (or Anderson-updated) one on return; density: device double[n], the density
 * of the last solve (at the potential before the last mixing); energies,
 * weights: device double[n_e]; *iterations (host) = iterations run; residuals
 * (host double[max_iter], may be NULL) = residual of each.  The tree must have
 * one site per grid point (n = nx ny nz).  opts->want and opts->potential are
 * ignored.  Synchronous.  Errors: HSC_E_ARG; a solve's per-energy status
 * (HSC_E_SINGULAR, HSC_E_NONFINITE, HSC_E_UNSTABLE) stops the loop and is
 * returned; HSC_E_OOM, HSC_E_HIP. */
hsc_status hsc_scf(hsc_ctx* ctx, const hsc_tree* tree, const hsc_grid* grid, int32_t n_e, const double* energies,
                   const double* weights, const hsc_solve_opts* opts, const hsc_scf_opts* scf, double* u,
                   double* density, int32_t* iterations, double* residuals);

/* Launch timing.  While enabled, every kernel launch of a solve is bracketed by
 * HIP events on the context's stream; hsc_sync() folds the elapsed times into
 * per-kind totals.  Enabling (or disabling) resets the totals.  Kinds:
 * 0 assemble, 1 inverse panel, 2 inverse swap, 3 inverse unscramble, 4 GEMM,
 * 5 gather, 6 N assembly, 7 diagonal output, 8 growth indicators, 9-13 the
 * double-double assemble / panel / swap / unscramble / GEMM, 14 inverse
 * super-panel preparation, 15 operand splitting into 8-bit slices, 16 slice
 * products on the integer matrix cores (precision 3), 17 double-double inverse
 * super-panel preparation, 18-19 the dense self-energy of whole-face contacts
 * (partial mode sums, then the face block), 20 bond entries (HSC_BOND_GR/GL).
 * hsc_ctx_profile_read writes out[3*k + {0,1,2}] = launches, milliseconds,
 * algorithmic real flops (GEMM: 8 M N K per problem) for k < n_kinds.
 * Errors: HSC_E_ARG. */
hsc_status hsc_ctx_profile(hsc_ctx* ctx, int32_t enable);
hsc_status hsc_ctx_profile_read(hsc_ctx* ctx, double* out, int32_t n_kinds);
/* out[k] = algorithmic bytes of the timed launches of kind k since profiling was enabled (so far
 * counted for the slice products, kind 16: slices of both operands read, 3 S B per complex
 * element with S slices per operand; row and column scales; the double-double result written, its rounded copy, and C when
 * accumulating); 0 for kinds not counted.  Errors: HSC_E_ARG. */
hsc_status hsc_ctx_profile_bytes(hsc_ctx* ctx, double* out, int32_t n_kinds);

/* Launch-by-launch record of the timed launches since hsc_ctx_profile(ctx, 1)
 * (after hsc_sync): out[4k] = kind (as in hsc_ctx_profile_read), out[4k+1] =
 * algorithmic flops of the launch, out[4k+2] = its duration in ms, out[4k+3] =
 * the part of the method it belongs to (0 other: energy set-up, growth
 * indicators; 1 pivot-block inverses of Algorithm 1; 2 the rest of the fold of
 * Algorithm 1: frontal assembly, multipliers, Schur updates; 3 extraction of
 * G^r; 4 fold of N in Algorithm 2; 5 extraction of P in Algorithm 2), for the
 * first min(count, max_launches) launches (host buffer of 4 * max_launches
 * doubles); *count receives the number recorded (at most 4,000,000). */
hsc_status hsc_ctx_profile_launches(hsc_ctx* ctx, int64_t max_launches, double* out, int64_t* count);

#ifdef __cplusplus
}
#endif

#endif /* HSC_H_ */
