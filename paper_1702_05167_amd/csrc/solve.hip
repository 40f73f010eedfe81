// Host orchestration of the batched HSC / HSC-extension solve.
//
// For one tree and a batch of B energy slots a Plan fixes, once:
//   * the device workspace layout (frontal matrices, inverses, multipliers,
//     G / N / P frontal blocks per cluster and slot),
//   * every launch of one chunk of B energies, level by level, with its job
//     and tile maps in one device blob.
// A chunk then replays the step list.  Levels are tree depths: the fold and
// the N fold run deepest level first (children before parents), the extracts
// run root first, as in Algorithms 1 and 2.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <map>
#include <memory>
#include <mutex>
#include <tuple>
#include <string>
#include <type_traits>
#include <vector>

#include "dd.h"
#include "hsc_internal.h"
#include "kern.h"
#include "lstsq.h"
#include "../../include/hsc_kernels.h"

namespace hsc {

namespace {

#define HIPCHK(x)                                                                     \
  do {                                                                                \
    hipError_t err_ = (x);                                                            \
    if (err_ != hipSuccess) {                                                         \
      set_error(std::string("HIP error: ") + hipGetErrorString(err_) + " at " #x);    \
      return HSC_E_HIP;                                                               \
    }                                                                                 \
  } while (0)

// Host image of the device blob; pointer fields that refer into the blob are
// stored as offsets and rebased at upload.
struct Blob {
  std::vector<char> data;
  std::vector<size_t> relocs;
  size_t alloc(size_t bytes, size_t align = 64) {
    size_t off = (data.size() + align - 1) / align * align;
    data.resize(off + bytes);
    return off;
  }
  template <class T>
  size_t push(const std::vector<T>& v) {
    size_t off = alloc(std::max<size_t>(1, v.size()) * sizeof(T));
    if (!v.empty()) std::memcpy(data.data() + off, v.data(), v.size() * sizeof(T));
    return off;
  }
  // mark a pointer field (at byte offset `field`) as holding a blob offset
  void reloc(size_t field) { relocs.push_back(field); }
  // pointer fields holding offsets into the plan's slice scratch (double-double products on the
  // integer matrix cores), rebased when the scratch is allocated
  std::vector<size_t> sc_relocs;
};

enum StepKind { S_ASSEMBLE, S_INV_PANEL, S_INV_SWAP, S_INV_UNSCR, S_GEMM, S_GATHER, S_ASSEMBLE_N, S_DIAG, S_GUARD,
                S_DD_ASSEMBLE, S_DD_INV_PANEL, S_DD_INV_SWAP, S_DD_INV_UNSCR, S_DD_GEMM, S_INV_SUPER,
                S_OZ_SPLIT, S_OZ_GEMM, S_DD_INV_SUPER, S_FACE_HALF, S_FACE_SIGMA, S_BONDS};
constexpr int kStepKinds = 21;

// Tile sizes a plan keeps GEMM problem lists and tile maps for: 64x64, 128x64, 64x128, 32x32,
// 128x128.  Every launch kind of launch_gemm uses one of them (tile_dims_of).
constexpr int kTileDims = 5;
constexpr int kTileDimM[kTileDims] = {64, 128, 64, 32, 128};
constexpr int kTileDimN[kTileDims] = {64, 64, 128, 32, 128};

struct Step {
  StepKind kind;
  size_t jobs = 0, map = 0;   // blob offsets
  int count = 0;              // rows / tiles / jobs
  // GEMM: problem list, tile map and tile count for every tile size; `tile` is the launch kind
  size_t jobs_k[kTileDims] = {}, map_k[kTileDims] = {};
  int count_k[kTileDims] = {};
  int tile = 0;
  int njobs = 0;
  int i0 = 0, i1 = 0, i2 = 0, i3 = 0;
  double ar = 1, ai = 0;
  int beta = 0;
  int out = 0;                // DIAG destination
  int dd = 0;                 // row kernels: operands in double-double
  double flops = 0;           // algorithmic real flops of this launch (GEMM: 8 M N K)
  double bytes = 0;           // algorithmic bytes of this launch (slice products: operands read, result written)
  int phase = 0;              // part of the method (Phase), for launch timing
};

// parts of the method a step belongs to (reported with every timed launch)
enum Phase { PH_OTHER = 0, PH_INVERSE = 1, PH_FOLD = 2, PH_EXTRACT_G = 3, PH_FOLD_N = 4, PH_EXTRACT_P = 5 };

enum OutSel { O_GR = 0, O_GL = 1, O_SPEC_L = 2, O_SPEC_R = 3, O_AR_TMP = 4, O_NONE = 5 };

// at most three lesser channels per plan (spectral L and R plus the combined one for bonds)
constexpr int kMaxChannels = 3;

// largest dense cluster block the batched inversion handles (512 threads x 8 rows)
constexpr int kMaxCluster = 4096;

struct Channel {
  int type;      // 0 both contacts (with occupations), 1 left, 2 right
  int fold;      // 0 = lpath||rpath, 1 = lpath, 2 = rpath
  int extract;   // 0 = all clusters, 1 = lpath only
  int out;       // OutSel
};

}  // namespace

struct Plan {
  uint64_t uid = 0;
  int B = 0;
  uint32_t want = 0;
  int prec = 0;
  int tune = 0;
  int m3 = 0;                    // complex products in the three-multiplication form
  int slices = kOzSlices;        // 8-bit slices per operand of the products on the integer matrix cores
  int inst = 0;                  // instance of this shape (one per stream of a call with concurrent batches)
  int64_t n = 0;
  char* ws = nullptr;
  size_t ws_bytes = 0;
  char* blob = nullptr;
  size_t blob_bytes = 0;
  EnergyScalars* es = nullptr;   // [B]
  int32_t* status = nullptr;     // [B]
  double* a_r = nullptr;         // [B][n] (transmission temp)
  int64_t* left = nullptr;       // left contact sites (device, inside blob)
  int nleft = 0;
  LeadParams lp{};
  std::vector<Step> steps;
  // graph replay of one batch: outputs to staging rows [B][n] (gr, gl) and [B][2][n] (spectral)
  hipGraph_t graph = nullptr;
  hipGraphExec_t gexec = nullptr;
  char* stage = nullptr;
  char* oz = nullptr;            // slice scratch of the products on the integer matrix cores
  size_t oz_bytes = 0;
  const FaceTransJob* face_tj = nullptr;   // [B] transmission over the left face (whole-face contacts)
  double* pot = nullptr;          // [n] on-site potential in cluster order (workspace)
  const int64_t* perm = nullptr;  // [n] site at each cluster-order position (blob)
  bool pot_dirty = true;          // pot may hold non-zero values (or was never written)
  ~Plan() {
    if (oz) (void)hipFree(oz);
    if (gexec) (void)hipGraphExecDestroy(gexec);
    if (graph) (void)hipGraphDestroy(graph);
    if (stage) (void)hipFree(stage);
    if (ws) (void)hipFree(ws);
    if (blob) (void)hipFree(blob);
  }
};

}  // namespace hsc

struct hsc_ctx {
  int device = 0;
  hipStream_t stream = nullptr;
  char* noalloc = nullptr;   // this device's allocation-free product scratch (static device array)
  std::vector<std::unique_ptr<hsc::Plan>> plans;
  // optional per-launch timing: events around every launch, grouped by step kind
  bool profile = false;
  std::vector<std::pair<hipEvent_t, hipEvent_t>> ev_pool;
  struct EvMeta { int kind; double flops; int phase; double bytes; };
  std::vector<EvMeta> ev_meta;                    // per recorded launch
  size_t ev_used = 0;
  double prof[24][3] = {};                        // kind -> launches, ms, flops (24 >= number of kinds)
  double prof_bytes[24] = {};                     // kind -> algorithmic bytes
  hipStream_t cap_stream = nullptr;               // graph capture (a stream of its own, default priority)
  hipStream_t sub[hsc::kMaxStreams] = {};              // streams of concurrent batches (default priority)
  hipEvent_t sub_ev[hsc::kMaxStreams + 1] = {};        // fork (last) and per-stream join events
  std::vector<double> launch_log;                 // (kind, flops, ms, phase) per timed launch since profiling was enabled
  // merged trees of the growth guard: key (tree uid, merged cluster ids), most recent last
  std::vector<std::pair<std::vector<int64_t>, std::shared_ptr<hsc_tree>>> guard_trees;
  // forest of the last multi-device batch and its output staging
  std::vector<uint64_t> forest_key;
  hsc_tree* forest = nullptr;
  char* bstage = nullptr;
  size_t bstage_bytes = 0;
};

namespace hsc {

int ctx_device(const hsc_ctx* ctx) { return ctx->device; }
void* ctx_stream(const hsc_ctx* ctx) { return reinterpret_cast<void*>(ctx->stream); }

namespace {

// ---------------------------------------------------------------------------------------------
// plan construction

struct Builder {
  const hsc_tree* t;
  int B;
  uint32_t want;
  bool gl;        // any lesser output -> full ancestor rows on contact paths
  bool ddf = false;   // double-double fold
  bool ddx = false;   // double-double extraction as well (G, the lesser channels)
  bool oz = false;    // double-double products from 8-bit slices on the integer matrix cores
  int slices = kOzSlices;   // slices per operand of those products
  size_t oz_need = 0; // largest slice scratch of one such product step
  size_t ws = 0;  // workspace bytes
  Blob blob;
  std::vector<Step> steps;
  std::vector<Channel> chans;
  char* wsbase = nullptr;   // device address (known before job pointers are written)
  size_t pot_off = 0;       // workspace offset of the on-site potential, cluster order
  int phase = PH_OTHER;     // stamped onto every step (launch timing)
  void push(Step s) {
    s.phase = phase;
    steps.push_back(s);
  }

  // per-cluster tree constants (blob offsets)
  std::vector<size_t> c_invrel, c_rel, c_gcol, c_trow, c_trowp, c_nfc, c_sites, c_fs;
  // per cluster x slot workspace offsets
  struct CS {
    size_t F, Inv, Psi, GX, GFF, GT, GAF, SD, piv, T, R;
    size_t Fd, Invd, Psid, Td, Rd;   // double-double fold
    size_t NF[kMaxChannels], NFc[kMaxChannels], M[kMaxChannels], PX[kMaxChannels], PFF[kMaxChannels],
        PT[kMaxChannels];
    // 8-bit slices of operands used by several products (precision 3): Psi (rows n, depth f),
    // Psi^T and A_ii^-1 of separators (rows f / n, depth n); 0 = none
    size_t PsiS, PsiTS, InvS;
  };
  std::vector<CS> cs;   // [cluster * B + slot]
  // whole-face contacts: per (contact, slot) the partial mode sums, the dense self-energy block,
  // Gamma (in the extraction's element type) and Gamma times the face's G rows
  struct FS { size_t half, sigma, gamma, gg; };
  std::vector<FS> fsl;  // [contact * B + slot]
  size_t f_tab1[2] = {}, f_tab2[2] = {}, f_jk[2] = {};   // blob: sine tables, face positions
  int face_of(int i) const {
    if (!t->dense) return -1;
    return i == t->face[0].cluster ? 0 : i == t->face[1].cluster ? 1 : -1;
  }

  size_t wsa(size_t bytes) {
    size_t off = (ws + 255) / 256 * 256;
    ws = off + std::max<size_t>(bytes, 16);
    return off;
  }
  double2* W(size_t off) const { return reinterpret_cast<double2*>(wsbase + off); }

  int n_of(int i) const { return t->cl[i].n; }
  int f_of(int i) const { return t->cl[i].f(); }
  int P_of(int i) const { return (int)t->cl[i].n_anc; }
  bool leaf(int i) const { return t->cl[i].children.empty(); }
  bool root(int i) const { return t->cl[i].parent < 0; }
  bool cp(int i) const { return gl && t->cl[i].cpath(); }
  int gcols(int i) const {
    if (root(i)) return n_of(i);
    return n_of(i) + (cp(i) ? P_of(i) : f_of(i));
  }
  bool in_fold(const Channel& ch, int i) const {
    const Cluster& c = t->cl[i];
    return ch.fold == 0 ? c.cpath() : ch.fold == 1 ? c.lpath : c.rpath;
  }
  bool in_extract(const Channel& ch, int i) const { return ch.extract == 0 || t->cl[i].lpath; }
  // own rows of cluster i in channel ch: (row0, r)
  void own_rows(const Channel& ch, int i, int* row0, int* r) const {
    const Cluster& c = t->cl[i];
    if (!leaf(i) || root(i)) { *row0 = 0; *r = c.n; return; }
    if (ch.type == 0) { *row0 = 0; *r = c.n_left + c.n_right; }
    else if (ch.type == 1) { *row0 = 0; *r = c.n_left; }
    else { *row0 = c.n_left; *r = c.n_right; }
  }
  int inv_nb(int maxn) const { return maxn <= 1024 ? 16 : maxn <= 2048 ? 8 : 4; }

  void channels() {
    if (want & HSC_SPECTRAL_LR) {
      chans.push_back({1, 1, 0, O_SPEC_L});
      chans.push_back({2, 2, 0, O_SPEC_R});
      // bond entries of G^< come from the combined channel's blocks
      if (want & HSC_BOND_GL) chans.push_back({0, 0, 0, O_NONE});
    } else {
      if (want & (HSC_DIAG_GL | HSC_BOND_GL)) chans.push_back({0, 0, 0, (want & HSC_DIAG_GL) ? O_GL : O_NONE});
      if (want & HSC_TRANS) chans.push_back({2, 2, 1, O_AR_TMP});
    }
  }

  // Workspace: blocks that live for the whole solve first; then the frontal matrices and Gauss-Jordan
  // work (read only by the fold) and the lesser channels' blocks (written only after the fold) from
  // one base, since every fold step precedes every channel step on the stream.  With per-site leads
  // nothing reads a channel's blocks once the next channel starts (the transmission and the bond
  // entries are taken inside their channel), so the channels share that region too; whole-face
  // leads read the right channel's face block at the end, so there each channel keeps its own.
  void layout() {
    const int nc = (int)t->cl.size();
    cs.assign((size_t)nc * B, CS{});
    const size_t ge = ddx ? 32 : 16;   // bytes per element of G and of the lesser channels
    for (int i = 0; i < nc; ++i) {
      const size_t n = n_of(i), f = f_of(i), P = P_of(i);
      const Cluster& c = t->cl[i];
      for (int e = 0; e < B; ++e) {
        CS& s = cs[(size_t)i * B + e];
        s.Inv = wsa(n * n * 16);
        s.piv = wsa(n * 4);
        if (ddf) {
          s.Invd = wsa(n * n * 32);
          if (!root(i)) s.Psid = wsa(n * f * 32);
          if (oz && !root(i) && (int)f >= kOzMinK) s.PsiS = wsa(oz_bytes((int)n, (int)f));
          if (oz && !root(i) && !leaf(i) && (int)n >= kOzMinK) {
            s.PsiTS = wsa(oz_bytes((int)f, (int)n));
            s.InvS = wsa(oz_bytes((int)n, (int)n));
          }
        }
        if (!root(i)) s.Psi = wsa(n * f * 16);
        if (root(i)) s.GX = ddx ? s.Invd : s.Inv;
        else if (!leaf(i)) s.GX = wsa((n + f) * gcols(i) * ge);
        else {
          s.GFF = wsa(f * f * ge);
          s.GT = wsa(n * f * ge);
          if (cp(i)) {
            s.GAF = wsa(f * P * ge);
            s.SD = wsa((size_t)(c.n_left + c.n_right) * (n + P) * ge);
          }
        }
      }
    }
    const size_t base = ws;
    for (int i = 0; i < nc; ++i) {
      const size_t n = n_of(i), f = f_of(i);
      const int nb = inv_nb((int)n);
      for (int e = 0; e < B; ++e) {
        CS& s = cs[(size_t)i * B + e];
        if (ddf) {
          const size_t nbd = dd_inv_nb((int)n);
          s.Fd = wsa((n + f) * (n + f) * 32);
          s.Td = wsa(n * std::max<size_t>(nbd, kDDSuper) * 32);
          s.Rd = wsa(std::max<size_t>(nbd, kDDSuper) * n * 32);
        } else {
          s.F = wsa((n + f) * (n + f) * 16);
          s.T = wsa(n * 4 * nb * 16);   // panel T (n x nb) and super-panel U (n x 4 nb)
          s.R = wsa(4 * nb * n * 16);   // pivot rows of a panel / super-panel
        }
      }
    }
    const size_t fold_end = ws;
    const bool share = !t->dense;
    size_t chan_end = base;
    ws = base;
    for (size_t k = 0; k < chans.size(); ++k) {
      if (share) ws = base;
      const Channel& ch = chans[k];
      for (int i = 0; i < nc; ++i) {
        const size_t n = n_of(i), f = f_of(i), P = P_of(i);
        for (int e = 0; e < B; ++e) {
          CS& s = cs[(size_t)i * B + e];
          if (in_fold(ch, i)) {
            int row0, r;
            own_rows(ch, i, &row0, &r);
            s.NF[k] = wsa((r + f) * (n + P) * ge);
            if (!root(i)) s.NFc[k] = wsa(r * (n + f) * ge);
            s.M[k] = wsa(n * (n + f) * ge);
          }
          if (in_extract(ch, i)) {
            if (root(i)) s.PX[k] = s.M[k];
            else if (!leaf(i)) s.PX[k] = wsa((n + f) * (n + f) * ge);
            else {
              s.PFF[k] = wsa(f * f * ge);
              s.PT[k] = wsa(n * f * ge);
            }
          }
        }
      }
      chan_end = std::max(chan_end, ws);
    }
    ws = std::max(fold_end, chan_end);
  }

  void layout_faces() {
    if (!t->dense) return;
    fsl.assign((size_t)2 * B, FS{});
    const size_t ge = ddx ? 32 : 16;
    for (int c = 0; c < 2; ++c) {
      const FaceInfo& fi = t->face[c];
      const size_t d1 = fi.dim[0], d2 = fi.dim[1], F = d1 * d2;
      const Cluster& fc = t->cl[fi.cluster];
      for (int e = 0; e < B; ++e) {
        FS& f = fsl[(size_t)c * B + e];
        f.half = wsa(d1 * d2 * d2 * 16);
        f.sigma = wsa(F * F * 16);
        f.gamma = wsa(F * F * ge);
        if (gl) f.gg = wsa(F * (size_t)(fc.n + fc.n_anc) * ge);
      }
    }
  }

  // tree constants
  void constants() {
    const int nc = (int)t->cl.size();
    c_invrel.assign(nc, 0); c_rel.assign(nc, 0); c_gcol.assign(nc, 0); c_trow.assign(nc, 0);
    c_trowp.assign(nc, 0); c_nfc.assign(nc, 0); c_sites.assign(nc, 0); c_fs.assign(nc, 0);
    if (t->dense)
      for (int c = 0; c < 2; ++c) {
        // transverse sine modes of the face (the lead layer's eigenvectors) and each face row's
        // position in the rectangle
        const FaceInfo& fi = t->face[c];
        for (int q = 0; q < 2; ++q) {
          const int d = fi.dim[q];
          std::vector<double> tab((size_t)d * d);
          for (int j = 0; j < d; ++j)
            for (int m = 0; m < d; ++m)
              tab[(size_t)j * d + m] = std::sqrt(2.0 / (d + 1)) * std::sin(M_PI * (double)(m + 1) * (j + 1) / (d + 1));
          (q == 0 ? f_tab1 : f_tab2)[c] = blob.push(tab);
        }
        const Cluster& fc = t->cl[fi.cluster];
        std::vector<int32_t> jk(fc.n);
        for (int a = 0; a < fc.n; ++a) {
          const int64_t site = t->perm[fc.first + a];
          jk[a] = (t->coords[3 * site + fi.ax[0]] - fi.lo[0]) * fi.dim[1] + (t->coords[3 * site + fi.ax[1]] - fi.lo[1]);
        }
        f_jk[c] = blob.push(jk);
      }
    for (int i = 0; i < nc; ++i) {
      const Cluster& c = t->cl[i];
      const int n = c.n, f = c.f();
      std::vector<int64_t> sites(t->perm.begin() + c.first, t->perm.begin() + c.first + n);
      c_sites[i] = blob.push(sites);
      std::vector<int32_t> nfc(n + f);
      for (int a = 0; a < n; ++a) nfc[a] = a;
      for (int k = 0; k < f; ++k) nfc[n + k] = n + c.frontpos[k];
      c_nfc[i] = blob.push(nfc);
      std::vector<int32_t> trow(f), trowp(f);
      for (int k = 0; k < f; ++k) {
        trow[k] = n + (cp(i) ? c.frontpos[k] : k);
        trowp[k] = n + k;
      }
      c_trow[i] = blob.push(trow);
      c_trowp[i] = blob.push(trowp);
      if (c.parent >= 0) {
        const Cluster& p = t->cl[c.parent];
        const int np = p.n, fp = p.f();
        std::vector<int32_t> inv(np + fp, -1);
        for (int k = 0; k < f; ++k) inv[c.rel[k]] = k;
        c_invrel[i] = blob.push(inv);
        c_rel[i] = blob.push(c.rel);
        std::vector<int32_t> gcol(f);
        for (int k = 0; k < f; ++k) {
          const int idx = c.rel[k];
          gcol[k] = idx < np ? idx : (cp(c.parent) ? np + p.frontpos[idx - np] : idx);
        }
        c_gcol[i] = blob.push(gcol);
      }
      // sparse A = -H entries of the frontal matrix: rows (own sites, front sites)
      std::vector<int32_t> fidx(0);
      std::vector<std::vector<std::pair<int32_t, double2>>> rows(n + f);
      // local index of a site within (own, front)
      auto local = [&](int64_t s) -> int {
        if (t->owner[s] == i) return (int)(t->pos[s] - c.first);
        return -1;
      };
      std::vector<int32_t> fpos;   // front site -> index in front (via sorted lookup)
      std::vector<std::pair<int64_t, int32_t>> fl(f);
      for (int k = 0; k < f; ++k) fl[k] = {c.front[k], k};
      std::sort(fl.begin(), fl.end());
      auto findf = [&](int64_t s) -> int {
        auto it = std::lower_bound(fl.begin(), fl.end(), std::make_pair(s, (int32_t)-1));
        return (it != fl.end() && it->first == s) ? it->second : -1;
      };
      for (int a = 0; a < n; ++a) {
        const int64_t r = t->perm[c.first + a];
        for (int64_t q = t->indptr[r]; q < t->indptr[r + 1]; ++q) {
          const int64_t s = t->indices[q];
          const double2 v = make_double2(-t->values[2 * q], -t->values[2 * q + 1]);
          const int b = local(s);
          if (b >= 0) { rows[a].push_back({b, v}); continue; }
          const int k = findf(s);
          if (k < 0) continue;   // (cannot happen: neighbours outside are front sites)
          rows[a].push_back({n + k, v});
          rows[n + k].push_back({a, v});   // A_fi = A_if^T
        }
      }
      std::vector<int32_t> ptr(n + f + 1, 0), col;
      std::vector<double2> val;
      for (int a = 0; a < n + f; ++a) {
        // merge duplicates
        std::sort(rows[a].begin(), rows[a].end(),
                  [](const std::pair<int32_t, double2>& x, const std::pair<int32_t, double2>& y) { return x.first < y.first; });
        for (size_t q = 0; q < rows[a].size(); ++q) {
          if (!col.empty() && (int)col.size() > ptr[a] && col.back() == rows[a][q].first) {
            val.back().x += rows[a][q].second.x;
            val.back().y += rows[a][q].second.y;
          } else {
            col.push_back(rows[a][q].first);
            val.push_back(rows[a][q].second);
          }
        }
        ptr[a + 1] = (int32_t)col.size();
      }
      size_t o_ptr = blob.push(ptr), o_col = blob.push(col), o_val = blob.push(val);
      size_t o_fs = blob.alloc(sizeof(FrontSparse));
      FrontSparse* fs = reinterpret_cast<FrontSparse*>(blob.data.data() + o_fs);
      fs->ptr = reinterpret_cast<const int32_t*>(o_ptr);
      fs->col = reinterpret_cast<const int32_t*>(o_col);
      fs->val = reinterpret_cast<const double2*>(o_val);
      fs->pot = reinterpret_cast<const double*>(wsbase + pot_off) + c.first;
      blob.reloc(o_fs + offsetof(FrontSparse, ptr));
      blob.reloc(o_fs + offsetof(FrontSparse, col));
      blob.reloc(o_fs + offsetof(FrontSparse, val));
      c_fs[i] = o_fs;
    }
  }

  // ---- step helpers ----
  template <class T> struct GPT {
    const T *A, *B, *C; T* D; int M, N, K, lda, ldb, ldc, ldd;
    size_t sa = 0;   // workspace offset of op(A)'s slices when they are kept for other products (0: none)
  };
  using GP = GPT<double2>;
  void gemm(int opA, int opB, const std::vector<GP>& ps, double ar, double ai, int beta) {
    Step s;
    s.kind = S_GEMM;
    for (int kind = 0; kind < kTileDims; ++kind) {
      std::vector<GemmProb> probs;
      std::vector<int32_t> tmap;
      const int tm = kTileDimM[kind], tn = kTileDimN[kind];
      for (const GP& g : ps) {
        if (g.M <= 0 || g.N <= 0) continue;
        GemmProb p{};
        p.A = g.A; p.B = g.B; p.C = g.C; p.D = g.D;
        p.M = g.M; p.N = g.N; p.K = g.K;
        p.lda = g.lda; p.ldb = g.ldb; p.ldc = g.ldc; p.ldd = g.ldd;
        p.tiles_n = (g.N + tn - 1) / tn;
        p.tile_off = (int32_t)tmap.size();
        const int tiles = ((g.M + tm - 1) / tm) * p.tiles_n;
        for (int k = 0; k < tiles; ++k) tmap.push_back((int32_t)probs.size());
        probs.push_back(p);
      }
      if (probs.empty()) return;
      if (kind == 0)
        for (const GemmProb& p : probs) s.flops += 8.0 * p.M * p.N * p.K;
      s.jobs_k[kind] = blob.push(probs);
      s.map_k[kind] = blob.push(tmap);
      s.count_k[kind] = (int)tmap.size();
    }
    s.jobs = s.jobs_k[0];
    s.map = s.map_k[0];
    s.count = s.count_k[0];
    s.i0 = opA; s.i1 = opB;
    s.ar = ar; s.ai = ai; s.beta = beta;
    push(s);
  }
  // RowJob list: child-ref arrays are given as host vectors to be placed in the blob
  struct RJ { RowJob j; std::vector<ChildRef> kids; std::vector<size_t> kid_invrel; bool p1_blob = false; bool p2_raw = false; };
  void rowstep(StepKind kind, std::vector<RJ>& jobs, int i0 = 0, int i1 = 0, int out = 0, int dd = 0) {
    std::vector<int32_t> rmap;
    std::vector<size_t> kid_off(jobs.size(), 0);
    for (size_t q = 0; q < jobs.size(); ++q) {
      if (!jobs[q].kids.empty()) {
        kid_off[q] = blob.alloc(jobs[q].kids.size() * sizeof(ChildRef));
        for (size_t k = 0; k < jobs[q].kids.size(); ++k) {
          size_t fo = kid_off[q] + k * sizeof(ChildRef);
          ChildRef cr = jobs[q].kids[k];
          cr.invrel = reinterpret_cast<const int32_t*>(jobs[q].kid_invrel[k]);
          std::memcpy(blob.data.data() + fo, &cr, sizeof(ChildRef));
          blob.reloc(fo + offsetof(ChildRef, invrel));
        }
      }
    }
    std::vector<RowJob> rj;
    for (size_t q = 0; q < jobs.size(); ++q) {
      RowJob j = jobs[q].j;
      if (j.rows <= 0) continue;
      j.row_off = (int32_t)rmap.size();
      for (int r = 0; r < j.rows; ++r) rmap.push_back((int32_t)rj.size());
      if (!jobs[q].kids.empty()) j.p0 = reinterpret_cast<const void*>(kid_off[q]);
      rj.push_back(j);
      // remember which entries of this job hold blob offsets
      (void)0;
    }
    if (rj.empty()) return;
    Step s;
    s.kind = kind;
    s.jobs = blob.alloc(rj.size() * sizeof(RowJob));
    std::memcpy(blob.data.data() + s.jobs, rj.data(), rj.size() * sizeof(RowJob));
    // relocate blob-resident pointer fields: rmap, cmap, p0 (kids / psi?), p1 (front sparse), p2 (sites)
    size_t qi = 0;
    for (size_t q = 0; q < jobs.size(); ++q) {
      if (jobs[q].j.rows <= 0) continue;
      const size_t base = s.jobs + qi * sizeof(RowJob);
      if (jobs[q].j.rmap) blob.reloc(base + offsetof(RowJob, rmap));
      if (jobs[q].j.cmap) blob.reloc(base + offsetof(RowJob, cmap));
      if (!jobs[q].kids.empty()) blob.reloc(base + offsetof(RowJob, p0));
      if (jobs[q].p1_blob) blob.reloc(base + offsetof(RowJob, p1));
      if (jobs[q].j.p2 && !jobs[q].p2_raw) blob.reloc(base + offsetof(RowJob, p2));
      ++qi;
    }
    s.map = blob.push(rmap);
    s.count = (int)rmap.size();
    s.i0 = i0; s.i1 = i1; s.out = out; s.dd = dd;
    push(s);
  }
  static const int32_t* off32(size_t o) { return reinterpret_cast<const int32_t*>(o); }

  std::vector<std::vector<int>> levels() const {
    std::vector<std::vector<int>> L(t->depth);
    for (int i = 0; i < (int)t->cl.size(); ++i) L[t->cl[i].depth].push_back(i);
    return L;
  }

  // ---- phases ----
  zdd* Z(size_t off) const { return reinterpret_cast<zdd*>(wsbase + off); }
  // the extraction is written once for complex128 (T = double2) and double-double (T = zdd)
  template <class T> static constexpr int kDD = std::is_same<T, zdd>::value ? 1 : 0;
  template <class T> T* X(size_t off) const { return reinterpret_cast<T*>(wsbase + off); }
  template <class T> T* inv_p(const CS& s) const { return X<T>(kDD<T> ? s.Invd : s.Inv); }
  template <class T> T* psi_p(const CS& s) const { return X<T>(kDD<T> ? s.Psid : s.Psi); }
  template <class T> static double2* d2(const T* p) { return reinterpret_cast<double2*>(const_cast<T*>(p)); }
  void gemm_x(int opA, int opB, const std::vector<GP>& ps, int beta) { gemm(opA, opB, ps, 1.0, 0.0, beta); }
  void gemm_x(int opA, int opB, const std::vector<GPT<zdd>>& ps, int beta) {
    std::vector<GPD> q;
    for (const GPT<zdd>& g : ps) q.push_back({g.A, g.B, g.C, g.D, nullptr, g.M, g.N, g.K, g.lda, g.ldb, g.ldc, g.ldd, 0,
                                             g.sa});
    dd_gemm(opA, opB, q, 0, beta);
  }

  struct GPD {
    const zdd *A, *B, *C; zdd* D; double2* D64; int M, N, K, lda, ldb, ldc, ldd, ldd64;
    size_t sa = 0;   // workspace offset of op(A)'s kept slices (0: split into the step's scratch)
  };
  std::vector<size_t> oz_kept;   // kept slice buffers already split by an earlier step
  // Double-double block products: with `oz`, every problem whose depth K lies in
  // [kOzMinK, kOzMaxK] and whose estimated time (splitting + slice product) beats the vector units
  // runs on the integer matrix cores; the others, and every product without `oz`, on the FP64
  // vector units.
  static constexpr int kOzMinK = 32;
  static constexpr size_t kOzStepCap = size_t(4) << 30;   // slice scratch of one product step
  // Measured costs on the target (seconds): splitting one complex double-double element into
  // slices, one padded multiply-add of the slice product, one multiply-add on the vector units.
  static constexpr double kOzSplitCost = 25e-12, kOzMacCost = 0.55e-12, kValuMacCost = 1.5e-12;
  bool oz_pays(const GPD& g) const {
    if (g.K < kOzMinK || g.K > oz_max_depth(slices)) return false;
    const double Mp = oz_round(g.M, 32), Np = oz_round(g.N, 32), Kp = oz_round(g.K, 64);
    const double t_oz = kOzSplitCost * ((g.sa ? 0.0 : Mp) + Np) * Kp + kOzMacCost * Mp * Np * Kp;
    return t_oz < kValuMacCost * (double)g.M * g.N * g.K;
  }
  void dd_gemm(int opA, int opB, const std::vector<GPD>& ps, int negate, int beta) {
    if (!oz) { dd_gemm_valu(opA, opB, ps, negate, beta); return; }
    std::vector<GPD> big, rest;
    for (const GPD& g : ps) (oz_pays(g) ? big : rest).push_back(g);
    if (!big.empty()) oz_gemm(opA, opB, big, negate, beta);
    if (!rest.empty()) dd_gemm_valu(opA, opB, rest, negate, beta);
  }

  static size_t oz_round(size_t v, size_t a) { return (v + a - 1) / a * a; }
  size_t oz_bytes(int R, int K) const {
    return oz_round((size_t)3 * slices * oz_round(R, 32) * oz_round(K, 64) + 4 * oz_round(R, 32), 256);
  }

  // split + product steps, the problem list cut into pieces whose slices fit kOzStepCap; an operand
  // shared by several problems of a piece is split once
  void oz_gemm(int opA, int opB, const std::vector<GPD>& ps, int negate, int beta) {
    size_t i0 = 0;
    while (i0 < ps.size()) {
      std::vector<OzSplitJob> sj;
      std::vector<int32_t> bmap, tmap_s;
      std::vector<GemmProbOZ> gp;
      std::vector<int32_t> tmap;
      std::map<std::tuple<const void*, int64_t, int64_t, int, int>, std::pair<size_t, size_t>> seen;
      size_t cur = 0, i = i0;
      double flops = 0, bytes = 0;
      // slices of one operand: in the step's scratch (offsets rebased later, `kept` false) or in a
      // workspace buffer kept for later products (absolute addresses, split by the first step using it)
      std::vector<char> kept_job;   // per split job: writes a kept buffer
      auto operand = [&](const zdd* X, int64_t ldr, int64_t ldk, int R, int K, size_t keep) {
        const auto key = std::make_tuple((const void*)X, ldr, ldk, R, K);
        auto it = seen.find(key);
        if (it != seen.end()) return it->second;
        const int Rp = (int)oz_round(R, 32), Kp = (int)oz_round(K, 64);
        size_t off;
        if (keep) {
          off = reinterpret_cast<size_t>(wsbase + keep);
          const auto r = std::make_pair(off, off + (size_t)3 * slices * Rp * Kp);
          seen[key] = r;
          if (std::find(oz_kept.begin(), oz_kept.end(), keep) != oz_kept.end()) return r;
          oz_kept.push_back(keep);
        } else {
          off = cur;
          cur += oz_bytes(R, K);
        }
        OzSplitJob j{};
        j.X = X; j.ldr = ldr; j.ldk = ldk; j.R = R; j.K = K; j.Rp = Rp; j.Kp = Kp;
        j.out = reinterpret_cast<int8_t*>(off);
        j.ex = reinterpret_cast<int32_t*>(off + (size_t)3 * slices * Rp * Kp);
        kept_job.push_back(keep ? 1 : 0);
        const int rblocks = (Rp + 63) / 64;
        j.blk_off = (int32_t)bmap.size();
        for (int b = 0; b < rblocks; ++b) bmap.push_back((int32_t)sj.size());
        j.tile_off = (int32_t)tmap_s.size();
        for (int b = 0; b < rblocks * (Kp / 32); ++b) tmap_s.push_back((int32_t)sj.size());
        sj.push_back(j);
        const auto r = std::make_pair(off, off + (size_t)3 * slices * Rp * Kp);
        seen[key] = r;
        return r;
      };
      std::vector<char> kept_a;   // per product: A's slices in a kept buffer
      for (; i < ps.size(); ++i) {
        const GPD& g = ps[i];
        if (g.M <= 0 || g.N <= 0) continue;
        const size_t need = (g.sa ? 0 : oz_bytes(g.M, g.K)) + oz_bytes(g.N, g.K);
        if (i > i0 && cur + need > kOzStepCap) break;
        const auto a = opA == 0 ? operand(g.A, g.lda, 1, g.M, g.K, g.sa) : operand(g.A, 1, g.lda, g.M, g.K, g.sa);
        const auto b = opB == 0 ? operand(g.B, 1, g.ldb, g.N, g.K, 0) : operand(g.B, g.ldb, 1, g.N, g.K, 0);
        kept_a.push_back(g.sa ? 1 : 0);
        GemmProbOZ p{};
        p.A8 = reinterpret_cast<const int8_t*>(a.first);
        p.ea = reinterpret_cast<const int32_t*>(a.second);
        p.B8 = reinterpret_cast<const int8_t*>(b.first);
        p.eb = reinterpret_cast<const int32_t*>(b.second);
        p.C = g.C; p.D = g.D; p.D64 = g.D64;
        p.M = g.M; p.N = g.N;
        p.Mp = (int)oz_round(g.M, 32); p.Np = (int)oz_round(g.N, 32); p.Kp = (int)oz_round(g.K, 64);
        p.ldc = g.ldc; p.ldd = g.ldd; p.ldd64 = g.ldd64;
        p.tiles_n = p.Np / 32;
        p.tile_off = (int32_t)tmap.size();
        const int tiles = (p.Mp / 32) * p.tiles_n;
        for (int k = 0; k < tiles; ++k) tmap.push_back((int32_t)gp.size());
        gp.push_back(p);
        flops += 8.0 * g.M * g.N * g.K;
        // slices of op(A) and op(B) (3 parts x S slices of one byte per complex element), their
        // scales, the double-double result (and its rounded copy), C when accumulating
        bytes += 3.0 * slices * ((double)g.M * g.K + (double)g.K * g.N) + 4.0 * (g.M + g.N) +
                 (double)g.M * g.N * (32.0 + (g.D64 ? 16.0 : 0.0) + (beta ? 32.0 : 0.0));
      }
      oz_need = std::max(oz_need, cur);
      if (!sj.empty()) {
        Step s;
        s.kind = S_OZ_SPLIT;
        s.jobs = blob.push(sj);
        for (size_t q = 0; q < sj.size(); ++q) {
          if (kept_job[q]) continue;
          blob.sc_relocs.push_back(s.jobs + q * sizeof(OzSplitJob) + offsetof(OzSplitJob, out));
          blob.sc_relocs.push_back(s.jobs + q * sizeof(OzSplitJob) + offsetof(OzSplitJob, ex));
        }
        s.map = blob.push(bmap);
        s.count = (int)bmap.size();
        s.map_k[0] = blob.push(tmap_s);
        s.count_k[0] = (int)tmap_s.size();
        push(s);
      }
      if (!gp.empty()) {
        Step s;
        s.kind = S_OZ_GEMM;
        s.jobs = blob.push(gp);
        for (size_t q = 0; q < gp.size(); ++q) {
          const size_t b0 = s.jobs + q * sizeof(GemmProbOZ);
          if (!kept_a[q]) {
            blob.sc_relocs.push_back(b0 + offsetof(GemmProbOZ, A8));
            blob.sc_relocs.push_back(b0 + offsetof(GemmProbOZ, ea));
          }
          blob.sc_relocs.push_back(b0 + offsetof(GemmProbOZ, B8));
          blob.sc_relocs.push_back(b0 + offsetof(GemmProbOZ, eb));
        }
        s.map = blob.push(tmap);
        s.count = (int)tmap.size();
        s.i1 = negate;
        s.beta = beta;
        s.flops = flops;
        s.bytes = bytes;
        push(s);
      }
      i0 = i;
    }
  }

  // one problem list and tile map per tile configuration of the double-double GEMM (the tuner picks
  // one per launch; `tile` is the configuration)
  void dd_gemm_valu(int opA, int opB, const std::vector<GPD>& ps, int negate, int beta) {
    Step s;
    s.kind = S_DD_GEMM;
    for (int cfg = 0; cfg < dd_gemm_configs(); ++cfg) {
      const int tm = dd_gemm_tile_m(cfg), tn = dd_gemm_tile_n(cfg);
      std::vector<GemmProbDD> probs;
      std::vector<int32_t> tmap;
      for (const GPD& g : ps) {
        if (g.M <= 0 || g.N <= 0) continue;
        GemmProbDD p{};
        p.A = g.A; p.B = g.B; p.C = g.C; p.D = g.D; p.D64 = g.D64;
        p.M = g.M; p.N = g.N; p.K = g.K;
        p.lda = g.lda; p.ldb = g.ldb; p.ldc = g.ldc; p.ldd = g.ldd; p.ldd64 = g.ldd64;
        p.tiles_n = (g.N + tn - 1) / tn;
        p.tile_off = (int32_t)tmap.size();
        const int tiles = ((g.M + tm - 1) / tm) * p.tiles_n;
        for (int k = 0; k < tiles; ++k) tmap.push_back((int32_t)probs.size());
        probs.push_back(p);
        if (cfg == 0) s.flops += 8.0 * g.M * g.N * g.K;
      }
      if (probs.empty()) return;
      s.jobs_k[cfg] = blob.push(probs);
      s.map_k[cfg] = blob.push(tmap);
      s.count_k[cfg] = (int)tmap.size();
    }
    s.jobs = s.jobs_k[0];
    s.map = s.map_k[0];
    s.count = s.count_k[0];
    s.i0 = opA;
    s.i1 = negate;
    s.i2 = opB;
    s.beta = beta;
    push(s);
  }

  // Batched Gauss-Jordan inverses in double-double (the pivot blocks A_ii^-1 of Algorithm 1), two
  // levels: panels of nb columns inside super-panels of kDDSuper columns; a panel's rank-nb update
  // touches only its super-panel's columns (vector units), and each super-panel then updates every
  // other column at once with its pivot rows (a rank-kDDSuper product, on the integer matrix cores
  // with `oz`).  Jobs need T (n x kDDSuper) and R (kDDSuper x n) workspaces.
  void dd_inverse(const std::vector<InvJobDD>& ij, int maxn) {
    const int nb = dd_inv_nb(maxn);
    const size_t ijo = blob.push(ij);
    const int SW = kDDSuper;
    for (int s0 = 0; s0 < maxn; s0 += SW) {
      for (int k0 = s0; k0 < std::min(s0 + SW, maxn); k0 += nb) {
        Step p; p.kind = S_DD_INV_PANEL; p.jobs = ijo; p.njobs = (int)ij.size(); p.i0 = k0; p.i1 = nb; p.i2 = maxn;
        push(p);
        Step w = p; w.kind = S_DD_INV_SWAP;
        push(w);
        std::vector<GPD> ps;
        for (const InvJobDD& j : ij) {
          if (k0 >= j.n) continue;
          const int kb = std::min(nb, j.n - k0);
          const int ns = std::min(s0 + SW, j.n) - s0;
          ps.push_back({j.T, j.R + s0, j.X + s0, j.X + s0, nullptr, j.n, ns, kb, kb, j.n, j.ld, j.ld, 0});
        }
        dd_gemm_valu(0, 0, ps, 0, 1);
      }
      Step sp; sp.kind = S_DD_INV_SUPER; sp.jobs = ijo; sp.njobs = (int)ij.size(); sp.i0 = s0; sp.i1 = SW; sp.i2 = maxn;
      push(sp);
      std::vector<GPD> pt;
      for (const InvJobDD& j : ij) {
        if (s0 >= j.n) continue;
        const int ws = std::min(SW, j.n - s0);
        if (s0 > 0) pt.push_back({j.T, j.R, j.X, j.X, nullptr, j.n, s0, ws, SW, j.n, j.ld, j.ld, 0});
        if (s0 + ws < j.n)
          pt.push_back({j.T, j.R + s0 + ws, j.X + s0 + ws, j.X + s0 + ws, nullptr, j.n, j.n - s0 - ws, ws, SW, j.n,
                        j.ld, j.ld, 0});
      }
      dd_gemm(0, 0, pt, 0, 1);
    }
    Step u; u.kind = S_DD_INV_UNSCR; u.jobs = ijo; u.njobs = (int)ij.size(); u.i2 = maxn;
    push(u);
  }

  void fold_dd(const std::vector<std::vector<int>>& L) {
    for (int d = (int)L.size() - 1; d >= 0; --d) {
      phase = PH_FOLD;
      std::vector<RJ> jobs;
      for (int i : L[d])
        for (int e = 0; e < B; ++e) {
          const Cluster& c = t->cl[i];
          const CS& s = cs[(size_t)i * B + e];
          RJ q{};
          q.j.rows = q.j.cols = c.n + c.f();
          q.j.e = e;
          q.j.dst = reinterpret_cast<double2*>(Z(s.Fd));
          q.j.ldd = c.n + c.f();
          for (int k : c.children) {
            const Cluster& kc = t->cl[k];
            const CS& ks = cs[(size_t)k * B + e];
            const int ldk = kc.n + kc.f();
            ChildRef cr{};
            cr.U = reinterpret_cast<const double2*>(Z(ks.Fd) + (size_t)kc.n * ldk + kc.n);
            cr.ldU = ldk;
            q.kids.push_back(cr);
            q.kid_invrel.push_back(c_invrel[k]);
          }
          q.j.aux0 = (int)c.children.size();
          q.j.p1 = reinterpret_cast<const void*>(c_fs[i]);
          q.p1_blob = true;
          q.j.aux1 = c.n; q.j.aux2 = c.n_left; q.j.aux3 = c.n_right;
          face_block(q, i, e);
          jobs.push_back(q);
        }
      rowstep(S_DD_ASSEMBLE, jobs);
      phase = PH_INVERSE;
      int maxn = 0;
      for (int i : L[d]) maxn = std::max(maxn, n_of(i));
      std::vector<InvJobDD> ij;
      for (int i : L[d])
        for (int e = 0; e < B; ++e) {
          const CS& s = cs[(size_t)i * B + e];
          InvJobDD j{};
          j.X = Z(s.Fd); j.ld = n_of(i) + f_of(i);
          j.Y = Z(s.Invd); j.ldy = n_of(i);
          j.Y64 = W(s.Inv); j.ldy64 = n_of(i);
          j.n = n_of(i); j.e = e;
          j.piv = reinterpret_cast<int32_t*>(wsbase + s.piv);
          j.T = Z(s.Td); j.R = Z(s.Rd);
          ij.push_back(j);
        }
      dd_inverse(ij, maxn);
      phase = PH_FOLD;
      std::vector<GPD> pp, pu;
      for (int i : L[d]) {
        if (root(i)) continue;
        const int n = n_of(i), f = f_of(i), ld = n + f;
        for (int e = 0; e < B; ++e) {
          const CS& s = cs[(size_t)i * B + e];
          pp.push_back({Z(s.Invd), Z(s.Fd) + n, nullptr, Z(s.Psid), W(s.Psi), n, f, n, n, ld, 0, f, f, s.InvS});
          pu.push_back({Z(s.Fd) + n, Z(s.Psid), Z(s.Fd) + (size_t)n * ld + n, Z(s.Fd) + (size_t)n * ld + n, nullptr,
                        f, f, n, ld, f, ld, ld, 0});
        }
      }
      dd_gemm(0, 0, pp, 1, 0);
      dd_gemm(1, 0, pu, 0, 1);
    }
    guard_step();
  }

  // the face cluster of a whole-face contact takes its dense self-energy block instead of the
  // per-site scalars
  void face_block(RJ& q, int i, int e) const {
    const int c = face_of(i);
    if (c < 0) return;
    q.j.p2 = W(fsl[(size_t)c * B + e].sigma);
    q.p2_raw = true;
    q.j.aux4 = t->cl[i].n;
    q.j.aux2 = q.j.aux3 = 0;
  }

  // dense self-energy blocks of both faces for every slot (before any assembly)
  void face_steps() {
    if (!t->dense) return;
    phase = PH_OTHER;
    std::vector<FaceJob> fj;
    int md1 = 0, md2 = 0, mf = 0;
    double fl_half = 0, fl_sig = 0;
    for (int c = 0; c < 2; ++c) {
      const FaceInfo& fi = t->face[c];
      for (int e = 0; e < B; ++e) {
        const FS& f = fsl[(size_t)c * B + e];
        FaceJob j{};
        j.e = e;
        j.d1 = fi.dim[0]; j.d2 = fi.dim[1]; j.F = j.d1 * j.d2;
        j.eps = t->contact[c].lead_onsite; j.tl = t->contact[c].lead_hopping; j.tc = t->contact[c].coupling;
        j.tab1 = reinterpret_cast<const double*>(f_tab1[c]);
        j.tab2 = reinterpret_cast<const double*>(f_tab2[c]);
        j.jk = reinterpret_cast<const int32_t*>(f_jk[c]);
        j.half = W(f.half);
        j.sigma = W(f.sigma);
        j.gamma = wsbase + f.gamma;
        j.gamma_dd = ddx ? 1 : 0;
        fj.push_back(j);
        md1 = std::max(md1, j.d1); md2 = std::max(md2, j.d2); mf = std::max(mf, j.F);
        fl_half += 5.0 * j.d1 * (double)j.d2 * j.d2 * j.d2;
        fl_sig += 5.0 * (double)j.F * j.F * j.d1;
      }
    }
    const size_t off = blob.push(fj);
    for (size_t q = 0; q < fj.size(); ++q) {
      const size_t base = off + q * sizeof(FaceJob);
      blob.reloc(base + offsetof(FaceJob, tab1));
      blob.reloc(base + offsetof(FaceJob, tab2));
      blob.reloc(base + offsetof(FaceJob, jk));
    }
    Step h;
    h.kind = S_FACE_HALF; h.jobs = off; h.njobs = (int)fj.size(); h.i0 = md1; h.i1 = md2; h.flops = fl_half;
    push(h);
    Step g;
    g.kind = S_FACE_SIGMA; g.jobs = off; g.njobs = (int)fj.size(); g.i0 = mf; g.flops = fl_sig;
    push(g);
  }

  // Gamma times the face's G rows (own sites and ancestors), the seed of every lesser channel
  template <class T>
  void face_gg() {
    if (!t->dense || !gl) return;
    phase = PH_EXTRACT_G;
    std::vector<GPT<T>> ps;
    for (int c = 0; c < 2; ++c) {
      const int i = t->face[c].cluster;
      const int n = n_of(i), P = P_of(i);
      for (int e = 0; e < B; ++e) {
        const CS& s = cs[(size_t)i * B + e];
        const FS& f = fsl[(size_t)c * B + e];
        const bool lf = leaf(i) && !root(i);
        ps.push_back({X<T>(f.gamma), lf ? X<T>(s.SD) : X<T>(s.GX), nullptr, X<T>(f.gg), n, n + P, n, n,
                      lf ? n + P : gcols(i), 0, n + P});
      }
    }
    gemm_x(OP_N, OP_N, ps, 0);
  }

  // per slot: Gamma_L and the left face's diagonal block of the right channel (A_R there)
  template <class T>
  size_t face_trans_jobs() {
    int k = -1;
    for (size_t q = 0; q < chans.size(); ++q)
      if (chans[q].type == 2) k = (int)q;
    if (!t->dense || k < 0) return 0;
    const int i = t->face[0].cluster;
    std::vector<FaceTransJob> tj;
    for (int e = 0; e < B; ++e) {
      const CS& s = cs[(size_t)i * B + e];
      FaceTransJob j{};
      j.gamma = wsbase + fsl[e].gamma;
      j.P = X<T>(s.PX[k]);
      j.F = n_of(i);
      j.ldp = n_of(i) + f_of(i);
      j.dd = kDD<T>;
      tj.push_back(j);
    }
    return blob.push(tj);
  }

  // bond entries of G^r (lesser = 0, after the extraction of Algorithm 1) or of the combined
  // lesser channel chan (lesser = 1, after its extraction): BondRef per bond, BondSrc per
  // (cluster, slot)
  size_t bond_refs = 0;
  int nbonds = 0;
  void make_bond_refs() {
    const std::vector<int64_t> bl = tree_bonds(t);
    nbonds = (int)(bl.size() / 2);
    std::vector<BondRef> refs(nbonds);
    std::vector<std::vector<std::pair<int64_t, int>>> fidx(t->cl.size());   // sorted (site, front index)
    for (size_t i = 0; i < t->cl.size(); ++i) {
      const Cluster& c = t->cl[i];
      for (int k = 0; k < c.f(); ++k) fidx[i].push_back({c.front[k], k});
      std::sort(fidx[i].begin(), fidx[i].end());
    }
    for (int q = 0; q < nbonds; ++q) {
      const int64_t si = bl[2 * q], sj = bl[2 * q + 1];
      const int ci = t->owner[si], cj = t->owner[sj];
      BondRef r{};
      if (ci == cj) {
        const Cluster& c = t->cl[ci];
        r.c = ci;
        r.a = (int)(t->pos[si] - c.first);
        r.colg = r.colp = (int)(t->pos[sj] - c.first);
        r.mode = (leaf(ci) && !root(ci)) ? 1 : 0;
      } else {
        // the descendant cluster holds the other site in its front (post-order: lower id)
        const int c = std::min(ci, cj);
        const int64_t own = c == ci ? si : sj, other = c == ci ? sj : si;
        const Cluster& cl = t->cl[c];
        auto it = std::lower_bound(fidx[c].begin(), fidx[c].end(), std::make_pair(other, -1));
        const int k = it->second;
        r.c = c;
        r.a = (int)(t->pos[own] - cl.first);
        r.flip = c == ci ? 0 : 1;
        if (leaf(c) && !root(c)) {
          r.mode = 2;
          r.colg = r.colp = k;
        } else {
          r.mode = 0;
          r.colg = cl.n + (cp(c) ? cl.frontpos[k] : k);
          r.colp = cl.n + k;
        }
      }
      refs[q] = r;
    }
    bond_refs = blob.push(refs);
  }
  template <class T>
  void bond_step(int lesser, int chan) {
    if (!(want & (lesser ? HSC_BOND_GL : HSC_BOND_GR))) return;
    if (!bond_refs) make_bond_refs();
    const int nc = (int)t->cl.size();
    std::vector<BondSrc> tab((size_t)nc * B);
    for (int i = 0; i < nc; ++i) {
      const int n = n_of(i), f = f_of(i);
      for (int e = 0; e < B; ++e) {
        const CS& s = cs[(size_t)i * B + e];
        BondSrc b{};
        b.n = n; b.f = f;
        if (leaf(i) && !root(i)) {
          b.psi = psi_p<T>(s);
          if (lesser) {
            b.d = in_fold(chans[chan], i) ? X<T>(s.M[chan]) : nullptr;
            b.ldd = n + f;
            b.xt = X<T>(s.PT[chan]);
          } else {
            b.d = inv_p<T>(s);
            b.ldd = n;
            b.xt = X<T>(s.GT);
          }
        } else if (lesser) {
          b.X = X<T>(s.PX[chan]);
          b.ld = n + f;
        } else {
          b.X = X<T>(s.GX);
          b.ld = gcols(i);
        }
        tab[(size_t)i * B + e] = b;
      }
    }
    Step st;
    st.kind = S_BONDS;
    st.jobs = bond_refs;
    st.map = blob.push(tab);
    st.count = nbonds;
    st.i0 = lesser;
    st.dd = kDD<T>;
    push(st);
  }

  void guard_step() {
    phase = PH_OTHER;
    // conditioning / growth indicators of every pivot block
    std::vector<RowJob> gj;
    for (int i = 0; i < (int)t->cl.size(); ++i)
      for (int e = 0; e < B; ++e) {
        const CS& s = cs[(size_t)i * B + e];
        RowJob j{};
        j.e = e;
        j.src = W(s.Inv); j.lds = n_of(i);
        j.p0 = root(i) ? nullptr : W(s.Psi);
        j.aux0 = n_of(i); j.aux1 = f_of(i); j.aux2 = i;
        gj.push_back(j);
      }
    Step g;
    g.kind = S_GUARD;
    g.jobs = blob.push(gj);
    g.njobs = (int)gj.size();
    push(g);
  }

  void fold(const std::vector<std::vector<int>>& L) {
    if (ddf) { fold_dd(L); return; }
    for (int d = (int)L.size() - 1; d >= 0; --d) {
      phase = PH_FOLD;
      // assemble
      std::vector<RJ> jobs;
      for (int i : L[d])
        for (int e = 0; e < B; ++e) {
          const Cluster& c = t->cl[i];
          const CS& s = cs[(size_t)i * B + e];
          RJ q{};
          q.j.rows = q.j.cols = c.n + c.f();
          q.j.e = e;
          q.j.dst = W(s.F);
          q.j.ldd = c.n + c.f();
          for (int k : c.children) {
            const Cluster& kc = t->cl[k];
            const CS& ks = cs[(size_t)k * B + e];
            const int ldk = kc.n + kc.f();
            ChildRef cr{};
            cr.U = W(ks.F) + (size_t)kc.n * ldk + kc.n;
            cr.ldU = ldk;
            q.kids.push_back(cr);
            q.kid_invrel.push_back(c_invrel[k]);
          }
          q.j.aux0 = (int)c.children.size();
          q.j.p1 = reinterpret_cast<const void*>(c_fs[i]);
          q.p1_blob = true;
          q.j.aux1 = c.n; q.j.aux2 = c.n_left; q.j.aux3 = c.n_right;
          face_block(q, i, e);
          jobs.push_back(q);
        }
      rowstep(S_ASSEMBLE, jobs);
      phase = PH_INVERSE;
      // inverse of the pivot blocks
      int maxn = 0;
      for (int i : L[d]) maxn = std::max(maxn, n_of(i));
      const int nb = inv_nb(maxn);
      std::vector<InvJob> ij;
      for (int i : L[d])
        for (int e = 0; e < B; ++e) {
          const CS& s = cs[(size_t)i * B + e];
          InvJob j{};
          j.X = W(s.F); j.ld = n_of(i) + f_of(i);
          j.Y = W(s.Inv); j.ldy = n_of(i);
          j.n = n_of(i); j.e = e;
          j.piv = reinterpret_cast<int32_t*>(wsbase + s.piv);
          j.T = W(s.T); j.R = W(s.R);
          ij.push_back(j);
        }
      const size_t ijo = blob.push(ij);
      // two-level blocked Gauss-Jordan: super-panels of 4 nb columns; inside one, the rank-nb
      // updates are confined to its columns; then one rank-4nb update of all other columns
      const int SW = 4 * nb;
      for (int s0 = 0; s0 < maxn; s0 += SW) {
        for (int k0 = s0; k0 < std::min(s0 + SW, maxn); k0 += nb) {
          Step p; p.kind = S_INV_PANEL; p.jobs = ijo; p.njobs = (int)ij.size(); p.i0 = k0; p.i1 = nb; p.i2 = maxn;
          push(p);
          Step w = p; w.kind = S_INV_SWAP;
          push(w);
          std::vector<GP> ps;
          for (const InvJob& j : ij) {
            if (k0 >= j.n) continue;
            const int kb = std::min(nb, j.n - k0);
            const int ns = std::min(s0 + SW, j.n) - s0;
            ps.push_back({j.T, j.R + s0, j.X + s0, j.X + s0, j.n, ns, kb, kb, j.n, j.ld, j.ld});
          }
          gemm(OP_N, OP_N, ps, 1.0, 0.0, 1);
        }
        Step sp; sp.kind = S_INV_SUPER; sp.jobs = ijo; sp.njobs = (int)ij.size(); sp.i0 = s0; sp.i1 = SW; sp.i2 = maxn;
        push(sp);
        std::vector<GP> pt;
        for (const InvJob& j : ij) {
          if (s0 >= j.n) continue;
          const int ws = std::min(SW, j.n - s0);
          if (s0 > 0) pt.push_back({j.T, j.R, j.X, j.X, j.n, s0, ws, SW, j.n, j.ld, j.ld});
          if (s0 + ws < j.n)
            pt.push_back({j.T, j.R + s0 + ws, j.X + s0 + ws, j.X + s0 + ws, j.n, j.n - s0 - ws, ws, SW, j.n, j.ld, j.ld});
        }
        gemm(OP_N, OP_N, pt, 1.0, 0.0, 1);
      }
      Step u; u.kind = S_INV_UNSCR; u.jobs = ijo; u.njobs = (int)ij.size(); u.i2 = maxn;
      push(u);
      phase = PH_FOLD;
      // Psi = -Inv * A_if ;  U = A_ff + A_if^T Psi
      std::vector<GP> pp, pu;
      for (int i : L[d]) {
        if (root(i)) continue;
        const int n = n_of(i), f = f_of(i), ld = n + f;
        for (int e = 0; e < B; ++e) {
          const CS& s = cs[(size_t)i * B + e];
          pp.push_back({W(s.Inv), W(s.F) + n, nullptr, W(s.Psi), n, f, n, n, ld, 0, f});
          pu.push_back({W(s.F) + n, W(s.Psi), W(s.F) + (size_t)n * ld + n, W(s.F) + (size_t)n * ld + n, f, f, n,
                        ld, f, ld, ld});
        }
      }
      gemm(OP_N, OP_N, pp, -1.0, 0.0, 0);
      gemm(OP_T, OP_N, pu, 1.0, 0.0, 1);
    }
    guard_step();
  }

  template <class T>
  void diag_step(const std::vector<int>& ids, int mode, int out, int chan, bool g_phase) {
    if (out == O_NONE || (g_phase && out == O_GR && !(want & HSC_DIAG_GR))) return;
    std::vector<RJ> jobs;
    for (int i : ids)
      for (int e = 0; e < B; ++e) {
        const CS& s = cs[(size_t)i * B + e];
        const int n = n_of(i), f = f_of(i);
        RJ q{};
        q.j.rows = n;
        q.j.cols = 1;
        q.j.e = e;
        q.j.p2 = reinterpret_cast<const void*>(c_sites[i]);
        if (mode == DIAG_SEP) {
          if (g_phase) { q.j.src = d2(X<T>(s.GX)); q.j.lds = gcols(i); }
          else { q.j.src = d2(X<T>(s.PX[chan])); q.j.lds = n + f; }
        } else if (mode == DIAG_LEAF_G) {
          q.j.src = d2(X<T>(s.GT)); q.j.lds = f;
          q.j.p0 = psi_p<T>(s); q.j.aux0 = f;
          q.j.p1 = inv_p<T>(s); q.j.aux1 = n;
        } else {
          q.j.src = d2(X<T>(s.PT[chan])); q.j.lds = f;
          q.j.p0 = psi_p<T>(s); q.j.aux0 = f;
          q.j.p1 = in_fold(chans[chan], i) ? X<T>(s.M[chan]) : nullptr;
          q.j.aux1 = n + f;
        }
        jobs.push_back(q);
      }
    rowstep(S_DIAG, jobs, mode, 0, out, kDD<T>);
  }

  template <class T>
  void extract_g(const std::vector<std::vector<int>>& L) {
    phase = PH_EXTRACT_G;
    diag_step<T>(L[0], DIAG_SEP, O_GR, 0, true);
    for (size_t d = 1; d < L.size(); ++d) {
      std::vector<int> seps, leaves;
      for (int i : L[d]) (leaf(i) ? leaves : seps).push_back(i);
      // separators
      {
        std::vector<RJ> g1, g2;
        std::vector<GPT<T>> m1, m2;
        for (int i : seps) {
          const Cluster& c = t->cl[i];
          const int n = c.n, f = c.f(), gc = gcols(i), p = c.parent;
          for (int e = 0; e < B; ++e) {
            const CS& s = cs[(size_t)i * B + e];
            const CS& ps = cs[(size_t)p * B + e];
            RJ q{};
            q.j.rows = f; q.j.cols = gc - n; q.j.e = e;
            q.j.src = d2(X<T>(ps.GX)); q.j.lds = gcols(p);
            q.j.dst = d2(X<T>(s.GX) + (size_t)n * gc + n); q.j.ldd = gc;
            q.j.rmap = off32(c_rel[i]);
            q.j.cmap = cp(i) ? nullptr : off32(c_gcol[i]);
            g1.push_back(q);
            m1.push_back({psi_p<T>(s), X<T>(s.GX) + (size_t)n * gc + n, nullptr, X<T>(s.GX) + n, n, gc - n, f, f, gc, 0, gc,
                          s.PsiS});
            RJ tq{};
            tq.j.rows = f; tq.j.cols = n; tq.j.e = e;
            tq.j.src = d2(X<T>(s.GX)); tq.j.lds = gc;
            tq.j.dst = d2(X<T>(s.GX) + (size_t)n * gc); tq.j.ldd = gc;
            tq.j.rmap = off32(c_trow[i]);
            g2.push_back(tq);
            m2.push_back({psi_p<T>(s), X<T>(s.GX) + (size_t)n * gc, inv_p<T>(s), X<T>(s.GX), n, n, f, f, gc, n, gc, s.PsiS});
          }
        }
        rowstep(S_GATHER, g1, 0, 0, 0, kDD<T>);
        gemm_x(OP_N, OP_N, m1, 0);
        rowstep(S_GATHER, g2, 1, 0, 0, kDD<T>);
        gemm_x(OP_N, OP_N, m2, 1);
        diag_step<T>(seps, DIAG_SEP, O_GR, 0, true);
      }
      // leaves
      {
        std::vector<RJ> g1, g3;
        std::vector<GPT<T>> m1, m3, m4;
        std::vector<int> cpl;
        for (int i : leaves) {
          const Cluster& c = t->cl[i];
          const int n = c.n, f = c.f(), p = c.parent, P = P_of(i), nc = c.n_left + c.n_right;
          if (cp(i)) cpl.push_back(i);
          for (int e = 0; e < B; ++e) {
            const CS& s = cs[(size_t)i * B + e];
            const CS& ps = cs[(size_t)p * B + e];
            RJ q{};
            q.j.rows = f; q.j.cols = f; q.j.e = e;
            q.j.src = d2(X<T>(ps.GX)); q.j.lds = gcols(p);
            q.j.dst = d2(X<T>(s.GFF)); q.j.ldd = f;
            q.j.rmap = off32(c_rel[i]);
            q.j.cmap = off32(c_gcol[i]);
            g1.push_back(q);
            m1.push_back({psi_p<T>(s), X<T>(s.GFF), nullptr, X<T>(s.GT), n, f, f, f, f, 0, f, s.PsiS});
            if (cp(i)) {
              RJ a{};
              a.j.rows = f; a.j.cols = P; a.j.e = e;
              a.j.src = d2(X<T>(ps.GX)); a.j.lds = gcols(p);
              a.j.dst = d2(X<T>(s.GAF)); a.j.ldd = P;
              a.j.rmap = off32(c_rel[i]);
              g3.push_back(a);
              m3.push_back({psi_p<T>(s), X<T>(s.GAF), nullptr, X<T>(s.SD) + n, nc, P, f, f, P, 0, n + P});
              m4.push_back({psi_p<T>(s), X<T>(s.GT), inv_p<T>(s), X<T>(s.SD), nc, n, f, f, f, n, n + P});
            }
          }
        }
        rowstep(S_GATHER, g1, 0, 0, 0, kDD<T>);
        gemm_x(OP_N, OP_N, m1, 0);
        diag_step<T>(leaves, DIAG_LEAF_G, O_GR, 0, true);
        rowstep(S_GATHER, g3, 0, 0, 0, kDD<T>);
        gemm_x(OP_N, OP_N, m3, 0);
        gemm_x(OP_N, OP_T, m4, 1);
      }
    }
    bond_step<T>(0, 0);
  }

  template <class T>
  void channel_steps(const std::vector<std::vector<int>>& L, int k) {
    const Channel& ch = chans[k];
    // N fold, bottom-up
    phase = PH_FOLD_N;
    for (int d = (int)L.size() - 1; d >= 0; --d) {
      std::vector<RJ> asm_jobs, nfc_jobs;
      std::vector<GPT<T>> nu, mm;
      for (int i : L[d]) {
        if (!in_fold(ch, i)) continue;
        const Cluster& c = t->cl[i];
        const int n = c.n, f = c.f(), P = P_of(i);
        int row0, r;
        own_rows(ch, i, &row0, &r);
        for (int e = 0; e < B; ++e) {
          const CS& s = cs[(size_t)i * B + e];
          RJ q{};
          q.j.rows = r + f; q.j.cols = n + P; q.j.e = e;
          q.j.dst = d2(X<T>(s.NF[k])); q.j.ldd = n + P;
          for (int kk : c.children) {
            if (!in_fold(ch, kk)) continue;
            const Cluster& kc = t->cl[kk];
            const CS& ks = cs[(size_t)kk * B + e];
            int kr0, kr;
            own_rows(ch, kk, &kr0, &kr);
            const int ldk = kc.n + P_of(kk);
            ChildRef cr{};
            cr.U = d2(X<T>(ks.NF[k]) + (size_t)kr * ldk + kc.n);
            cr.ldU = ldk;
            q.kids.push_back(cr);
            q.kid_invrel.push_back(c_invrel[kk]);
          }
          q.j.aux0 = (int)q.kids.size();
          q.j.aux1 = r; q.j.aux2 = row0; q.j.aux3 = n; q.j.aux4 = c.n_left; q.j.aux5 = c.n_right;
          if (leaf(i) && !root(i)) { q.j.src = d2(X<T>(s.SD)); q.j.lds = n + P; }
          else { q.j.src = d2(X<T>(s.GX)); q.j.lds = gcols(i); }
          if (face_of(i) >= 0) q.j.p1 = d2(X<T>(fsl[(size_t)face_of(i) * B + e].gg));
          asm_jobs.push_back(q);
          if (!root(i)) {
            nu.push_back({psi_p<T>(s) + (size_t)row0 * f, X<T>(s.NF[k]) + n, X<T>(s.NF[k]) + (size_t)r * (n + P) + n,
                          X<T>(s.NF[k]) + (size_t)r * (n + P) + n, f, P, r, f, n + P, n + P, n + P,
                          (row0 == 0 && r == n) ? s.PsiTS : 0});
            RJ g{};
            g.j.rows = r; g.j.cols = n + f; g.j.e = e;
            g.j.src = d2(X<T>(s.NF[k])); g.j.lds = n + P;
            g.j.dst = d2(X<T>(s.NFc[k])); g.j.ldd = n + f;
            g.j.cmap = off32(c_nfc[i]);
            nfc_jobs.push_back(g);
            mm.push_back({inv_p<T>(s) + row0, X<T>(s.NFc[k]), nullptr, X<T>(s.M[k]), n, n + f, r, n, n + f, 0, n + f,
                          (row0 == 0 && r == n) ? s.InvS : 0});
          } else {
            mm.push_back({inv_p<T>(s) + row0, X<T>(s.NF[k]), nullptr, X<T>(s.M[k]), n, n, r, n, n, 0, n});
          }
        }
      }
      rowstep(S_ASSEMBLE_N, asm_jobs, ch.type, 0, 0, kDD<T>);
      gemm_x(OP_T, OP_N, nu, 1);
      rowstep(S_GATHER, nfc_jobs, 0, 0, 0, kDD<T>);
      gemm_x(OP_N, OP_N, mm, 0);
    }
    // P extract, top-down
    phase = PH_EXTRACT_P;
    diag_step<T>(L[0], DIAG_SEP, ch.out, k, false);
    for (size_t d = 1; d < L.size(); ++d) {
      std::vector<int> seps, leaves;
      for (int i : L[d]) {
        if (!in_extract(ch, i)) continue;
        (leaf(i) ? leaves : seps).push_back(i);
      }
      std::vector<RJ> g1, g2, g3;
      std::vector<GPT<T>> m1a, m1b, m2a, m2b, m3a, m3b;
      for (int i : seps) {
        const Cluster& c = t->cl[i];
        const int n = c.n, f = c.f(), ld = n + f, p = c.parent;
        const bool fm = in_fold(ch, i);
        for (int e = 0; e < B; ++e) {
          const CS& s = cs[(size_t)i * B + e];
          const CS& ps = cs[(size_t)p * B + e];
          RJ q{};
          q.j.rows = f; q.j.cols = f; q.j.e = e;
          q.j.src = d2(X<T>(ps.PX[k])); q.j.lds = n_of(p) + f_of(p);
          q.j.dst = d2(X<T>(s.PX[k]) + (size_t)n * ld + n); q.j.ldd = ld;
          q.j.rmap = off32(c_rel[i]); q.j.cmap = off32(c_rel[i]);
          g1.push_back(q);
          GPT<T> a{psi_p<T>(s), X<T>(s.PX[k]) + (size_t)n * ld + n, fm ? X<T>(s.M[k]) + n : nullptr, X<T>(s.PX[k]) + n, n, f, f, f,
               ld, ld, ld, s.PsiS};
          (fm ? m1b : m1a).push_back(a);
          RJ tq{};
          tq.j.rows = f; tq.j.cols = n; tq.j.e = e;
          tq.j.src = d2(X<T>(s.PX[k])); tq.j.lds = ld;
          tq.j.dst = d2(X<T>(s.PX[k]) + (size_t)n * ld); tq.j.ldd = ld;
          tq.j.rmap = off32(c_trowp[i]);
          g2.push_back(tq);
          GPT<T> b{psi_p<T>(s), X<T>(s.PX[k]) + (size_t)n * ld, fm ? X<T>(s.M[k]) : nullptr, X<T>(s.PX[k]), n, n, f, f, ld, ld, ld,
                   s.PsiS};
          (fm ? m2b : m2a).push_back(b);
        }
      }
      for (int i : leaves) {
        const Cluster& c = t->cl[i];
        const int n = c.n, f = c.f(), p = c.parent;
        const bool fm = in_fold(ch, i);
        for (int e = 0; e < B; ++e) {
          const CS& s = cs[(size_t)i * B + e];
          const CS& ps = cs[(size_t)p * B + e];
          RJ q{};
          q.j.rows = f; q.j.cols = f; q.j.e = e;
          q.j.src = d2(X<T>(ps.PX[k])); q.j.lds = n_of(p) + f_of(p);
          q.j.dst = d2(X<T>(s.PFF[k])); q.j.ldd = f;
          q.j.rmap = off32(c_rel[i]); q.j.cmap = off32(c_rel[i]);
          g3.push_back(q);
          GPT<T> a{psi_p<T>(s), X<T>(s.PFF[k]), fm ? X<T>(s.M[k]) + n : nullptr, X<T>(s.PT[k]), n, f, f, f, f, n + f, f,
                   s.PsiS};
          (fm ? m3b : m3a).push_back(a);
        }
      }
      rowstep(S_GATHER, g1, 0, 0, 0, kDD<T>);
      rowstep(S_GATHER, g3, 0, 0, 0, kDD<T>);
      gemm_x(OP_N, OP_N, m1a, 0);
      gemm_x(OP_N, OP_N, m1b, 1);
      gemm_x(OP_N, OP_N, m3a, 0);
      gemm_x(OP_N, OP_N, m3b, 1);
      rowstep(S_GATHER, g2, 1, 1, 0, kDD<T>);
      gemm_x(OP_N, OP_N, m2a, 0);
      gemm_x(OP_N, OP_N, m2b, 1);
      diag_step<T>(seps, DIAG_SEP, ch.out, k, false);
      diag_step<T>(leaves, DIAG_LEAF_P, ch.out, k, false);
    }
    if (ch.type == 0) bond_step<T>(1, k);
  }
};

// Launch timing keeps at most kEventPairs event pairs alive: a full pool is drained (wait for
// the last recorded launch, add the durations to the per-kind totals) and reused.
constexpr size_t kEventPairs = 512;

hsc_status fold_events(hsc_ctx* ctx) {
  if (ctx->ev_used == 0) return HSC_OK;
  HIPCHK(hipEventSynchronize(ctx->ev_pool[ctx->ev_used - 1].second));
  for (size_t k = 0; k < ctx->ev_used; ++k) {
    float ms = 0.f;
    HIPCHK(hipEventElapsedTime(&ms, ctx->ev_pool[k].first, ctx->ev_pool[k].second));
    const int kind = ctx->ev_meta[k].kind;
    ctx->prof[kind][0] += 1;
    ctx->prof[kind][1] += ms;
    ctx->prof[kind][2] += ctx->ev_meta[k].flops;
    ctx->prof_bytes[kind] += ctx->ev_meta[k].bytes;
    if (ctx->launch_log.size() < 4 * (size_t)4000000) {
      ctx->launch_log.push_back(kind);
      ctx->launch_log.push_back(ctx->ev_meta[k].flops);
      ctx->launch_log.push_back(ms);
      ctx->launch_log.push_back(ctx->ev_meta[k].phase);
    }
  }
  ctx->ev_used = 0;
  return HSC_OK;
}

// double-double GEMM tile configuration of an untuned plan (64x32)
constexpr int kDefaultDDConfig = 1;

// tile size used by a launch kind of launch_gemm
int tile_dims_of(int kind) {
  switch (kind) {
    case 1: return 1;
    case 2: return 2;
    case 3: case 5: return 3;
    case 8: return 4;
    default: return 0;   // 0, 4, 6, 7: 64x64
  }
}

// launch kinds a plan may use: the four-product kernels, or with the three-product form its
// kernels plus the 128x128 four-product kernel (which has no three-product variant)
const int kKinds4[] = {0, 1, 2, 3, 6, 8};
const int kKinds3[] = {4, 5, 7, 8};

bool step_empty(const Step& s) {
  switch (s.kind) {
    case S_INV_PANEL: case S_INV_SWAP: case S_INV_UNSCR: case S_INV_SUPER: case S_GUARD:
    case S_DD_INV_PANEL: case S_DD_INV_SWAP: case S_DD_INV_UNSCR: case S_DD_INV_SUPER:
    case S_FACE_HALF: case S_FACE_SIGMA:
      return s.njobs <= 0;
    case S_BONDS:
      return s.count <= 0;
    default:
      return s.count <= 0;
  }
}

int run_steps(hsc_ctx* ctx, hipStream_t st, Plan* pl, int e_base, int nvalid, void* gr, void* glo,
              double* spectral, double* guard, int nclusters, void* bond_gr = nullptr, void* bond_gl = nullptr) {
  const int64_t n = pl->n;
  for (const Step& s : pl->steps) {
    if (step_empty(s)) continue;
    hipEvent_t ev1 = nullptr;
    if (ctx->profile) {
      if (ctx->ev_used == kEventPairs) {
        const hsc_status r = fold_events(ctx);
        if (r != HSC_OK) return r;
      }
      if (ctx->ev_used == ctx->ev_pool.size()) {
        hipEvent_t a, b;
        HIPCHK(hipEventCreate(&a));
        HIPCHK(hipEventCreate(&b));
        ctx->ev_pool.push_back({a, b});
        ctx->ev_meta.push_back({0, 0.0, 0, 0.0});
      }
      HIPCHK(hipEventRecord(ctx->ev_pool[ctx->ev_used].first, st));
      ev1 = ctx->ev_pool[ctx->ev_used].second;
      ctx->ev_meta[ctx->ev_used] = {(int)s.kind, s.flops, s.phase, s.bytes};
      ctx->ev_used++;
    }
    const void* jobs = pl->blob + s.jobs;
    const int32_t* map = reinterpret_cast<const int32_t*>(pl->blob + s.map);
    switch (s.kind) {
      case S_ASSEMBLE:
        launch_assemble(st, (const RowJob*)jobs, map, s.count, pl->es);
        break;
      case S_ASSEMBLE_N:
        if (s.dd) launch_dd_assemble_n(st, (const RowJob*)jobs, map, s.count, pl->es, s.i0);
        else launch_assemble_n(st, (const RowJob*)jobs, map, s.count, pl->es, s.i0);
        break;
      case S_GATHER:
        if (s.dd) launch_dd_gather(st, (const RowJob*)jobs, map, s.count, s.i0, s.i1);
        else launch_gather(st, (const RowJob*)jobs, map, s.count, s.i0, s.i1);
        break;
      case S_GEMM:
      {
        const int d = tile_dims_of(s.tile);
        launch_gemm(st, s.i0, s.i1, (const GemmProb*)(pl->blob + s.jobs_k[d]),
                    reinterpret_cast<const int32_t*>(pl->blob + s.map_k[d]), s.count_k[d], s.ar, s.ai, s.beta, s.tile);
      }
        break;
      case S_INV_PANEL:
        launch_inv_panel(st, (const InvJob*)jobs, s.njobs, s.i0, s.i1, s.i2, pl->status);
        break;
      case S_INV_SWAP:
        launch_inv_swap(st, (const InvJob*)jobs, s.njobs, s.i0, s.i1, s.i2);
        break;
      case S_INV_UNSCR:
        launch_inv_unscramble(st, (const InvJob*)jobs, s.njobs, s.i2);
        break;
      case S_INV_SUPER:
        launch_inv_super(st, (const InvJob*)jobs, s.njobs, s.i0, s.i1, s.i2);
        break;
      case S_GUARD:
        launch_guard(st, (const RowJob*)jobs, s.njobs, nclusters, e_base, nvalid, guard);
        break;
      case S_DD_ASSEMBLE:
        launch_dd_assemble(st, (const RowJob*)jobs, map, s.count, pl->es);
        break;
      case S_DD_INV_PANEL:
        launch_dd_inv_panel(st, (const InvJobDD*)jobs, s.njobs, s.i0, s.i1, s.i2, pl->status);
        break;
      case S_DD_INV_SWAP:
        launch_dd_inv_swap(st, (const InvJobDD*)jobs, s.njobs, s.i0, s.i1, s.i2);
        break;
      case S_DD_INV_UNSCR:
        launch_dd_inv_unscramble(st, (const InvJobDD*)jobs, s.njobs, s.i2);
        break;
      case S_DD_INV_SUPER:
        launch_dd_inv_super(st, (const InvJobDD*)jobs, s.njobs, s.i0, s.i1, s.i2);
        break;
      case S_DD_GEMM:
        launch_dd_gemm(st, s.i0, s.i2, s.tile, (const GemmProbDD*)(pl->blob + s.jobs_k[s.tile]),
                       reinterpret_cast<const int32_t*>(pl->blob + s.map_k[s.tile]), s.count_k[s.tile], s.i1, s.beta);
        break;
      case S_OZ_SPLIT:
        launch_oz_split(st, pl->slices, (const OzSplitJob*)jobs, map, s.count,
                        reinterpret_cast<const int32_t*>(pl->blob + s.map_k[0]), s.count_k[0]);
        break;
      case S_OZ_GEMM:
        launch_oz_gemm(st, pl->slices, (const GemmProbOZ*)jobs, map, s.count, s.i1, s.beta);
        break;
      case S_FACE_HALF:
        launch_face_half(st, (const FaceJob*)jobs, s.njobs, s.i0, s.i1, pl->es);
        break;
      case S_FACE_SIGMA:
        launch_face_sigma(st, (const FaceJob*)jobs, s.njobs, s.i0);
        break;
      case S_BONDS:
        launch_bonds(st, (const BondRef*)jobs, s.count, reinterpret_cast<const BondSrc*>(map), pl->B, nvalid, e_base,
                     s.i0, s.dd, static_cast<double2*>(s.i0 ? bond_gl : bond_gr));
        break;
      case S_DIAG: {
        void* out = nullptr;
        int kind = OUT_COMPLEX, eb = e_base;
        int64_t stride = n;
        switch (s.out) {
          case O_GR: out = gr; break;
          case O_GL: out = glo; break;
          case O_SPEC_L: out = spectral; kind = OUT_IMAG; stride = 2 * n; break;
          case O_SPEC_R: out = spectral ? spectral + n : nullptr; kind = OUT_IMAG; stride = 2 * n; break;
          case O_AR_TMP: out = pl->a_r; kind = OUT_IMAG; eb = 0; break;
        }
        if (out && s.dd) launch_dd_diag(st, (const RowJob*)jobs, map, s.count, s.i0, kind, out, stride, eb, nvalid);
        else if (out) launch_diag(st, (const RowJob*)jobs, map, s.count, s.i0, kind, out, stride, eb, nvalid);
        break;
      }
    }
    if (ev1) HIPCHK(hipEventRecord(ev1, st));
  }
  HIPCHK(hipGetLastError());
  return HSC_OK;
}

// Tile autotuner: every GEMM step of the plan is timed once with each tile shape on the
// plan's own problem list and keeps the fastest.  The workspace holds no results yet; the
// solve rewrites every buffer of a batch before reading it.
hsc_status tune_plan(hsc_ctx* ctx, Plan* pl) {
  hipEvent_t a, b;
  HIPCHK(hipEventCreate(&a));
  HIPCHK(hipEventCreate(&b));
  hipStream_t st = ctx->stream;
  hsc_status rc = HSC_OK;
  for (Step& s : pl->steps) {
    if (s.kind == S_DD_GEMM) {
      float best = 0.f;
      int best_c = s.tile;
      for (int c = 0; c < dd_gemm_configs() && rc == HSC_OK; ++c) {
        float ms = 0.f;
        for (int rep = 0; rep < 2; ++rep) {
          if (hipEventRecord(a, st) != hipSuccess) { rc = HSC_E_HIP; break; }
          launch_dd_gemm(st, s.i0, s.i2, c, (const GemmProbDD*)(pl->blob + s.jobs_k[c]),
                         reinterpret_cast<const int32_t*>(pl->blob + s.map_k[c]), s.count_k[c], s.i1, s.beta);
          if (hipEventRecord(b, st) != hipSuccess || hipEventSynchronize(b) != hipSuccess ||
              hipEventElapsedTime(&ms, a, b) != hipSuccess) {
            rc = HSC_E_HIP;
            break;
          }
        }
        if (rc == HSC_OK && (c == 0 || ms < best)) { best = ms; best_c = c; }
      }
      if (rc != HSC_OK) break;
      s.tile = best_c;
      continue;
    }
    if (s.kind != S_GEMM) continue;
    float best = 0.f;
    int best_k = s.tile;
    const int* kinds = pl->m3 ? kKinds3 : kKinds4;
    const int nkinds = pl->m3 ? (int)(sizeof(kKinds3) / sizeof(int)) : (int)(sizeof(kKinds4) / sizeof(int));
    for (int q = 0; q < nkinds && rc == HSC_OK; ++q) {
      const int k = kinds[q], d = tile_dims_of(k);
      float ms = 0.f;
      for (int rep = 0; rep < 2; ++rep) {
        if (hipEventRecord(a, st) != hipSuccess) { rc = HSC_E_HIP; break; }
        launch_gemm(st, s.i0, s.i1, (const GemmProb*)(pl->blob + s.jobs_k[d]),
                    reinterpret_cast<const int32_t*>(pl->blob + s.map_k[d]), s.count_k[d], s.ar, s.ai, s.beta, k);
        if (hipEventRecord(b, st) != hipSuccess || hipEventSynchronize(b) != hipSuccess ||
            hipEventElapsedTime(&ms, a, b) != hipSuccess) {
          rc = HSC_E_HIP;
          break;
        }
      }
      if (rc == HSC_OK && (q == 0 || ms < best)) { best = ms; best_k = k; }
    }
    if (rc != HSC_OK) break;
    s.tile = best_k;
  }
  (void)hipEventDestroy(a);
  (void)hipEventDestroy(b);
  if (rc != HSC_OK) {
    (void)hipGetLastError();
    set_error("GEMM tile tuning failed");
  }
  return rc;
}

// Allocate the slice scratch, rebase the blob's pointer fields, upload it and take the steps.
hsc_status upload_plan(Builder& b, Plan* pl) {
  if (b.oz_need > 0) {
    pl->oz_bytes = b.oz_need;
    if (hipMalloc(&pl->oz, pl->oz_bytes) != hipSuccess) {
      (void)hipGetLastError();
      pl->oz = nullptr;
      set_error("slice scratch allocation failed (" + std::to_string(pl->oz_bytes) + " bytes)");
      return HSC_E_OOM;
    }
    for (size_t f : b.blob.sc_relocs) {
      uint64_t v;
      std::memcpy(&v, b.blob.data.data() + f, 8);
      v += reinterpret_cast<uint64_t>(pl->oz);
      std::memcpy(b.blob.data.data() + f, &v, 8);
    }
  }
  pl->blob_bytes = b.blob.data.size();
  if (hipMalloc(&pl->blob, pl->blob_bytes) != hipSuccess) {
    (void)hipGetLastError();
    pl->blob = nullptr;
    set_error("device plan allocation failed");
    return HSC_E_OOM;
  }
  for (size_t f : b.blob.relocs) {
    uint64_t v;
    std::memcpy(&v, b.blob.data.data() + f, 8);
    v += reinterpret_cast<uint64_t>(pl->blob);
    std::memcpy(b.blob.data.data() + f, &v, 8);
  }
  HIPCHK(hipMemcpy(pl->blob, b.blob.data.data(), pl->blob_bytes, hipMemcpyHostToDevice));
  pl->steps = std::move(b.steps);
  for (Step& s : pl->steps) {
    if (s.kind == S_GEMM) s.tile = pl->m3 ? 4 : 0;   // default kernels: 64x64 tiles, 16x16x4 MFMA
    if (s.kind == S_DD_GEMM) s.tile = kDefaultDDConfig;
  }
  return HSC_OK;
}

// slices: 8-bit slices per operand of the integer-matrix-core products (precision 3), kOzSlices
// for the other precisions
// Plan of this shape and instance (a call with concurrent batches holds instances 0 .. inst - 1 of
// the shape while it builds instance inst: nothing here frees those).
int build_plan(hsc_ctx* ctx, const hsc_tree* t, int B, uint32_t want, int prec, int tune, int m3, int slices,
               Plan** out, int inst = 0) {
  auto same_shape = [&](const Plan& p) {
    return p.uid == t->uid && p.B == B && p.want == want && p.prec == prec && p.tune == tune && p.m3 == m3 &&
           p.slices == slices;
  };
  auto held = [&](const std::unique_ptr<Plan>& p) { return same_shape(*p) && p->inst < inst; };
  for (size_t k = 0; k < ctx->plans.size(); ++k)
    if (same_shape(*ctx->plans[k]) && ctx->plans[k]->inst == inst) {
      // most recently used goes last
      std::unique_ptr<Plan> p = std::move(ctx->plans[k]);
      ctx->plans.erase(ctx->plans.begin() + k);
      ctx->plans.push_back(std::move(p));
      *out = ctx->plans.back().get();
      return HSC_OK;
    }
  // keep memory bounded: drop plans of this tree with other shapes, then the
  // least recently used ones beyond a few
  ctx->plans.erase(std::remove_if(ctx->plans.begin(), ctx->plans.end(),
                                  [&](const std::unique_ptr<Plan>& p) { return p->uid == t->uid && !same_shape(*p); }),
                   ctx->plans.end());
  HIPCHK(hipSetDevice(ctx->device));
  if (ctx->stream) { HIPCHK(hipStreamSynchronize(ctx->stream)); }
  else { HIPCHK(hipDeviceSynchronize()); }
  for (size_t k = 0; ctx->plans.size() > (size_t)std::max(3, inst + 1) && k < ctx->plans.size();)
    if (held(ctx->plans[k])) ++k;
    else ctx->plans.erase(ctx->plans.begin() + k);
  // drop every plan but the ones this call holds (to make room)
  auto drop_unheld = [&]() {
    ctx->plans.erase(std::remove_if(ctx->plans.begin(), ctx->plans.end(),
                                    [&](const std::unique_ptr<Plan>& p) { return !held(p); }),
                     ctx->plans.end());
  };
  for (const Cluster& c : t->cl)
    if (c.n > kMaxCluster) {
      set_error("cluster of " + std::to_string(c.n) + " sites exceeds the dense-block limit of " +
                std::to_string(kMaxCluster) + " (use a smaller leaf side)");
      return HSC_E_ARG;
    }
  std::unique_ptr<Plan> pl(new Plan());
  pl->uid = t->uid; pl->B = B; pl->want = want; pl->n = t->n; pl->prec = prec; pl->tune = tune; pl->m3 = m3;
  pl->slices = slices; pl->inst = inst;
  Builder b{t, B, want, (want & (HSC_DIAG_GL | HSC_TRANS | HSC_SPECTRAL_LR | HSC_BOND_GL)) != 0};
  b.ddf = prec >= 1;
  b.ddx = prec >= 2;
  b.oz = prec == 3;
  b.slices = slices;
  b.channels();
  b.layout();
  b.layout_faces();
  // per-plan small buffers at the end of the workspace
  const size_t o_es = b.wsa(sizeof(EnergyScalars) * B);
  const size_t o_st = b.wsa(sizeof(int32_t) * B);
  const size_t o_ar = b.wsa(sizeof(double) * (size_t)B * t->n);
  b.pot_off = b.wsa(sizeof(double) * (size_t)t->n);
  pl->ws_bytes = b.ws;
  HIPCHK(hipSetDevice(ctx->device));
  if (hipMalloc(&pl->ws, pl->ws_bytes) != hipSuccess) {
    (void)hipGetLastError();
    pl->ws = nullptr;
    // make room: drop every cached plan this call does not hold and try once more
    drop_unheld();
    if (hipMalloc(&pl->ws, pl->ws_bytes) != hipSuccess) {
      (void)hipGetLastError();
      pl->ws = nullptr;
      set_error("device workspace allocation failed (" + std::to_string(pl->ws_bytes) + " bytes)");
      return HSC_E_OOM;
    }
  }
  b.wsbase = pl->ws;
  pl->es = reinterpret_cast<EnergyScalars*>(pl->ws + o_es);
  pl->status = reinterpret_cast<int32_t*>(pl->ws + o_st);
  pl->a_r = reinterpret_cast<double*>(pl->ws + o_ar);
  pl->pot = reinterpret_cast<double*>(pl->ws + b.pot_off);
  b.blob.alloc(64);   // offset 0 stays unused: a zero field means "null", not "blob start"
  b.constants();
  const size_t o_left = b.blob.push(t->contact[0].sites);
  const size_t o_perm = b.blob.push(t->perm);
  pl->nleft = (int)t->contact[0].sites.size();
  const auto L = b.levels();
  b.face_steps();
  b.fold(L);
  if (want & (HSC_DIAG_GR | HSC_DIAG_GL | HSC_TRANS | HSC_SPECTRAL_LR | HSC_BOND_GR | HSC_BOND_GL)) {
    if (b.ddx) b.extract_g<zdd>(L);
    else b.extract_g<double2>(L);
  }
  if (b.ddx) b.face_gg<zdd>();
  else b.face_gg<double2>();
  for (size_t k = 0; k < b.chans.size(); ++k) {
    if (b.ddx) b.channel_steps<zdd>(L, (int)k);
    else b.channel_steps<double2>(L, (int)k);
  }
  const size_t o_ftj = b.ddx ? b.face_trans_jobs<zdd>() : b.face_trans_jobs<double2>();
  {
    hsc_status rc = upload_plan(b, pl.get());
    if (rc == HSC_E_OOM && b.oz_need > 0 && !pl->oz && !ctx->plans.empty()) {
      // the slice scratch did not fit beside the cached plans (nothing of this plan was uploaded
      // yet): drop the ones this call does not hold and try once more
      drop_unheld();
      rc = upload_plan(b, pl.get());
    }
    if (rc != HSC_OK) return rc;
  }
  pl->left = reinterpret_cast<int64_t*>(pl->blob + o_left);
  pl->perm = reinterpret_cast<const int64_t*>(pl->blob + o_perm);
  if (o_ftj) pl->face_tj = reinterpret_cast<const FaceTransJob*>(pl->blob + o_ftj);
  for (int c = 0; c < 2; ++c) {
    pl->lp.onsite[c] = t->contact[c].lead_onsite;
    pl->lp.hopping[c] = t->contact[c].lead_hopping;
    pl->lp.coupling[c] = t->contact[c].coupling;
  }
  if (tune) {
    const hsc_status rc = tune_plan(ctx, pl.get());
    if (rc != HSC_OK) return rc;
  }
  *out = pl.get();
  ctx->plans.push_back(std::move(pl));
  return HSC_OK;
}

size_t plan_bytes_per_slot(const hsc_tree* t, uint32_t want, int prec, int slices) {
  Builder b{t, 1, want, (want & (HSC_DIAG_GL | HSC_TRANS | HSC_SPECTRAL_LR | HSC_BOND_GL)) != 0};
  b.ddf = prec >= 1;
  b.ddx = prec >= 2;
  b.oz = prec == 3;
  b.slices = slices;
  b.channels();
  b.layout();
  b.layout_faces();
  return b.ws;
}

}  // namespace

}  // namespace hsc

using namespace hsc;

namespace {
struct GuardItem {
  int e;                                   // index into the caller's arrays
  std::shared_ptr<hsc_tree> tree;          // null: the caller's tree
  std::vector<int> bad;                    // flagged clusters of that tree
};
constexpr int kGuardSets = 8;
// flagged clusters: ||Psi_i||_inf above tau (the extract multiplies rounding
// errors of G_ff by Psi on both sides)
std::vector<int> flagged(const double* g, int nc, double tau) {
  std::vector<int> b;
  for (int i = 0; i < nc - 1; ++i)
    if (!(g[2 * i + 1] <= tau)) b.push_back(i);
  return b;
}
}  // namespace

extern "C" {

hsc_status hsc_ctx_create(int32_t device, void* hip_stream, hsc_ctx** out) {
  if (!out) { set_error("out is NULL"); return HSC_E_ARG; }
  *out = nullptr;
  int count = 0;
  if (hipGetDeviceCount(&count) != hipSuccess || count <= 0) {
    (void)hipGetLastError();
    set_error("no HIP device available");
    return HSC_E_HIP;
  }
  if (device < 0 || device >= count) { set_error("device index out of range"); return HSC_E_ARG; }
  hsc_ctx* c = new hsc_ctx();
  c->device = device;
  c->stream = reinterpret_cast<hipStream_t>(hip_stream);
  {
    // address of the allocation-free product's scratch array on this device, looked up once per
    // device (with the device current) and kept for every later context
    static std::mutex mu;
    static std::vector<char*> addr;
    std::lock_guard<std::mutex> lock(mu);
    if ((int)addr.size() < count) addr.resize(count, nullptr);
    if (!addr[device] && hipSetDevice(device) == hipSuccess)
      addr[device] = static_cast<char*>(oz_noalloc_scratch_address());
    (void)hipGetLastError();
    c->noalloc = addr[device];
  }
  *out = c;
  return HSC_OK;
}

hsc_status hsc_ctx_destroy(hsc_ctx* ctx) {
  if (!ctx) return HSC_OK;
  (void)hipSetDevice(ctx->device);
  if (ctx->stream) (void)hipStreamSynchronize(ctx->stream);
  else (void)hipDeviceSynchronize();
  // the streams of concurrent batches are joined into the context's stream by every call that
  // completes; one that failed between fork and join may have left work on them
  for (int k = 0; k < kMaxStreams; ++k)
    if (ctx->sub[k]) (void)hipStreamSynchronize(ctx->sub[k]);
  for (auto& e : ctx->ev_pool) {
    (void)hipEventDestroy(e.first);
    (void)hipEventDestroy(e.second);
  }
  ctx->plans.clear();
  if (ctx->forest) hsc_tree_destroy(ctx->forest);
  if (ctx->bstage) (void)hipFree(ctx->bstage);
  if (ctx->cap_stream) (void)hipStreamDestroy(ctx->cap_stream);
  for (int k = 0; k < kMaxStreams; ++k)
    if (ctx->sub[k]) (void)hipStreamDestroy(ctx->sub[k]);
  for (int k = 0; k <= kMaxStreams; ++k)
    if (ctx->sub_ev[k]) (void)hipEventDestroy(ctx->sub_ev[k]);
  delete ctx;
  return HSC_OK;
}

// slices per operand of a solve's integer-matrix-core products: the option (0 = kOzSlices) with
// precision 3, kOzSlices otherwise (no such products); -1 when the option is out of range
static int opts_slices(const hsc_solve_opts* o) {
  if (o->slices != 0 && (o->slices < kOzSlicesMin || o->slices > kOzSlicesMax)) return -1;
  return o->precision == 3 && o->slices != 0 ? o->slices : kOzSlices;
}

static hsc_status solve_core(hsc_ctx* ctx, const hsc_tree* tree, int32_t n_e, const double* energies,
                             const hsc_solve_opts* opts, void* diag_gr, void* diag_gl, double* trans,
                             double* spectral_lr, int32_t* status, double* guard, void* bond_gr = nullptr,
                             void* bond_gl = nullptr) {
  if (!ctx || !tree || !opts || n_e < 0) { set_error("null argument to hsc_solve"); return HSC_E_ARG; }
  if (n_e == 0) return HSC_OK;
  if (!energies) { set_error("energies is NULL"); return HSC_E_ARG; }
  if (!(opts->eta > 0.0) || !(opts->kT > 0.0)) { set_error("eta and kT must be > 0"); return HSC_E_ARG; }
  uint32_t want = opts->want;
  if ((want & HSC_DIAG_GR) && !diag_gr) { set_error("diag_gr requested but NULL"); return HSC_E_ARG; }
  if ((want & HSC_DIAG_GL) && !diag_gl) { set_error("diag_gl requested but NULL"); return HSC_E_ARG; }
  if ((want & HSC_TRANS) && !trans) { set_error("trans requested but NULL"); return HSC_E_ARG; }
  if ((want & HSC_SPECTRAL_LR) && !spectral_lr) { set_error("spectral_lr requested but NULL"); return HSC_E_ARG; }
  if ((want & HSC_BOND_GR) && !bond_gr) { set_error("bond_gr requested but NULL (bond outputs go through hsc_solve_ex)"); return HSC_E_ARG; }
  if ((want & HSC_BOND_GL) && !bond_gl) { set_error("bond_gl requested but NULL (bond outputs go through hsc_solve_ex)"); return HSC_E_ARG; }
  if ((want & (HSC_DIAG_GR | HSC_DIAG_GL | HSC_TRANS | HSC_SPECTRAL_LR | HSC_BOND_GR | HSC_BOND_GL)) == 0) {
    set_error("nothing requested");
    return HSC_E_ARG;
  }
  const int slices = opts_slices(opts);
  if (slices < 0) { set_error("slices must be 0, 15 or 16"); return HSC_E_ARG; }
  HIPCHK(hipSetDevice(ctx->device));
  int B = opts->batch;
  if (B <= 0) {
    // a plan already built for this tree and these options keeps its batch: recomputing it from
    // the memory that plan now holds would shrink the batch and rebuild the plan on every call
    for (const auto& p : ctx->plans)
      if (p->uid == tree->uid && p->want == want && p->prec == opts->precision && p->tune == (opts->tune != 0) &&
          p->m3 == opts->complex3m && p->slices == slices && p->B <= n_e)
        B = std::max(B, p->B);
  }
  if (B <= 0) {
    // as many slots as 70 % of the free memory holds (at most 64; shared by the plans of concurrent
    // batches), then the energies spread evenly over the fewest batches that count allows (no
    // mostly empty last batch)
    size_t freeb = 0, totalb = 0;
    HIPCHK(hipMemGetInfo(&freeb, &totalb));
    const size_t per = std::max<size_t>(1, plan_bytes_per_slot(tree, want, opts->precision, slices));
    const size_t plans = (size_t)std::min(std::max(opts->streams, 1), kMaxStreams);
    const int bmax = (int)std::max<size_t>(1, std::min<size_t>(64, (size_t)(0.70 * (double)freeb) / per / plans));
    const int chunks = (n_e + bmax - 1) / bmax;
    B = (n_e + chunks - 1) / chunks;
  }
  B = std::min(B, n_e);
  Plan* pl = nullptr;
  if (opts->precision < 0 || opts->precision > 3) { set_error("precision must be 0, 1, 2 or 3"); return HSC_E_ARG; }
  if (opts->complex3m != 0 && opts->complex3m != 1) { set_error("complex3m must be 0 or 1"); return HSC_E_ARG; }
  if (opts->streams < 0 || opts->streams > kMaxStreams) {
    set_error("streams must lie in [0, " + std::to_string(kMaxStreams) + "]");
    return HSC_E_ARG;
  }
  // concurrent batches: one plan (and stream) per instance, batches round-robin
  const int K = (opts->streams > 1 && n_e > B && !guard && !ctx->profile && !(want & (HSC_BOND_GR | HSC_BOND_GL)))
                    ? std::min(opts->streams, (n_e + B - 1) / B)
                    : 1;
  std::vector<Plan*> pls;
  for (int k = 0; k < K; ++k) {
    const int st = build_plan(ctx, tree, B, want, opts->precision, opts->tune != 0, opts->complex3m, slices, &pl, k);
    if (st != HSC_OK) return (hsc_status)st;
    pls.push_back(pl);
  }
  const int64_t n = tree->n;
  const bool use_graph = opts->graph != 0 && !guard && !ctx->profile && !(want & (HSC_BOND_GR | HSC_BOND_GL));
  for (Plan* p : pls) {
    // the on-site potential of this call (cluster order), or zeros once after a call that had one
    if (opts->potential) {
      launch_potential(ctx->stream, n, p->perm, opts->potential, p->pot);
      p->pot_dirty = true;
    } else if (p->pot_dirty) {
      launch_potential(ctx->stream, n, p->perm, nullptr, p->pot);
      p->pot_dirty = false;
    }
    if (use_graph) {
      const size_t row = (size_t)B * n;
      if (!p->stage && hipMalloc(&p->stage, row * 48) != hipSuccess) {
        (void)hipGetLastError();
        set_error("graph staging allocation failed");
        return HSC_E_OOM;
      }
      if (!p->gexec) {
        if (!ctx->cap_stream) HIPCHK(hipStreamCreateWithFlags(&ctx->cap_stream, hipStreamNonBlocking));
        double2* sg_gr = (double2*)p->stage;
        HIPCHK(hipStreamBeginCapture(ctx->cap_stream, hipStreamCaptureModeRelaxed));
        const int st = run_steps(ctx, ctx->cap_stream, p, 0, B, sg_gr, sg_gr + row, (double*)(sg_gr + 2 * row),
                                 nullptr, (int)tree->cl.size());
        hipGraph_t g = nullptr;
        const hipError_t ce = hipStreamEndCapture(ctx->cap_stream, &g);
        if (st != HSC_OK) {
          if (g) (void)hipGraphDestroy(g);
          return (hsc_status)st;
        }
        HIPCHK(ce);
        p->graph = g;
        HIPCHK(hipGraphInstantiate(&p->gexec, g, nullptr, nullptr, 0));
      }
    }
  }
  if (K > 1) {
    // fork: every stream of the call starts after what the context's stream holds so far
    for (int k = 0; k < K; ++k)
      if (!ctx->sub[k]) HIPCHK(hipStreamCreateWithFlags(&ctx->sub[k], hipStreamNonBlocking));
    for (int k = 0; k <= kMaxStreams; ++k)
      if (!ctx->sub_ev[k]) HIPCHK(hipEventCreateWithFlags(&ctx->sub_ev[k], hipEventDisableTiming));
    HIPCHK(hipEventRecord(ctx->sub_ev[kMaxStreams], ctx->stream));
    for (int k = 0; k < K; ++k) HIPCHK(hipStreamWaitEvent(ctx->sub[k], ctx->sub_ev[kMaxStreams], 0));
  }
  const int nseg = std::max<int>(1, (int)tree->seg_site.size() - 1);
  for (int e0 = 0, c = 0; e0 < n_e; e0 += B, ++c) {
    Plan* p = pls[c % K];
    hipStream_t s = K > 1 ? ctx->sub[c % K] : ctx->stream;
    const int nv = std::min(B, n_e - e0);
    launch_energy_setup(s, energies + e0, nv, B, opts->eta, opts->kT, opts->mu_L, opts->mu_R, p->lp, p->es,
                        p->status);
    const double* spec_rows = spectral_lr ? spectral_lr + (size_t)e0 * 2 * n : nullptr;
    if (use_graph) {
      const double2* sg_gr = (const double2*)p->stage;
      const double2* sg_gl = sg_gr + (size_t)B * n;
      const double* sg_sp = (const double*)(sg_gl + (size_t)B * n);
      HIPCHK(hipGraphLaunch(p->gexec, s));
      const size_t rows = (size_t)nv * n;
      if (want & HSC_DIAG_GR)
        HIPCHK(hipMemcpyAsync((double2*)diag_gr + (size_t)e0 * n, sg_gr, rows * 16, hipMemcpyDeviceToDevice, s));
      if (want & HSC_DIAG_GL)
        HIPCHK(hipMemcpyAsync((double2*)diag_gl + (size_t)e0 * n, sg_gl, rows * 16, hipMemcpyDeviceToDevice, s));
      if (want & HSC_SPECTRAL_LR)
        HIPCHK(hipMemcpyAsync(spectral_lr + (size_t)e0 * 2 * n, sg_sp, rows * 16, hipMemcpyDeviceToDevice, s));
      spec_rows = sg_sp;
    } else {
      const int st = run_steps(ctx, s, p, e0, nv, diag_gr, diag_gl, spectral_lr, guard, (int)tree->cl.size(),
                               bond_gr, bond_gl);
      if (st != HSC_OK) return (hsc_status)st;
    }
    if ((want & HSC_TRANS) && tree->dense) {
      launch_face_trans(s, p->face_tj, nv, e0, trans);
    } else if (want & HSC_TRANS) {
      // one transmission per device of a forest, from its own left-contact sites
      for (int d = 0; d < nseg; ++d) {
        const int64_t l0 = tree->seg_left.empty() ? 0 : tree->seg_left[d];
        const int64_t l1 = tree->seg_left.empty() ? p->nleft : tree->seg_left[d + 1];
        double* td = trans + (size_t)d * n_e;
        if (want & HSC_SPECTRAL_LR)
          launch_trans(s, spec_rows + n, 2 * n, p->left + l0, (int)(l1 - l0), B, nv, e0, p->es, td);
        else
          launch_trans(s, p->a_r, n, p->left + l0, (int)(l1 - l0), B, nv, e0, p->es, td);
      }
    }
    if ((want & HSC_SPECTRAL_LR) && (want & HSC_DIAG_GL))
      launch_combine_gl(s, spectral_lr, nv, e0, n, p->es, (double2*)diag_gl);
    if (status) launch_status_out(s, p->status, nv, status + e0);
  }
  if (K > 1) {
    // join: the context's stream continues after every batch of the call
    for (int k = 0; k < K; ++k) {
      HIPCHK(hipEventRecord(ctx->sub_ev[k], ctx->sub[k]));
      HIPCHK(hipStreamWaitEvent(ctx->stream, ctx->sub_ev[k], 0));
    }
  }
  HIPCHK(hipGetLastError());
  return HSC_OK;
}

// Growth guard: re-solve flagged energies on merged trees (delayed pivots).
// Each round, the flagged energies of one tree are grouped by their set of
// flagged clusters, and each group is solved again on a tree in which those
// clusters are merged into their parents (never beyond the dense-block limit).
// When one tree has more than kGuardSets different sets in a round, its energies
// are solved together on one tree merging the union of their sets instead: one
// plan per round and tree however many energies are flagged.  Merged trees (and
// so their plans) are kept in the context, keyed by the tree and the merged
// clusters, for later calls.  Rounds repeat until no block is flagged or the
// rounds run out.

static hsc_status guard_loop(hsc_ctx* ctx, const hsc_tree* tree, int32_t n_e, const double* energies,
                             const hsc_solve_opts* opts, void* diag_gr, void* diag_gl, double* trans,
                             double* spectral_lr, int32_t* status, double* guard_dev) {
  const int64_t n = tree->n;
  const uint32_t want = opts->want;
  std::vector<double> e_host(n_e);
  HIPCHK(hipMemcpy(e_host.data(), energies, sizeof(double) * n_e, hipMemcpyDeviceToHost));
  const int nc0 = (int)tree->cl.size();
  std::vector<double> g((size_t)n_e * nc0 * 2);
  HIPCHK(hipMemcpy(g.data(), guard_dev, sizeof(double) * g.size(), hipMemcpyDeviceToHost));
  std::vector<GuardItem> items;
  for (int e = 0; e < n_e; ++e) {
    std::vector<int> b = flagged(&g[(size_t)e * nc0 * 2], nc0, opts->guard_tau);
    if (!b.empty()) items.push_back({e, nullptr, b});
  }
  auto al = [](size_t x) { return (x + 255) / 256 * 256; };
  for (int round = 0; round < opts->guard_rounds && !items.empty(); ++round) {
    // group by (tree, flagged set); a tree with more than kGuardSets sets: one group, union of the sets
    std::sort(items.begin(), items.end(), [](const GuardItem& a, const GuardItem& b) {
      if (a.tree.get() != b.tree.get()) return a.tree.get() < b.tree.get();
      return a.bad < b.bad;
    });
    std::vector<char> unite(items.size(), 0);
    for (size_t t0 = 0; t0 < items.size();) {
      size_t t1 = t0;
      int sets = 0;
      for (; t1 < items.size() && items[t1].tree.get() == items[t0].tree.get(); ++t1)
        if (t1 == t0 || items[t1].bad != items[t1 - 1].bad) ++sets;
      if (sets > kGuardSets)
        for (size_t q = t0; q < t1; ++q) unite[q] = 1;
      t0 = t1;
    }
    std::vector<GuardItem> next;
    for (size_t g0 = 0; g0 < items.size();) {
      size_t g1 = g0;
      while (g1 < items.size() && items[g1].tree.get() == items[g0].tree.get() &&
             (unite[g0] || items[g1].bad == items[g0].bad))
        ++g1;
      const hsc_tree* t = items[g0].tree ? items[g0].tree.get() : tree;
      // merge the flagged clusters, parents first, within the block-size limit
      std::vector<char> mark(t->cl.size(), 0);
      for (size_t q = g0; q < g1; ++q)
        for (int i : items[q].bad) mark[i] = 1;
      std::vector<int64_t> size(t->cl.size());
      for (size_t i = 0; i < t->cl.size(); ++i) size[i] = t->cl[i].n;
      std::vector<int32_t> ids;
      for (int i = (int)mark.size() - 2; i >= 0; --i) {
        if (!mark[i]) continue;
        int p = t->cl[i].parent;
        while (p >= 0 && mark[p]) p = t->cl[p].parent;   // nearest surviving ancestor
        if (p < 0 || size[p] + size[i] > kMaxCluster) { mark[i] = 0; continue; }
        size[p] += size[i];
        size[i] = 0;
        ids.push_back((int32_t)i);
      }
      if (ids.empty()) {   // nothing can be merged: these energies stay flagged
        for (size_t q = g0; q < g1; ++q) next.push_back(items[q]);
        g0 = g1;
        continue;
      }
      std::vector<int64_t> key{(int64_t)t->uid};
      key.insert(key.end(), ids.begin(), ids.end());
      std::shared_ptr<hsc_tree> mt;
      for (size_t c = 0; c < ctx->guard_trees.size(); ++c)
        if (ctx->guard_trees[c].first == key) {
          mt = ctx->guard_trees[c].second;
          auto kept = ctx->guard_trees[c];
          ctx->guard_trees.erase(ctx->guard_trees.begin() + c);
          ctx->guard_trees.push_back(kept);
          break;
        }
      hsc_status rc = HSC_OK;
      if (!mt) {
        hsc_tree* mm = nullptr;
        rc = hsc_tree_merge(t, (int32_t)ids.size(), ids.data(), &mm);
        if (rc != HSC_OK) return rc;
        mt = std::shared_ptr<hsc_tree>(mm, hsc_tree_destroy);
        ctx->guard_trees.push_back({key, mt});
        while (ctx->guard_trees.size() > 4) ctx->guard_trees.erase(ctx->guard_trees.begin());
      }
      hsc_tree* m = mt.get();
      const int nc = (int)m->cl.size();
      const int k = (int)(g1 - g0);
      std::vector<double> eh(k);
      for (int q = 0; q < k; ++q) eh[q] = e_host[items[g0 + q].e];
      const size_t o_e = 0, o_gr = al(8 * (size_t)k), o_gl = al(o_gr + 16 * (size_t)k * n),
                   o_sp = al(o_gl + 16 * (size_t)k * n), o_tr = al(o_sp + 16 * (size_t)k * n),
                   o_st = al(o_tr + 8 * (size_t)k), o_gd = al(o_st + 4 * (size_t)k),
                   bytes = al(o_gd + 16 * (size_t)k * nc);
      char* tmp = nullptr;
      if (hipMalloc(&tmp, bytes) != hipSuccess) { (void)hipGetLastError(); set_error("guard temporaries"); return HSC_E_OOM; }
      std::unique_ptr<char, hipError_t (*)(void*)> hold(tmp, hipFree);
      HIPCHK(hipMemcpy(tmp + o_e, eh.data(), 8 * k, hipMemcpyHostToDevice));
      rc = solve_core(ctx, m, k, (double*)(tmp + o_e), opts, tmp + o_gr, tmp + o_gl, (double*)(tmp + o_tr),
                      (double*)(tmp + o_sp), (int32_t*)(tmp + o_st), (double*)(tmp + o_gd));
      if (rc != HSC_OK) return rc;
      hipStream_t st = ctx->stream;
      for (int q = 0; q < k; ++q) {
        const int e = items[g0 + q].e;
        if ((want & HSC_DIAG_GR) && diag_gr)
          HIPCHK(hipMemcpyAsync((char*)diag_gr + 16 * (size_t)e * n, tmp + o_gr + 16 * (size_t)q * n, 16 * n,
                                hipMemcpyDeviceToDevice, st));
        if ((want & HSC_DIAG_GL) && diag_gl)
          HIPCHK(hipMemcpyAsync((char*)diag_gl + 16 * (size_t)e * n, tmp + o_gl + 16 * (size_t)q * n, 16 * n,
                                hipMemcpyDeviceToDevice, st));
        if ((want & HSC_SPECTRAL_LR) && spectral_lr)
          HIPCHK(hipMemcpyAsync(spectral_lr + 2 * (size_t)e * n, tmp + o_sp + 16 * (size_t)q * n, 16 * n,
                                hipMemcpyDeviceToDevice, st));
        if ((want & HSC_TRANS) && trans)
          HIPCHK(hipMemcpyAsync(trans + e, tmp + o_tr + 8 * (size_t)q, 8, hipMemcpyDeviceToDevice, st));
        if (status)
          HIPCHK(hipMemcpyAsync(status + e, tmp + o_st + 4 * (size_t)q, 4, hipMemcpyDeviceToDevice, st));
      }
      std::vector<double> gk((size_t)k * nc * 2);
      HIPCHK(hipMemcpyAsync(gk.data(), tmp + o_gd, sizeof(double) * gk.size(), hipMemcpyDeviceToHost, st));
      HIPCHK(st ? hipStreamSynchronize(st) : hipDeviceSynchronize());
      for (int q = 0; q < k; ++q) {
        std::vector<int> b = flagged(&gk[(size_t)q * nc * 2], nc, opts->guard_tau);
        if (!b.empty()) next.push_back({items[g0 + q].e, mt, b});
      }
      g0 = g1;
    }
    items.swap(next);
  }
  if (!items.empty() && status) {
    const int32_t code = HSC_E_UNSTABLE;
    for (const GuardItem& it : items) HIPCHK(hipMemcpy(status + it.e, &code, 4, hipMemcpyHostToDevice));
  }
  return HSC_OK;
}

hsc_status hsc_solve_ex(hsc_ctx* ctx, const hsc_tree* tree, int32_t n_e, const double* energies,
                        const hsc_solve_opts* opts, const hsc_outputs* out) {
  if (!out || !opts) { set_error("null argument to hsc_solve_ex"); return HSC_E_ARG; }
  if ((opts->want & (HSC_BOND_GR | HSC_BOND_GL)) == 0)
    return hsc_solve(ctx, tree, n_e, energies, opts, out->diag_gr, out->diag_gl, out->trans, out->spectral_lr,
                     out->status, out->guard);
  if (opts->guard_tau > 0.0) { set_error("bond outputs do not combine with the growth guard"); return HSC_E_ARG; }
  return solve_core(ctx, tree, n_e, energies, opts, out->diag_gr, out->diag_gl, out->trans, out->spectral_lr,
                    out->status, out->guard, out->bond_gr, out->bond_gl);
}

hsc_status hsc_solve(hsc_ctx* ctx, const hsc_tree* tree, int32_t n_e, const double* energies,
                     const hsc_solve_opts* opts, void* diag_gr, void* diag_gl, double* trans,
                     double* spectral_lr, int32_t* status, double* guard) {
  if (!opts || !(opts->guard_tau > 0.0))
    return solve_core(ctx, tree, n_e, energies, opts, diag_gr, diag_gl, trans, spectral_lr, status, guard);
  if (!ctx || !tree || n_e < 0 || opts->guard_rounds < 0) { set_error("bad arguments to hsc_solve"); return HSC_E_ARG; }
  if (tree->dense) { set_error("the growth guard merges clusters: not available with whole-face contacts"); return HSC_E_ARG; }
  if (n_e == 0) return HSC_OK;
  HIPCHK(hipSetDevice(ctx->device));
  double* gd = guard;
  char* own = nullptr;
  if (!gd) {
    if (hipMalloc(&own, sizeof(double) * 2 * (size_t)n_e * tree->cl.size()) != hipSuccess) {
      (void)hipGetLastError();
      set_error("guard buffer allocation failed");
      return HSC_E_OOM;
    }
    gd = (double*)own;
  }
  hsc_status rc = solve_core(ctx, tree, n_e, energies, opts, diag_gr, diag_gl, trans, spectral_lr, status, gd);
  if (rc == HSC_OK) {
    if (ctx->stream) { HIPCHK(hipStreamSynchronize(ctx->stream)); } else { HIPCHK(hipDeviceSynchronize()); }
    rc = guard_loop(ctx, tree, n_e, energies, opts, diag_gr, diag_gl, trans, spectral_lr, status, gd);
  }
  if (own) {
    (void)hipDeviceSynchronize();
    (void)hipFree(own);
  }
  return rc;
}

static hsc_status solve_each(hsc_ctx* ctx, int32_t n_trees, const hsc_tree* const* trees, const int32_t* n_e,
                             const double* const* energies, const hsc_solve_opts* opts, void* const* diag_gr,
                             void* const* diag_gl, double* const* trans, double* const* spectral_lr,
                             int32_t* const* status, double* const* guard) {
  for (int d = 0; d < n_trees; ++d) {
    hsc_status s = hsc_solve(ctx, trees[d], n_e[d], energies[d], opts, diag_gr ? diag_gr[d] : nullptr,
                             diag_gl ? diag_gl[d] : nullptr, trans ? trans[d] : nullptr,
                             spectral_lr ? spectral_lr[d] : nullptr, status ? status[d] : nullptr,
                             guard ? guard[d] : nullptr);
    if (s != HSC_OK) return s;
  }
  return HSC_OK;
}

// one forest of n_trees devices with a shared energy list; outputs staged and copied per device
static hsc_status solve_forest(hsc_ctx* ctx, int32_t n_trees, const hsc_tree* const* trees, int ne,
                               const double* energies, const hsc_solve_opts* opts, void* const* diag_gr,
                               void* const* diag_gl, double* const* trans, double* const* spectral_lr,
                               int32_t* const* status) {
  const uint32_t want = opts->want;
  std::vector<uint64_t> key;
  for (int d = 0; d < n_trees; ++d) key.push_back(trees[d]->uid);
  if (!ctx->forest || ctx->forest_key != key) {
    if (ctx->forest) {
      const uint64_t old = ctx->forest->uid;
      ctx->plans.erase(std::remove_if(ctx->plans.begin(), ctx->plans.end(),
                                      [&](const std::unique_ptr<Plan>& p) { return p->uid == old; }),
                       ctx->plans.end());
      hsc_tree_destroy(ctx->forest);
      ctx->forest = nullptr;
      ctx->forest_key.clear();
    }
    hsc_tree* f = nullptr;
    hsc_status rc = hsc_tree_concat(n_trees, trees, &f);
    if (rc != HSC_OK) return rc;
    ctx->forest = f;
    ctx->forest_key = key;
  }
  const hsc_tree* F = ctx->forest;
  const int64_t N = F->n;
  // staging: gr, gl [ne][N] complex; spectral [ne][2][N]; trans [n_trees][ne]; status [ne]
  auto al = [](size_t x) { return (x + 255) / 256 * 256; };
  const size_t o_gr = 0, o_gl = al(o_gr + 16 * (size_t)ne * N), o_sp = al(o_gl + 16 * (size_t)ne * N),
               o_tr = al(o_sp + 16 * (size_t)ne * N), o_st = al(o_tr + 8 * (size_t)ne * n_trees),
               bytes = al(o_st + 4 * (size_t)ne);
  if (ctx->bstage_bytes < bytes) {
    if (ctx->bstage) {
      HIPCHK(hipDeviceSynchronize());
      (void)hipFree(ctx->bstage);
      ctx->bstage = nullptr;
      ctx->bstage_bytes = 0;
    }
    if (hipMalloc(&ctx->bstage, bytes) != hipSuccess) {
      (void)hipGetLastError();
      set_error("hsc_solve_batch: output staging allocation failed");
      return HSC_E_OOM;
    }
    ctx->bstage_bytes = bytes;
  }
  char* sb = ctx->bstage;
  hsc_status rc = solve_core(ctx, F, ne, energies, opts, sb + o_gr, sb + o_gl, (double*)(sb + o_tr),
                             (double*)(sb + o_sp), (int32_t*)(sb + o_st), nullptr);
  if (rc != HSC_OK) return rc;
  hipStream_t st = ctx->stream;
  for (int d = 0; d < n_trees; ++d) {
    const int64_t s0 = F->seg_site[d], nd = F->seg_site[d + 1] - s0;
    if (want & HSC_DIAG_GR)
      HIPCHK(hipMemcpy2DAsync(diag_gr[d], 16 * nd, sb + o_gr + 16 * s0, 16 * N, 16 * nd, ne, hipMemcpyDeviceToDevice, st));
    if (want & HSC_DIAG_GL)
      HIPCHK(hipMemcpy2DAsync(diag_gl[d], 16 * nd, sb + o_gl + 16 * s0, 16 * N, 16 * nd, ne, hipMemcpyDeviceToDevice, st));
    if (want & HSC_SPECTRAL_LR)
      HIPCHK(hipMemcpy2DAsync(spectral_lr[d], 8 * nd, sb + o_sp + 8 * s0, 8 * N, 8 * nd, 2 * (size_t)ne,
                              hipMemcpyDeviceToDevice, st));
    if (want & HSC_TRANS)
      HIPCHK(hipMemcpyAsync(trans[d], sb + o_tr + 8 * (size_t)d * ne, 8 * (size_t)ne, hipMemcpyDeviceToDevice, st));
    if (status && status[d])
      HIPCHK(hipMemcpyAsync(status[d], sb + o_st, 4 * (size_t)ne, hipMemcpyDeviceToDevice, st));
  }
  return HSC_OK;
}

hsc_status hsc_solve_batch(hsc_ctx* ctx, int32_t n_trees, const hsc_tree* const* trees, const int32_t* n_e,
                           const double* const* energies, const hsc_solve_opts* opts, void* const* diag_gr,
                           void* const* diag_gl, double* const* trans, double* const* spectral_lr,
                           int32_t* const* status, double* const* guard) {
  if (!ctx || !opts || n_trees < 0 || (n_trees > 0 && (!trees || !n_e || !energies))) {
    set_error("bad arguments to hsc_solve_batch");
    return HSC_E_ARG;
  }
  for (int d = 0; d < n_trees; ++d)
    if (!trees[d] || n_e[d] < 0 || (n_e[d] > 0 && !energies[d])) { set_error("bad device entry in hsc_solve_batch"); return HSC_E_ARG; }
  if (opts_slices(opts) < 0) { set_error("slices must be 0, 15 or 16"); return HSC_E_ARG; }
  if (opts->potential) { set_error("an on-site potential applies to single-device solves"); return HSC_E_ARG; }
  if (n_trees <= 1 || opts->guard_tau > 0.0 || guard)
    return solve_each(ctx, n_trees, trees, n_e, energies, opts, diag_gr, diag_gl, trans, spectral_lr, status, guard);
  // one forest when every device has the same energies and lead model (and per-site leads)
  const int ne = n_e[0];
  bool same = ne > 0;
  for (int d = 0; d < n_trees && same; ++d) same = !trees[d]->dense;
  for (int d = 1; d < n_trees && same; ++d) same = n_e[d] == ne;
  for (int d = 1; d < n_trees && same; ++d)
    for (int k = 0; k < 2 && same; ++k) {
      const auto &a = trees[0]->contact[k], &b = trees[d]->contact[k];
      same = a.lead_onsite == b.lead_onsite && a.lead_hopping == b.lead_hopping && a.coupling == b.coupling;
    }
  HIPCHK(hipSetDevice(ctx->device));
  std::vector<double> e0h(same ? ne : 0), edh(same ? ne : 0);
  if (same) HIPCHK(hipMemcpy(e0h.data(), energies[0], 8 * (size_t)ne, hipMemcpyDeviceToHost));
  for (int d = 1; d < n_trees && same; ++d) {
    if (energies[d] == energies[0]) continue;
    HIPCHK(hipMemcpy(edh.data(), energies[d], 8 * (size_t)ne, hipMemcpyDeviceToHost));
    same = std::memcmp(e0h.data(), edh.data(), 8 * (size_t)ne) == 0;
  }
  if (!same)
    return solve_each(ctx, n_trees, trees, n_e, energies, opts, diag_gr, diag_gl, trans, spectral_lr, status, guard);
  const uint32_t want = opts->want;
  for (int d = 0; d < n_trees; ++d)
    if (((want & HSC_DIAG_GR) && !(diag_gr && diag_gr[d])) || ((want & HSC_DIAG_GL) && !(diag_gl && diag_gl[d])) ||
        ((want & HSC_TRANS) && !(trans && trans[d])) || ((want & HSC_SPECTRAL_LR) && !(spectral_lr && spectral_lr[d]))) {
      set_error("hsc_solve_batch: a requested output of a device is NULL");
      return HSC_E_ARG;
    }
  // devices go into forests in order, each forest's workspace per energy slot within
  // 0.45/4 of the free memory (room for about six energy slots at the default batch);
  // a device above that budget on its own is solved alone
  size_t freeb = 0, totalb = 0;
  HIPCHK(hipMemGetInfo(&freeb, &totalb));
  const double budget = 0.45 * (double)freeb / 4.0;
  std::vector<std::pair<int, int>> groups;
  {
    int g0 = 0;
    double acc = 0;
    for (int d = 0; d < n_trees; ++d) {
      const double bd = (double)plan_bytes_per_slot(trees[d], want, opts->precision, opts_slices(opts));
      if (d > g0 && acc + bd > budget) {
        groups.push_back({g0, d});
        g0 = d;
        acc = 0;
      }
      acc += bd;
    }
    groups.push_back({g0, n_trees});
  }
  for (const auto& g : groups) {
    if (g.second - g.first == 1) {
      const int d = g.first;
      hsc_status rc = hsc_solve(ctx, trees[d], ne, energies[d], opts, diag_gr ? diag_gr[d] : nullptr,
                                diag_gl ? diag_gl[d] : nullptr, trans ? trans[d] : nullptr,
                                spectral_lr ? spectral_lr[d] : nullptr, status ? status[d] : nullptr, nullptr);
      if (rc != HSC_OK) return rc;
      continue;
    }
    hsc_status rc = solve_forest(ctx, g.second - g.first, trees + g.first, ne, energies[g.first], opts,
                                 diag_gr ? diag_gr + g.first : nullptr, diag_gl ? diag_gl + g.first : nullptr,
                                 trans ? trans + g.first : nullptr, spectral_lr ? spectral_lr + g.first : nullptr,
                                 status ? status + g.first : nullptr);
    if (rc != HSC_OK) return rc;
  }
  return HSC_OK;
}

hsc_status hsc_sync(hsc_ctx* ctx) {
  if (!ctx) { set_error("null ctx"); return HSC_E_ARG; }
  HIPCHK(hipSetDevice(ctx->device));
  if (ctx->stream) { HIPCHK(hipStreamSynchronize(ctx->stream)); }
  else { HIPCHK(hipDeviceSynchronize()); }
  // concurrent batches of a call that failed before its join
  for (int k = 0; k < kMaxStreams; ++k)
    if (ctx->sub[k]) HIPCHK(hipStreamSynchronize(ctx->sub[k]));
  HIPCHK(hipGetLastError());
  return fold_events(ctx);   // recorded launch timings into the per-kind totals
}

hsc_status hsc_totals(hsc_ctx* ctx, int32_t n_e, int64_t n, const void* diag_gr, const void* diag_gl,
                      const double* spectral_lr, double* totals) {
  if (!ctx || n_e < 0 || n < 0 || (n_e > 0 && !totals)) { set_error("bad arguments to hsc_totals"); return HSC_E_ARG; }
  if (n_e == 0) return HSC_OK;
  HIPCHK(hipSetDevice(ctx->device));
  launch_totals(ctx->stream, n_e, n, (const double2*)diag_gr, (const double2*)diag_gl, spectral_lr, totals);
  HIPCHK(hipGetLastError());
  return HSC_OK;
}

hsc_status hsc_scf(hsc_ctx* ctx, const hsc_tree* tree, const hsc_grid* grid, int32_t n_e, const double* energies,
                   const double* weights, const hsc_solve_opts* opts, const hsc_scf_opts* scf, double* u,
                   double* density, int32_t* iterations, double* residuals) {
  std::string why;
  if (!ctx || !tree || !opts || !scf || n_e < 1 || !energies || !weights || !u || !density || !iterations ||
      poisson_check(grid, &why) != 0 || scf->max_iter < 1 || !(scf->mixing > 0.0 && scf->mixing <= 1.0) ||
      !(scf->coupling >= 0.0) || !(scf->tol >= 0.0) || scf->history < 0 || scf->history > kScfMaxHistory) {
    set_error(why.empty() ? std::string("bad arguments to hsc_scf") : "hsc_scf: " + why);
    return HSC_E_ARG;
  }
  const int64_t n = tree->n;
  if ((int64_t)grid->nx * grid->ny * grid->nz != n) {
    set_error("hsc_scf: the grid has " + std::to_string((int64_t)grid->nx * grid->ny * grid->nz) +
              " points, the tree " + std::to_string(n) + " sites");
    return HSC_E_ARG;
  }
  *iterations = 0;
  HIPCHK(hipSetDevice(ctx->device));
  PoissonWork pw;
  if (pw.create(*grid) != 0) { set_error("hsc_scf: Poisson workspace allocation failed"); return HSC_E_OOM; }
  char* buf = nullptr;
  // diag G^< [n_e][n], U_new [n], per-energy status [n_e], residual bits; with Anderson mixing f, the
  // previous U and f, the m differences of each, and the step's coefficients and slot order
  const int m = scf->history;
  auto pad = [](size_t v) { return (v + 255) / 256 * 256; };
  const size_t o_un = pad((size_t)n_e * n * 16), o_st = o_un + pad((size_t)n * 8), o_r = o_st + pad((size_t)n_e * 4),
               o_f = o_r + 256, o_hist = o_f + (m ? pad((size_t)n * 8 * (3 + 2 * (size_t)m)) : 0),
               total = o_hist + (m ? pad((size_t)m * 12) : 0);
  if (hipMalloc(&buf, total) != hipSuccess) {
    (void)hipGetLastError();
    pw.destroy();
    set_error("hsc_scf: buffer allocation failed (" + std::to_string(total) + " bytes)");
    return HSC_E_OOM;
  }
  void* gl = buf;
  double* u_new = reinterpret_cast<double*>(buf + o_un);
  int32_t* status = reinterpret_cast<int32_t*>(buf + o_st);
  unsigned long long* rbits = reinterpret_cast<unsigned long long*>(buf + o_r);
  double* f = m ? reinterpret_cast<double*>(buf + o_f) : nullptr;
  double* u_prev = m ? f + n : nullptr;
  double* f_prev = m ? f + 2 * n : nullptr;
  double* dX = m ? f + 3 * n : nullptr;
  double* dF = m ? dX + (size_t)m * n : nullptr;
  double* gamma_d = m ? reinterpret_cast<double*>(buf + o_hist) : nullptr;
  int32_t* order_d = m ? reinterpret_cast<int32_t*>(gamma_d + m) : nullptr;
  std::vector<int32_t> order;   // history slots, oldest first
  int pushes = 0;
  std::vector<double> a_h, b_h, gamma_h(m > 0 ? m : 1);
  hsc_solve_opts o = *opts;
  o.want = HSC_DIAG_GL;
  o.potential = u;
  hsc_status rc = HSC_OK;
  std::vector<int32_t> st_h(n_e);
  for (int it = 0; it < scf->max_iter && rc == HSC_OK; ++it) {
    rc = hsc_solve(ctx, tree, n_e, energies, &o, nullptr, gl, nullptr, nullptr, status, nullptr);
    if (rc != HSC_OK) break;
    launch_density(ctx->stream, n_e, n, weights, gl, density);
    pw.run(ctx->stream, nullptr, density, scf->n0, scf->coupling, u_new);
    hipError_t e = hipSuccess;
    if (m == 0) {
      launch_mix(ctx->stream, n, u, u_new, scf->mixing, rbits);
    } else {
      launch_scf_resid(ctx->stream, n, u, u_new, f, rbits);
      int slot = -1;
      if (it > 0) {
        slot = pushes++ % m;
        order.push_back(slot);
        if ((int)order.size() > m) order.erase(order.begin());
      }
      launch_scf_hist(ctx->stream, n, u, f, u_prev, f_prev, slot >= 0 ? dX + (size_t)slot * n : nullptr,
                      slot >= 0 ? dF + (size_t)slot * n : nullptr);
      int mk = (int)order.size();
      if (mk > 0) {
        a_h.resize((size_t)mk * n);
        b_h.resize(n);
        for (int j = 0; j < mk && e == hipSuccess; ++j)
          e = hipMemcpyAsync(a_h.data() + (size_t)j * n, dF + (size_t)order[j] * n, 8 * (size_t)n,
                             hipMemcpyDeviceToHost, ctx->stream);
        if (e == hipSuccess) e = hipMemcpyAsync(b_h.data(), f, 8 * (size_t)n, hipMemcpyDeviceToHost, ctx->stream);
        if (e == hipSuccess) e = ctx->stream ? hipStreamSynchronize(ctx->stream) : hipDeviceSynchronize();
        if (e == hipSuccess && !lstsq_householder(n, mk, a_h, b_h, gamma_h.data())) {
          order.clear();   // numerically dependent differences: a plain linear step, history restarts
          mk = 0;
        }
        if (e == hipSuccess && mk > 0) {
          e = hipMemcpyAsync(gamma_d, gamma_h.data(), 8 * (size_t)mk, hipMemcpyHostToDevice, ctx->stream);
          if (e == hipSuccess)
            e = hipMemcpyAsync(order_d, order.data(), 4 * (size_t)mk, hipMemcpyHostToDevice, ctx->stream);
        }
      }
      if (e == hipSuccess) launch_scf_update(ctx->stream, n, u, f, scf->mixing, mk, dX, dF, order_d, gamma_d);
    }
    unsigned long long rb = 0;
    if (e == hipSuccess) e = hipGetLastError();
    if (e == hipSuccess) e = hipMemcpyAsync(st_h.data(), status, 4 * (size_t)n_e, hipMemcpyDeviceToHost, ctx->stream);
    if (e == hipSuccess) e = hipMemcpyAsync(&rb, rbits, 8, hipMemcpyDeviceToHost, ctx->stream);
    if (e == hipSuccess) e = ctx->stream ? hipStreamSynchronize(ctx->stream) : hipDeviceSynchronize();
    if (e != hipSuccess) {
      set_error(std::string("HIP error in hsc_scf: ") + hipGetErrorString(e));
      rc = HSC_E_HIP;
      break;
    }
    for (int k = 0; k < n_e; ++k)
      if (st_h[k] != 0) {
        set_error("hsc_scf: energy " + std::to_string(k) + " of iteration " + std::to_string(it) + " has status " +
                  std::to_string(st_h[k]));
        rc = (hsc_status)st_h[k];
        break;
      }
    if (rc != HSC_OK) break;
    double r;
    std::memcpy(&r, &rb, 8);
    if (residuals) residuals[it] = r;
    *iterations = it + 1;
    if (r < scf->tol) break;
  }
  (void)hipFree(buf);
  pw.destroy();
  return rc;
}

hsc_status hsc_ctx_profile(hsc_ctx* ctx, int32_t enable) {
  if (!ctx) { set_error("null ctx"); return HSC_E_ARG; }
  ctx->profile = enable != 0;
  ctx->ev_used = 0;
  std::memset(ctx->prof, 0, sizeof(ctx->prof));
  std::memset(ctx->prof_bytes, 0, sizeof(ctx->prof_bytes));
  ctx->launch_log.clear();
  return HSC_OK;
}

hsc_status hsc_ctx_profile_bytes(hsc_ctx* ctx, double* out, int32_t n_kinds) {
  if (!ctx || !out || n_kinds < 0) { set_error("bad arguments"); return HSC_E_ARG; }
  for (int k = 0; k < n_kinds && k < kStepKinds; ++k) out[k] = ctx->prof_bytes[k];
  return HSC_OK;
}

hsc_status hsc_ctx_profile_launches(hsc_ctx* ctx, int64_t max_launches, double* out, int64_t* count) {
  if (!ctx || !count || max_launches < 0 || (max_launches > 0 && !out)) { set_error("bad arguments"); return HSC_E_ARG; }
  const int64_t n = (int64_t)(ctx->launch_log.size() / 4);
  *count = n;
  const int64_t m = std::min(n, max_launches);
  if (m > 0) std::memcpy(out, ctx->launch_log.data(), sizeof(double) * 4 * (size_t)m);
  return HSC_OK;
}

hsc_status hsc_ctx_profile_read(hsc_ctx* ctx, double* out, int32_t n_kinds) {
  if (!ctx || !out || n_kinds < 0) { set_error("bad arguments"); return HSC_E_ARG; }
  for (int k = 0; k < n_kinds && k < kStepKinds; ++k)
    for (int q = 0; q < 3; ++q) out[3 * k + q] = ctx->prof[k][q];
  return HSC_OK;
}

}  // extern "C"

// ---------------------------------------------------------------------------------------------
// kernel-level entry points (synchronous: they return after the work is done)

namespace hsc {
namespace {

size_t oz_pad(size_t v, size_t a) { return (v + a - 1) / a * a; }

// one product on the integer matrix cores (split A', split B', slice product), synchronous
hsc_status kern_zgemm_oz(hsc_ctx* ctx, int slices, int opA, int opB, int M, int N, int K, int negate, const void* A,
                         int lda, const void* B, int ldb, int beta, const void* C, int ldc, void* D, int ldd) {
  const int Mp = (int)oz_pad(M, 32), Np = (int)oz_pad(N, 32), Kp = (int)oz_pad(K, 64);
  const size_t sa = (size_t)3 * slices * Mp * Kp, sb = (size_t)3 * slices * Np * Kp;
  const int ba = (Mp + 63) / 64, bb = (Np + 63) / 64;
  const int ta = ba * (Kp / 32), tb = bb * (Kp / 32);
  const int tiles = (Mp / 32) * (Np / 32);
  // layout: [jobs: A, B split; product][maps: scale blocks, digit tiles, product tiles][A8][B8][ea][eb]
  const size_t nmap = (size_t)(ba + bb) + (size_t)(ta + tb) + (size_t)tiles;
  const size_t o_map = 1024, o_a8 = oz_pad(o_map + 4 * nmap, 256);
  const size_t o_b8 = oz_pad(o_a8 + sa, 256), o_ea = oz_pad(o_b8 + sb, 256), o_eb = oz_pad(o_ea + 4 * (size_t)Mp, 256);
  const size_t bytes = o_eb + 4 * (size_t)Np;
  char* dev = nullptr;
  if (hipMalloc(&dev, bytes) != hipSuccess) { (void)hipGetLastError(); set_error("alloc failed"); return HSC_E_OOM; }
  OzSplitJob job[2] = {};
  OzSplitJob& ja = job[0];
  OzSplitJob& jb = job[1];
  ja.X = (const zdd*)A; ja.R = M; ja.K = K; ja.Rp = Mp; ja.Kp = Kp;
  if (opA == 0) { ja.ldr = lda; ja.ldk = 1; } else { ja.ldr = 1; ja.ldk = lda; }
  ja.out = (int8_t*)(dev + o_a8); ja.ex = (int32_t*)(dev + o_ea);
  ja.blk_off = 0; ja.tile_off = 0;
  jb.X = (const zdd*)B; jb.R = N; jb.K = K; jb.Rp = Np; jb.Kp = Kp;
  if (opB == 0) { jb.ldr = 1; jb.ldk = ldb; } else { jb.ldr = ldb; jb.ldk = 1; }
  jb.out = (int8_t*)(dev + o_b8); jb.ex = (int32_t*)(dev + o_eb);
  jb.blk_off = ba; jb.tile_off = ta;
  GemmProbOZ p{};
  p.A8 = ja.out; p.B8 = jb.out; p.ea = ja.ex; p.eb = jb.ex;
  p.C = (const zdd*)C; p.D = (zdd*)D; p.D64 = nullptr;
  p.M = M; p.N = N; p.Mp = Mp; p.Np = Np; p.Kp = Kp; p.ldc = ldc; p.ldd = ldd; p.ldd64 = 0;
  p.tiles_n = Np / 32; p.tile_off = 0;
  std::vector<char> host(o_map + 4 * nmap, 0);
  std::memcpy(host.data(), job, sizeof(job));
  std::memcpy(host.data() + 512, &p, sizeof(p));
  int32_t* m = reinterpret_cast<int32_t*>(host.data() + o_map);
  for (int b = 0; b < ba + bb; ++b) m[b] = b < ba ? 0 : 1;                        // scale blocks
  for (int b = 0; b < ta + tb; ++b) m[ba + bb + b] = b < ta ? 0 : 1;              // digit tiles
  // product tiles: all 0 (one problem)
  hipError_t e = hipMemcpy(dev, host.data(), host.size(), hipMemcpyHostToDevice);
  if (e == hipSuccess) {
    const int32_t* dm = (const int32_t*)(dev + o_map);
    launch_oz_split(ctx->stream, slices, (const OzSplitJob*)dev, dm, ba + bb, dm + ba + bb, ta + tb);
    launch_oz_gemm(ctx->stream, slices, (const GemmProbOZ*)(dev + 512), dm + ba + bb + ta + tb, tiles, negate, beta);
    e = hipGetLastError();
    if (e == hipSuccess) e = ctx->stream ? hipStreamSynchronize(ctx->stream) : hipDeviceSynchronize();
  }
  (void)hipFree(dev);
  if (e != hipSuccess) {
    set_error(std::string("HIP error in hsc_kern_zgemm_dd: ") + hipGetErrorString(e));
    return HSC_E_HIP;
  }
  return HSC_OK;
}

}  // namespace
}  // namespace hsc

extern "C" {

hsc_status hsc_kern_zgemm(hsc_ctx* ctx, int32_t opA, int32_t opB, int32_t M, int32_t N, int32_t K,
                          double alpha_re, double alpha_im, const void* A, int32_t lda, const void* B,
                          int32_t ldb, int32_t beta, const void* C, int32_t ldc, void* D, int32_t ldd) {
  return hsc_kern_zgemm_tile(ctx, 0, opA, opB, M, N, K, alpha_re, alpha_im, A, lda, B, ldb, beta, C, ldc, D, ldd);
}

hsc_status hsc_kern_zgemm_tile(hsc_ctx* ctx, int32_t tile_kind, int32_t opA, int32_t opB, int32_t M, int32_t N,
                               int32_t K, double alpha_re, double alpha_im, const void* A, int32_t lda,
                               const void* B, int32_t ldb, int32_t beta, const void* C, int32_t ldc, void* D,
                               int32_t ldd) {
  if (!ctx || M < 0 || N < 0 || K < 0 || opA < 0 || opA > 2 || opB < 0 || opB > 2 || (beta != 0 && beta != 1) ||
      tile_kind < 0 || tile_kind >= gemm_tile_kinds()) {
    set_error("bad arguments to hsc_kern_zgemm");
    return HSC_E_ARG;
  }
  const int a_cols = opA == OP_N ? K : M, b_cols = opB == OP_N ? N : K;
  if ((K > 0 && M > 0 && (!A || lda < a_cols)) || (K > 0 && N > 0 && (!B || ldb < b_cols)) || !D ||
      ldd < N || (beta && (!C || ldc < N))) {
    set_error("bad pointer or leading dimension in hsc_kern_zgemm");
    return HSC_E_ARG;
  }
  if (M == 0 || N == 0) return HSC_OK;
  HIPCHK(hipSetDevice(ctx->device));
  GemmProb p{};
  p.A = (const double2*)A; p.B = (const double2*)B; p.C = (const double2*)C; p.D = (double2*)D;
  p.M = M; p.N = N; p.K = K; p.lda = lda; p.ldb = ldb; p.ldc = ldc; p.ldd = ldd;
  p.tiles_n = (N + gemm_tile_n(tile_kind) - 1) / gemm_tile_n(tile_kind);
  p.tile_off = 0;
  const int tiles = ((M + gemm_tile_m(tile_kind) - 1) / gemm_tile_m(tile_kind)) * p.tiles_n;
  std::vector<int32_t> map(tiles, 0);
  char* dev = nullptr;
  const size_t bytes = 256 + sizeof(int32_t) * tiles;
  if (hipMalloc(&dev, bytes) != hipSuccess) { (void)hipGetLastError(); set_error("alloc failed"); return HSC_E_OOM; }
  hipError_t e1 = hipMemcpy(dev, &p, sizeof(p), hipMemcpyHostToDevice);
  hipError_t e2 = hipMemcpy(dev + 256, map.data(), sizeof(int32_t) * tiles, hipMemcpyHostToDevice);
  if (e1 == hipSuccess && e2 == hipSuccess) {
    launch_gemm(ctx->stream, opA, opB, (const GemmProb*)dev, (const int32_t*)(dev + 256), tiles, alpha_re,
                alpha_im, beta, tile_kind);
    e1 = hipGetLastError();
    if (e1 == hipSuccess) e1 = ctx->stream ? hipStreamSynchronize(ctx->stream) : hipDeviceSynchronize();
  }
  (void)hipFree(dev);
  if (e1 != hipSuccess || e2 != hipSuccess) {
    set_error(std::string("HIP error in hsc_kern_zgemm: ") + hipGetErrorString(e1 != hipSuccess ? e1 : e2));
    return HSC_E_HIP;
  }
  return HSC_OK;
}

hsc_status hsc_kern_zgemm_dd(hsc_ctx* ctx, int32_t config, int32_t opA, int32_t opB, int32_t M, int32_t N,
                             int32_t K, int32_t negate, const void* A, int32_t lda, const void* B, int32_t ldb,
                             int32_t beta, const void* C, int32_t ldc, void* D, int32_t ldd) {
  // configs past the vector-unit tiles: the slice product with 16 slices (3) or 15 (4)
  const int oz_slices = config == dd_gemm_configs() ? 16 : config == dd_gemm_configs() + 1 ? 15 : 0;
  if (!ctx || M < 0 || N < 0 || K < 0 || opA < 0 || opA > 1 || opB < 0 || opB > 1 || (beta != 0 && beta != 1) ||
      (negate != 0 && negate != 1) || config < 0 || config > dd_gemm_configs() + 1 ||
      (oz_slices && K > oz_max_depth(oz_slices))) {
    set_error("bad arguments to hsc_kern_zgemm_dd");
    return HSC_E_ARG;
  }
  const int a_cols = opA == OP_N ? K : M, b_cols = opB == OP_N ? N : K;
  if ((K > 0 && M > 0 && (!A || lda < a_cols)) || (K > 0 && N > 0 && (!B || ldb < b_cols)) || !D ||
      ldd < N || (beta && (!C || ldc < N))) {
    set_error("bad pointer or leading dimension in hsc_kern_zgemm_dd");
    return HSC_E_ARG;
  }
  if (M == 0 || N == 0) return HSC_OK;
  HIPCHK(hipSetDevice(ctx->device));
  if (oz_slices)
    return kern_zgemm_oz(ctx, oz_slices, opA, opB, M, N, K, negate, A, lda, B, ldb, beta, C, ldc, D, ldd);
  GemmProbDD p{};
  p.A = (const zdd*)A; p.B = (const zdd*)B; p.C = (const zdd*)C; p.D = (zdd*)D; p.D64 = nullptr;
  p.M = M; p.N = N; p.K = K; p.lda = lda; p.ldb = ldb; p.ldc = ldc; p.ldd = ldd; p.ldd64 = 0;
  const int tm = dd_gemm_tile_m(config), tn = dd_gemm_tile_n(config);
  p.tiles_n = (N + tn - 1) / tn;
  p.tile_off = 0;
  const int tiles = ((M + tm - 1) / tm) * p.tiles_n;
  std::vector<int32_t> map(tiles, 0);
  char* dev = nullptr;
  const size_t bytes = 256 + sizeof(int32_t) * tiles;
  if (hipMalloc(&dev, bytes) != hipSuccess) { (void)hipGetLastError(); set_error("alloc failed"); return HSC_E_OOM; }
  hipError_t e1 = hipMemcpy(dev, &p, sizeof(p), hipMemcpyHostToDevice);
  hipError_t e2 = hipMemcpy(dev + 256, map.data(), sizeof(int32_t) * tiles, hipMemcpyHostToDevice);
  if (e1 == hipSuccess && e2 == hipSuccess) {
    launch_dd_gemm(ctx->stream, opA, opB, config, (const GemmProbDD*)dev, (const int32_t*)(dev + 256), tiles, negate,
                   beta);
    e1 = hipGetLastError();
    if (e1 == hipSuccess) e1 = ctx->stream ? hipStreamSynchronize(ctx->stream) : hipDeviceSynchronize();
  }
  (void)hipFree(dev);
  if (e1 != hipSuccess || e2 != hipSuccess) {
    set_error(std::string("HIP error in hsc_kern_zgemm_dd: ") + hipGetErrorString(e1 != hipSuccess ? e1 : e2));
    return HSC_E_HIP;
  }
  return HSC_OK;
}

hsc_status hsc_kern_zgemm_dd_noalloc(hsc_ctx* ctx, int32_t opA, int32_t opB, int32_t M, int32_t N, int32_t K,
                                     int32_t negate, const void* A, int32_t lda, const void* B, int32_t ldb,
                                     int32_t beta, const void* C, int32_t ldc, void* D, int32_t ldd) {
  if (!ctx || M < 0 || N < 0 || K < 0 || opA < 0 || opA > 1 || opB < 0 || opB > 1 || (beta != 0 && beta != 1) ||
      (negate != 0 && negate != 1) || K > oz_max_depth(kOzSlices)) {
    set_error("bad arguments to hsc_kern_zgemm_dd_noalloc");
    return HSC_E_ARG;
  }
  const int a_cols = opA == OP_N ? K : M, b_cols = opB == OP_N ? N : K;
  if ((K > 0 && M > 0 && (!A || lda < a_cols)) || (K > 0 && N > 0 && (!B || ldb < b_cols)) || !D ||
      ldd < N || (beta && (!C || ldc < N))) {
    set_error("bad pointer or leading dimension in hsc_kern_zgemm_dd_noalloc");
    return HSC_E_ARG;
  }
  if (M == 0 || N == 0) return HSC_OK;
  const size_t need = oz_noalloc_bytes(M, N, K);
  if (need > kOzNoAllocScratch) {
    set_error("hsc_kern_zgemm_dd_noalloc: the product needs " + std::to_string(need) + " bytes of scratch, more than the " +
              std::to_string(kOzNoAllocScratch) + " of the static device array");
    return HSC_E_ARG;
  }
  if (!ctx->noalloc) {
    set_error("hsc_kern_zgemm_dd_noalloc: the scratch array's device address is unknown");
    return HSC_E_HIP;
  }
  HIPCHK(hipSetDevice(ctx->device));
  if (launch_oz_gemm_noalloc(ctx->stream, ctx->noalloc, opA, opB, M, N, K, negate, A, lda, B, ldb, beta, C, ldc, D,
                             ldd) != 0) {
    set_error("launch failed in hsc_kern_zgemm_dd_noalloc");
    return HSC_E_HIP;
  }
  return HSC_OK;
}

hsc_status hsc_kern_zinv_dd(hsc_ctx* ctx, int32_t n, void* X, int32_t ld, void* Y, int32_t ldy, int32_t* status,
                            int32_t matrix_cores) {
  if (!ctx || n < 1 || n > kMaxCluster || !X || !Y || ld < n || ldy < n || (matrix_cores != 0 && matrix_cores != 1)) {
    set_error("bad arguments to hsc_kern_zinv_dd");
    return HSC_E_ARG;
  }
  HIPCHK(hipSetDevice(ctx->device));
  // the solver's own inverse steps (Builder::dd_inverse) for one block
  const size_t W = std::max<size_t>(dd_inv_nb(n), kDDSuper);
  size_t ws = 0;
  auto wa = [&](size_t b) { size_t o = (ws + 255) / 256 * 256; ws = o + b; return o; };
  const size_t o_piv = wa(sizeof(int32_t) * n), o_t = wa(32 * W * n), o_r = wa(32 * W * n);
  const size_t o_st = wa(sizeof(int32_t));
  const size_t o_y64 = wa(16ull * n * n);   // the unscramble step always writes the rounded inverse too
  Plan pl;
  if (hipMalloc(&pl.ws, ws) != hipSuccess) {
    (void)hipGetLastError();
    pl.ws = nullptr;
    set_error("alloc failed");
    return HSC_E_OOM;
  }
  pl.B = 1;
  pl.status = reinterpret_cast<int32_t*>(pl.ws + o_st);
  Builder b{nullptr, 1, 0, false};
  b.oz = matrix_cores != 0;
  b.wsbase = pl.ws;
  b.blob.alloc(64);
  InvJobDD j{};
  j.X = (zdd*)X; j.ld = ld; j.Y = (zdd*)Y; j.ldy = ldy; j.Y64 = (double2*)(pl.ws + o_y64); j.ldy64 = n; j.n = n;
  j.e = 0;
  j.piv = (int32_t*)(pl.ws + o_piv); j.T = (zdd*)(pl.ws + o_t); j.R = (zdd*)(pl.ws + o_r);
  b.dd_inverse(std::vector<InvJobDD>{j}, n);
  hsc_status rc = upload_plan(b, &pl);
  if (rc != HSC_OK) return rc;
  HIPCHK(hipMemsetAsync(pl.status, 0, sizeof(int32_t), ctx->stream));
  rc = (hsc_status)run_steps(ctx, ctx->stream, &pl, 0, 1, nullptr, nullptr, nullptr, nullptr, 0);
  if (rc != HSC_OK) return rc;
  HIPCHK(ctx->stream ? hipStreamSynchronize(ctx->stream) : hipDeviceSynchronize());
  if (status) HIPCHK(hipMemcpy(status, pl.status, sizeof(int32_t), hipMemcpyDeviceToDevice));
  return HSC_OK;
}

hsc_status hsc_kern_mfma_rate(hsc_ctx* ctx, double* tflops) {
  if (!ctx || !tflops) { set_error("bad arguments to hsc_kern_mfma_rate"); return HSC_E_ARG; }
  HIPCHK(hipSetDevice(ctx->device));
  const int blocks = 4096, iters = 2048;
  double* out = nullptr;
  if (hipMalloc(&out, sizeof(double) * blocks * 256) != hipSuccess) {
    (void)hipGetLastError();
    set_error("alloc failed");
    return HSC_E_OOM;
  }
  hipEvent_t a = nullptr, b = nullptr;
  hipError_t e = hipEventCreate(&a);
  if (e == hipSuccess) e = hipEventCreate(&b);
  float best = 0.f;
  for (int rep = 0; rep < 3 && e == hipSuccess; ++rep) {
    e = hipEventRecord(a, ctx->stream);
    if (e != hipSuccess) break;
    launch_mfma_rate(ctx->stream, out, blocks, iters);
    e = hipEventRecord(b, ctx->stream);
    if (e == hipSuccess) e = hipEventSynchronize(b);
    float ms = 0.f;
    if (e == hipSuccess) e = hipEventElapsedTime(&ms, a, b);
    if (e == hipSuccess && (rep == 0 || ms < best)) best = ms;
  }
  if (a) (void)hipEventDestroy(a);
  if (b) (void)hipEventDestroy(b);
  (void)hipFree(out);
  if (e != hipSuccess || !(best > 0.f)) {
    set_error(std::string("HIP error in hsc_kern_mfma_rate: ") + hipGetErrorString(e));
    return HSC_E_HIP;
  }
  const double flops = (double)blocks * 4 * iters * 8 * 2048.0;   // 4 waves, 8 MFMAs of 16x16x4x2 flops
  *tflops = flops / (best * 1e-3) / 1e12;
  return HSC_OK;
}

hsc_status hsc_kern_zinv_batched(hsc_ctx* ctx, int32_t count, const int32_t* n, void* const* X,
                                 const int32_t* ld, void* const* Y, const int32_t* ldy, int32_t* status) {
  if (!ctx || count < 0 || (count > 0 && (!n || !X || !ld || !Y || !ldy))) {
    set_error("bad arguments to hsc_kern_zinv_batched");
    return HSC_E_ARG;
  }
  int maxn = 0;
  for (int k = 0; k < count; ++k) {
    if (n[k] < 1 || n[k] > 4096 || ld[k] < n[k] || ldy[k] < n[k] || !X[k] || !Y[k]) {
      set_error("bad matrix in hsc_kern_zinv_batched");
      return HSC_E_ARG;
    }
    maxn = std::max(maxn, n[k]);
  }
  if (count == 0) return HSC_OK;
  HIPCHK(hipSetDevice(ctx->device));
  const int nb = maxn <= 1024 ? 16 : maxn <= 2048 ? 8 : 4;
  size_t ws = 0;
  std::vector<size_t> o_piv(count), o_t(count), o_r(count);
  auto wa = [&](size_t b) { size_t o = (ws + 255) / 256 * 256; ws = o + b; return o; };
  for (int k = 0; k < count; ++k) {
    o_piv[k] = wa(sizeof(int32_t) * n[k]);
    o_t[k] = wa(16ull * n[k] * nb);
    o_r[k] = wa(16ull * n[k] * nb);
  }
  const size_t o_jobs = wa(sizeof(InvJob) * count);
  const size_t o_st = wa(sizeof(int32_t) * count);
  char* dev = nullptr;
  if (hipMalloc(&dev, ws) != hipSuccess) { (void)hipGetLastError(); set_error("alloc failed"); return HSC_E_OOM; }
  std::vector<InvJob> jobs(count);
  for (int k = 0; k < count; ++k) {
    InvJob& j = jobs[k];
    j.X = (double2*)X[k]; j.Y = (double2*)Y[k]; j.n = n[k]; j.ld = ld[k]; j.ldy = ldy[k]; j.e = k;
    j.piv = (int32_t*)(dev + o_piv[k]); j.T = (double2*)(dev + o_t[k]); j.R = (double2*)(dev + o_r[k]);
  }
  std::vector<int32_t> zero(count, 0);
  hipError_t err = hipMemcpy(dev + o_jobs, jobs.data(), sizeof(InvJob) * count, hipMemcpyHostToDevice);
  if (err == hipSuccess) err = hipMemcpy(dev + o_st, zero.data(), sizeof(int32_t) * count, hipMemcpyHostToDevice);
  std::vector<char*> gbufs;
  if (err == hipSuccess) {
    const InvJob* dj = (const InvJob*)(dev + o_jobs);
    int32_t* dst = (int32_t*)(dev + o_st);
    for (int k0 = 0; k0 < maxn && err == hipSuccess; k0 += nb) {
      launch_inv_panel(ctx->stream, dj, count, k0, nb, maxn, dst);
      launch_inv_swap(ctx->stream, dj, count, k0, nb, maxn);
      std::vector<GemmProb> probs;
      std::vector<int32_t> tmap;
      for (int k = 0; k < count; ++k) {
        if (k0 >= n[k]) continue;
        const int kb = std::min(nb, n[k] - k0);
        GemmProb p{};
        p.A = jobs[k].T; p.B = jobs[k].R; p.C = jobs[k].X; p.D = jobs[k].X;
        p.M = n[k]; p.N = n[k]; p.K = kb; p.lda = kb; p.ldb = n[k]; p.ldc = ld[k]; p.ldd = ld[k];
        p.tiles_n = (n[k] + 63) / 64;
        p.tile_off = (int32_t)tmap.size();
        const int tiles = ((n[k] + 63) / 64) * p.tiles_n;
        for (int q = 0; q < tiles; ++q) tmap.push_back((int32_t)probs.size());
        probs.push_back(p);
      }
      char* gb = nullptr;
      const size_t gbytes = sizeof(GemmProb) * probs.size() + 256 + sizeof(int32_t) * tmap.size();
      err = hipMalloc(&gb, gbytes);
      if (err != hipSuccess) break;
      gbufs.push_back(gb);
      const size_t o_map = (sizeof(GemmProb) * probs.size() + 255) / 256 * 256;
      err = hipMemcpy(gb, probs.data(), sizeof(GemmProb) * probs.size(), hipMemcpyHostToDevice);
      if (err == hipSuccess) err = hipMemcpy(gb + o_map, tmap.data(), sizeof(int32_t) * tmap.size(), hipMemcpyHostToDevice);
      if (err == hipSuccess)
        launch_gemm(ctx->stream, OP_N, OP_N, (const GemmProb*)gb, (const int32_t*)(gb + o_map), (int)tmap.size(),
                    1.0, 0.0, 1, 0);
    }
    if (err == hipSuccess) launch_inv_unscramble(ctx->stream, dj, count, maxn);
    if (err == hipSuccess) err = hipGetLastError();
    if (err == hipSuccess) err = ctx->stream ? hipStreamSynchronize(ctx->stream) : hipDeviceSynchronize();
    if (err == hipSuccess && status)
      err = hipMemcpy(status, dev + o_st, sizeof(int32_t) * count, hipMemcpyDeviceToDevice);
  }
  for (char* g : gbufs) (void)hipFree(g);
  (void)hipFree(dev);
  if (err != hipSuccess) {
    set_error(std::string("HIP error in hsc_kern_zinv_batched: ") + hipGetErrorString(err));
    return HSC_E_HIP;
  }
  return HSC_OK;
}

hsc_status hsc_kern_mfma_probe(hsc_ctx* ctx, double* out) {
  if (!ctx || !out) { set_error("null argument"); return HSC_E_ARG; }
  HIPCHK(hipSetDevice(ctx->device));
  launch_mfma_probe(ctx->stream, out);
  HIPCHK(hipGetLastError());
  HIPCHK(ctx->stream ? hipStreamSynchronize(ctx->stream) : hipDeviceSynchronize());
  return HSC_OK;
}

}  // extern "C"
