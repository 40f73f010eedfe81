// hsc_run: a native driver of the solver's C ABI, for profilers that should see no Python
// process (hardware-counter passes).  It reads a device file, builds the tree, and solves the
// energy grid in steps of one batch, exactly as the throughput benchmark walks it.
//
//   hsc_run DEVICE_FILE [--batch B] [--steps K] [--warmup W] [--precision P] [--leaf L]
//                       [--dense 0|1] [--tune 0|1] [--slices S] [--copy-mib M]
//
// --copy-mib M first runs one elementwise copy kernel of M MiB (read M, write M), whose counter
// readings calibrate the HBM byte counters.
//
// Device file (little-endian, written by `bench.py --write-device`):
//   char[8] "HSCDEV1" ; int64 n ; int64 nnz ; int64 indptr[n+1] ; int32 indices[nnz] ;
//   double values[2 nnz] (re, im) ; int32 coords[3 n] ;
//   two contacts: int64 count ; int64 sites[count] ; double lead_onsite, lead_hopping, coupling ;
//   int64 n_e ; double energies[n_e]
#include <hip/hip_runtime.h>

#include <chrono>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <string>
#include <vector>

#include "../../include/hsc.h"

namespace {

__global__ void k_copy(const double* __restrict__ src, double* __restrict__ dst, size_t n) {
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x)
    dst[i] = src[i];
}

template <class T>
bool rd(FILE* f, T* p, size_t count) {
  return count == 0 || fread(p, sizeof(T), count, f) == count;
}

int fail(const char* what) {
  fprintf(stderr, "hsc_run: %s (%s)\n", what, hsc_last_error());
  return 1;
}

}  // namespace

int main(int argc, char** argv) {
  if (argc < 2) {
    fprintf(stderr, "usage: hsc_run DEVICE_FILE [--batch B] [--steps K] [--warmup W] [--precision P] "
                    "[--leaf L] [--dense 0|1] [--tune 0|1] [--slices S] [--copy-mib M]\n");
    return 2;
  }
  int batch = 16, steps = 1, warmup = 1, precision = 3, leaf = 8, dense = 0, tune = 1, slices = 0, copy_mib = 0;
  for (int a = 2; a + 1 < argc; a += 2) {
    const std::string k = argv[a];
    const int v = atoi(argv[a + 1]);
    if (k == "--batch") batch = v;
    else if (k == "--steps") steps = v;
    else if (k == "--warmup") warmup = v;
    else if (k == "--precision") precision = v;
    else if (k == "--leaf") leaf = v;
    else if (k == "--dense") dense = v;
    else if (k == "--tune") tune = v;
    else if (k == "--slices") slices = v;
    else if (k == "--copy-mib") copy_mib = v;
    else { fprintf(stderr, "hsc_run: unknown option %s\n", k.c_str()); return 2; }
  }
  FILE* f = fopen(argv[1], "rb");
  if (!f) { perror("hsc_run: device file"); return 1; }
  char magic[8];
  int64_t n = 0, nnz = 0;
  if (!rd(f, magic, 8) || std::memcmp(magic, "HSCDEV1", 8) != 0 || !rd(f, &n, 1) || !rd(f, &nnz, 1) || n <= 0 ||
      nnz < 0) {
    fprintf(stderr, "hsc_run: not a device file\n");
    return 1;
  }
  std::vector<int64_t> indptr(n + 1);
  std::vector<int32_t> indices(nnz), coords(3 * n);
  std::vector<double> values(2 * nnz);
  bool ok = rd(f, indptr.data(), indptr.size()) && rd(f, indices.data(), indices.size()) &&
            rd(f, values.data(), values.size()) && rd(f, coords.data(), coords.size());
  std::vector<int64_t> sites[2];
  hsc_contact contacts[2];
  for (int c = 0; c < 2 && ok; ++c) {
    int64_t cnt = 0;
    ok = rd(f, &cnt, 1) && cnt > 0 && cnt <= n;
    if (!ok) break;
    sites[c].resize(cnt);
    double p[3];
    ok = rd(f, sites[c].data(), cnt) && rd(f, p, 3);
    contacts[c] = hsc_contact{cnt, sites[c].data(), p[0], p[1], p[2]};
  }
  int64_t ne = 0;
  ok = ok && rd(f, &ne, 1) && ne > 0 && ne < (1 << 24);
  std::vector<double> energies(ok ? ne : 0);
  ok = ok && rd(f, energies.data(), energies.size());
  fclose(f);
  if (!ok) { fprintf(stderr, "hsc_run: truncated device file\n"); return 1; }
  if (batch < 1 || batch > ne || steps < 0 || warmup < 0) { fprintf(stderr, "hsc_run: bad batch / steps\n"); return 2; }

  if (copy_mib > 0) {
    const size_t cnt = (size_t)copy_mib * 131072;
    double *src = nullptr, *dst = nullptr;
    if (hipMalloc(&src, cnt * 8) != hipSuccess || hipMalloc(&dst, cnt * 8) != hipSuccess) return fail("copy buffers");
    if (hipMemset(src, 0, cnt * 8) != hipSuccess) return fail("copy memset");
    hipLaunchKernelGGL(k_copy, dim3(4096), dim3(256), 0, nullptr, src, dst, cnt);
    if (hipDeviceSynchronize() != hipSuccess) return fail("copy kernel");
    (void)hipFree(src);
    (void)hipFree(dst);
    printf("copy of %d MiB done\n", copy_mib);
    fflush(stdout);
  }

  hsc_tree_opts topts{coords.data(), 7, leaf, 0, dense};
  hsc_tree* tree = nullptr;
  if (hsc_tree_build(n, indptr.data(), indices.data(), values.data(), 2, contacts, &topts, &tree) != HSC_OK)
    return fail("tree build");
  hsc_ctx* ctx = nullptr;
  if (hsc_ctx_create(0, nullptr, &ctx) != HSC_OK) return fail("context");
  double* d_e = nullptr;
  double* d_tr = nullptr;
  void *d_gr = nullptr, *d_gl = nullptr;
  int32_t* d_st = nullptr;
  if (hipMalloc(&d_e, 8 * ne) != hipSuccess || hipMalloc(&d_gr, 16 * (size_t)batch * n) != hipSuccess ||
      hipMalloc(&d_gl, 16 * (size_t)batch * n) != hipSuccess || hipMalloc(&d_tr, 8 * batch) != hipSuccess ||
      hipMalloc(&d_st, 4 * batch) != hipSuccess)
    return fail("output buffers");
  if (hipMemcpy(d_e, energies.data(), 8 * ne, hipMemcpyHostToDevice) != hipSuccess) return fail("energies");
  hsc_solve_opts o{};
  o.eta = 1e-8; o.kT = 0.025; o.mu_L = 0.1; o.mu_R = -0.1;
  o.want = HSC_DIAG_GR | HSC_DIAG_GL | HSC_TRANS;
  o.batch = batch; o.precision = precision; o.tune = tune; o.complex3m = 1; o.slices = slices;
  // step k solves the next `batch` grid points (wrapping around), as the benchmark does
  std::vector<double> e_step(batch);
  double* d_step = nullptr;
  if (hipMalloc(&d_step, 8 * batch) != hipSuccess) return fail("step energies");
  auto step = [&](int k) -> bool {
    for (int j = 0; j < batch; ++j) e_step[j] = energies[((int64_t)k * batch + j) % ne];
    if (hipMemcpy(d_step, e_step.data(), 8 * batch, hipMemcpyHostToDevice) != hipSuccess) return false;
    return hsc_solve(ctx, tree, batch, d_step, &o, d_gr, d_gl, d_tr, nullptr, d_st, nullptr) == HSC_OK &&
           hsc_sync(ctx) == HSC_OK;
  };
  if (!step(0)) return fail("set-up step");
  printf("set-up done\n");
  fflush(stdout);
  for (int k = 0; k < warmup; ++k)
    if (!step(k)) return fail("warm-up step");
  const auto t0 = std::chrono::steady_clock::now();
  for (int k = 0; k < steps; ++k) {
    if (!step(k)) return fail("step");
    printf("step %d of %d done\n", k + 1, steps);
    fflush(stdout);
  }
  const double dt = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
  std::vector<int32_t> st(batch);
  if (hipMemcpy(st.data(), d_st, 4 * batch, hipMemcpyDeviceToHost) != hipSuccess) return fail("status");
  int bad = 0;
  for (int32_t s : st) bad += s != 0;
  printf("{\"sites\": %lld, \"batch\": %d, \"steps\": %d, \"seconds\": %.6f, \"energies_per_s\": %.4f, "
         "\"bad_status\": %d}\n",
         (long long)n, batch, steps, dt, steps > 0 ? steps * batch / dt : 0.0, bad);
  (void)hipFree(d_step);
  (void)hipFree(d_e);
  (void)hipFree(d_gr);
  (void)hipFree(d_gl);
  (void)hipFree(d_tr);
  (void)hipFree(d_st);
  hsc_ctx_destroy(ctx);
  hsc_tree_destroy(tree);
  return 0;
}
