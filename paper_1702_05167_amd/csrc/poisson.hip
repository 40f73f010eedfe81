// The electrostatic half of the self-consistent NEGF-Poisson loop (the setting the method serves,
// abstract and Section 1): electron density from the diagonal of G^< (Eq. 2), a 7-point Poisson
// solve on the device grid, source and mixing.
//
// Poisson: sum over the three axes of (2 U_i - U_prev - U_next) = rho_i on an Nx x Ny x Nz grid
// (site (x, y, z) at x + Nx (y + Ny z)); outside neighbours along x are the lead planes x = -1 and
// x = Nx with fixed values (Dirichlet), along y and z the site itself (zero normal derivative).
// The operator is a sum of three commuting 1D operators, each diagonalised by a closed-form
// orthonormal basis:
//   x (Dirichlet): Q[j][k] = sqrt(2 / (Nx + 1)) sin(pi (k + 1)(j + 1) / (Nx + 1)),
//                  lambda_k = 2 - 2 cos(pi (k + 1) / (Nx + 1));
//   y, z (Neumann): Q[j][k] = c_k cos(pi k (j + 1/2) / N), c_0 = sqrt(1 / N), c_k = sqrt(2 / N),
//                  lambda_k = 2 - 2 cos(pi k / N).
// U = (Qx Qy Qz) diag(1 / (lx + ly + lz)) (Qx Qy Qz)^T (rho + lead-plane terms): three forward
// axis transforms, a scale, three backward ones.  Every sum along an axis is a plain FP64 loop of
// length N (the grids are at most a few hundred per side; the transforms are bandwidth-bound and a
// negligible part of a self-consistent iteration next to the NEGF solve).
#include <hip/hip_runtime.h>

#include <cmath>
#include <string>
#include <vector>

#include "hsc_internal.h"
#include "kern.h"
#include "poisson_basis.h"

namespace hsc {

namespace {

constexpr int PB = 256;
constexpr double kPi = 3.14159265358979323846;

// out[i] = sum_j M(kk, j) in[base + j stride] with kk the coordinate of i along the axis (len,
// stride) and base = i - kk stride; M(kk, j) = Q[kk][j] when backward, Q[j][kk] when forward
__global__ __launch_bounds__(PB) void k_axis(int64_t n, int len, int64_t stride, const double* __restrict__ Q,
                                             int forward, const double* __restrict__ in, double* __restrict__ out) {
  const int64_t i = (int64_t)blockIdx.x * PB + threadIdx.x;
  if (i >= n) return;
  const int kk = (int)((i / stride) % len);
  const int64_t base = i - (int64_t)kk * stride;
  double s = 0.0;
  if (forward) {
    for (int j = 0; j < len; ++j) s = fma(Q[(int64_t)j * len + kk], in[base + j * stride], s);
  } else {
    for (int j = 0; j < len; ++j) s = fma(Q[(int64_t)kk * len + j], in[base + j * stride], s);
  }
  out[i] = s;
}

// c[i] /= lx[x] + ly[y] + lz[z]
__global__ __launch_bounds__(PB) void k_pscale(int64_t n, int nx, int ny, const double* __restrict__ lx,
                                               const double* __restrict__ ly, const double* __restrict__ lz,
                                               double* __restrict__ c) {
  const int64_t i = (int64_t)blockIdx.x * PB + threadIdx.x;
  if (i >= n) return;
  const int x = (int)(i % nx), y = (int)((i / nx) % ny);
  const int64_t z = i / ((int64_t)nx * ny);
  c[i] = c[i] / ((lx[x] + ly[y]) + lz[z]);
}

// out = coupling (dens - n0) (n0 may be null) when dens is given, else rho; plus the lead planes
__global__ __launch_bounds__(PB) void k_psource(int64_t n, int nx, const double* __restrict__ rho,
                                                const double* __restrict__ dens, const double* __restrict__ n0,
                                                double coupling, double u_left, double u_right,
                                                double* __restrict__ out) {
  const int64_t i = (int64_t)blockIdx.x * PB + threadIdx.x;
  if (i >= n) return;
  double v = dens ? coupling * (dens[i] - (n0 ? n0[i] : 0.0)) : rho[i];
  const int x = (int)(i % nx);
  if (x == 0) v += u_left;
  if (x == nx - 1) v += u_right;
  out[i] = v;
}

// dens[i] = sum_e w[e] Im G^<_ii(E_e) / (2 pi), energies in order
__global__ __launch_bounds__(PB) void k_density(int ne, int64_t n, const double* __restrict__ w,
                                                const double2* __restrict__ gl, double* __restrict__ dens) {
  const int64_t i = (int64_t)blockIdx.x * PB + threadIdx.x;
  if (i >= n) return;
  double s = 0.0;
  for (int e = 0; e < ne; ++e) s = fma(w[e], gl[(int64_t)e * n + i].y, s);
  dens[i] = s / (2.0 * kPi);
}

// r = max_i |u_new - u| (as the ordered bits of a non-negative double), then u += beta (u_new - u)
__global__ __launch_bounds__(PB) void k_mix(int64_t n, double* __restrict__ u, const double* __restrict__ u_new,
                                            double beta, unsigned long long* __restrict__ r) {
  const int64_t i = (int64_t)blockIdx.x * PB + threadIdx.x;
  double d = 0.0;
  if (i < n) {
    d = u_new[i] - u[i];
    u[i] = u[i] + beta * d;
  }
  double m = fabs(d);
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) m = fmax(m, __shfl_xor(m, off, 64));
  if ((threadIdx.x & 63) == 0) atomicMax(r, (unsigned long long)__double_as_longlong(m));
}

// f = u_new - u and *r = max_i |f_i| (ordered bits), u unchanged
__global__ __launch_bounds__(PB) void k_scf_resid(int64_t n, const double* __restrict__ u,
                                                  const double* __restrict__ u_new, double* __restrict__ f,
                                                  unsigned long long* __restrict__ r) {
  const int64_t i = (int64_t)blockIdx.x * PB + threadIdx.x;
  double d = 0.0;
  if (i < n) {
    d = u_new[i] - u[i];
    f[i] = d;
  }
  double m = fabs(d);
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) m = fmax(m, __shfl_xor(m, off, 64));
  if ((threadIdx.x & 63) == 0) atomicMax(r, (unsigned long long)__double_as_longlong(m));
}

// Anderson history: dX = u - u_prev, dF = f - f_prev (when given), then u_prev = u, f_prev = f
__global__ __launch_bounds__(PB) void k_scf_hist(int64_t n, const double* __restrict__ u, const double* __restrict__ f,
                                                 double* __restrict__ u_prev, double* __restrict__ f_prev,
                                                 double* __restrict__ dX, double* __restrict__ dF) {
  const int64_t i = (int64_t)blockIdx.x * PB + threadIdx.x;
  if (i >= n) return;
  if (dX) {
    dX[i] = u[i] - u_prev[i];
    dF[i] = f[i] - f_prev[i];
  }
  u_prev[i] = u[i];
  f_prev[i] = f[i];
}

// u = u + beta f - sum_j gamma_j (dX_j + beta dF_j), history slots in `order`
__global__ __launch_bounds__(PB) void k_scf_update(int64_t n, double* __restrict__ u, const double* __restrict__ f,
                                                   double beta, int mk, const double* __restrict__ dX,
                                                   const double* __restrict__ dF, const int32_t* __restrict__ order,
                                                   const double* __restrict__ gamma) {
  const int64_t i = (int64_t)blockIdx.x * PB + threadIdx.x;
  if (i >= n) return;
  double x = u[i] + beta * f[i];
  for (int j = 0; j < mk; ++j) {
    const int64_t o = (int64_t)order[j] * n + i;
    x -= gamma[j] * (dX[o] + beta * dF[o]);
  }
  u[i] = x;
}

__global__ void k_zero_u64(unsigned long long* p) {
  if (threadIdx.x == 0 && blockIdx.x == 0) *p = 0ull;
}

// pot[p] = U[perm[p]] (site order -> cluster order), or 0 without U
__global__ __launch_bounds__(PB) void k_potential(int64_t n, const int64_t* __restrict__ perm,
                                                  const double* __restrict__ U, double* __restrict__ pot) {
  const int64_t p = (int64_t)blockIdx.x * PB + threadIdx.x;
  if (p >= n) return;
  pot[p] = U ? U[perm[p]] : 0.0;
}

unsigned blocks(int64_t n) { return (unsigned)((n + PB - 1) / PB); }

}  // namespace

void launch_potential(hipStream_t st, int64_t n, const int64_t* perm, const double* U, double* pot) {
  if (n > 0) hipLaunchKernelGGL(k_potential, dim3(blocks(n)), dim3(PB), 0, st, n, perm, U, pot);
}

void launch_density(hipStream_t st, int ne, int64_t n, const double* w, const void* gl, double* dens) {
  if (n > 0) hipLaunchKernelGGL(k_density, dim3(blocks(n)), dim3(PB), 0, st, ne, n, w, (const double2*)gl, dens);
}

void launch_mix(hipStream_t st, int64_t n, double* u, const double* u_new, double beta, unsigned long long* r) {
  hipLaunchKernelGGL(k_zero_u64, dim3(1), dim3(64), 0, st, r);
  if (n > 0) hipLaunchKernelGGL(k_mix, dim3(blocks(n)), dim3(PB), 0, st, n, u, u_new, beta, r);
}

void launch_scf_resid(hipStream_t st, int64_t n, const double* u, const double* u_new, double* f,
                      unsigned long long* r) {
  hipLaunchKernelGGL(k_zero_u64, dim3(1), dim3(64), 0, st, r);
  if (n > 0) hipLaunchKernelGGL(k_scf_resid, dim3(blocks(n)), dim3(PB), 0, st, n, u, u_new, f, r);
}

void launch_scf_hist(hipStream_t st, int64_t n, const double* u, const double* f, double* u_prev, double* f_prev,
                     double* dX, double* dF) {
  if (n > 0) hipLaunchKernelGGL(k_scf_hist, dim3(blocks(n)), dim3(PB), 0, st, n, u, f, u_prev, f_prev, dX, dF);
}

void launch_scf_update(hipStream_t st, int64_t n, double* u, const double* f, double beta, int mk, const double* dX,
                       const double* dF, const int32_t* order, const double* gamma) {
  if (n > 0)
    hipLaunchKernelGGL(k_scf_update, dim3(blocks(n)), dim3(PB), 0, st, n, u, f, beta, mk, dX, dF, order, gamma);
}

int poisson_check(const hsc_grid* g, std::string* why) {
  if (!g || g->nx < 1 || g->ny < 1 || g->nz < 1 || g->nx > kPoissonMaxSide || g->ny > kPoissonMaxSide ||
      g->nz > kPoissonMaxSide) {
    *why = "grid sides must lie in [1, " + std::to_string(kPoissonMaxSide) + "]";
    return -1;
  }
  if (!std::isfinite(g->u_left) || !std::isfinite(g->u_right)) {
    *why = "lead-plane potentials must be finite";
    return -1;
  }
  return 0;
}

int PoissonWork::create(const hsc_grid& g) {
  grid = g;
  n = (int64_t)g.nx * g.ny * g.nz;
  const int side[3] = {g.nx, g.ny, g.nz};
  size_t doubles = 2 * (size_t)n;
  for (int a = 0; a < 3; ++a) doubles += (size_t)side[a] * side[a] + side[a];
  if (hipMalloc(&buf, doubles * sizeof(double)) != hipSuccess) {
    (void)hipGetLastError();
    buf = nullptr;
    return -1;
  }
  std::vector<double> host(doubles - 2 * (size_t)n);
  double* p = buf + 2 * (size_t)n;
  double* h = host.data();
  t1 = buf;
  t2 = buf + n;
  for (int a = 0; a < 3; ++a) {
    // x: Dirichlet (the lead planes); y, z: zero normal derivative
    const int N = side[a];
    poisson_basis(N, a == 0, h, h + (size_t)N * N);
    Q[a] = p;
    lam[a] = p + (size_t)N * N;
    p += (size_t)N * N + N;
    h += (size_t)N * N + N;
  }
  if (hipMemcpy(buf + 2 * (size_t)n, host.data(), host.size() * sizeof(double), hipMemcpyHostToDevice) != hipSuccess) {
    (void)hipGetLastError();
    return -1;
  }
  return 0;
}

void PoissonWork::destroy() {
  if (buf) (void)hipFree(buf);
  buf = nullptr;
}

void PoissonWork::run(hipStream_t st, const double* rho, const double* dens, const double* n0, double coupling,
                      double* u) const {
  const unsigned nb = blocks(n);
  const int side[3] = {grid.nx, grid.ny, grid.nz};
  const int64_t stride[3] = {1, grid.nx, (int64_t)grid.nx * grid.ny};
  hipLaunchKernelGGL(k_psource, dim3(nb), dim3(PB), 0, st, n, grid.nx, rho, dens, n0, coupling, grid.u_left,
                     grid.u_right, t1);
  // forward transforms x, y, z (t1 -> t2 -> t1 -> t2), scale, backward z, y, x (t2 -> t1 -> t2 -> u)
  double* a = t1;
  double* b = t2;
  for (int ax = 0; ax < 3; ++ax) {
    hipLaunchKernelGGL(k_axis, dim3(nb), dim3(PB), 0, st, n, side[ax], stride[ax], Q[ax], 1, a, b);
    std::swap(a, b);
  }
  hipLaunchKernelGGL(k_pscale, dim3(nb), dim3(PB), 0, st, n, grid.nx, grid.ny, lam[0], lam[1], lam[2], a);
  for (int ax = 2; ax >= 0; --ax) {
    double* dst = ax == 0 ? u : b;
    hipLaunchKernelGGL(k_axis, dim3(nb), dim3(PB), 0, st, n, side[ax], stride[ax], Q[ax], 0, a, dst);
    std::swap(a, b);
  }
}

}  // namespace hsc

using namespace hsc;

extern "C" {

hsc_status hsc_poisson_solve(hsc_ctx* ctx, const hsc_grid* grid, const double* rho, double* u) {
  std::string why;
  if (!ctx || poisson_check(grid, &why) != 0 || !rho || !u) {
    set_error(why.empty() ? std::string("bad arguments to hsc_poisson_solve") : "hsc_poisson_solve: " + why);
    return HSC_E_ARG;
  }
  if (hipSetDevice(ctx_device(ctx)) != hipSuccess) {
    (void)hipGetLastError();
    set_error("hsc_poisson_solve: cannot select the device");
    return HSC_E_HIP;
  }
  PoissonWork w;
  if (w.create(*grid) != 0) {
    set_error("hsc_poisson_solve: workspace allocation failed");
    return HSC_E_OOM;
  }
  hipStream_t st = reinterpret_cast<hipStream_t>(ctx_stream(ctx));
  w.run(st, rho, nullptr, nullptr, 0.0, u);
  hipError_t e = hipGetLastError();
  if (e == hipSuccess) e = st ? hipStreamSynchronize(st) : hipDeviceSynchronize();
  w.destroy();
  if (e != hipSuccess) {
    set_error(std::string("HIP error in hsc_poisson_solve: ") + hipGetErrorString(e));
    return HSC_E_HIP;
  }
  return HSC_OK;
}

hsc_status hsc_density(hsc_ctx* ctx, int32_t n_e, int64_t n, const double* weights, const void* diag_gl,
                       double* density) {
  if (!ctx || n_e < 0 || n < 0 || (n > 0 && !density) || (n > 0 && n_e > 0 && (!weights || !diag_gl))) {
    set_error("bad arguments to hsc_density");
    return HSC_E_ARG;
  }
  if (n == 0) return HSC_OK;
  if (hipSetDevice(ctx_device(ctx)) != hipSuccess) {
    (void)hipGetLastError();
    set_error("hsc_density: cannot select the device");
    return HSC_E_HIP;
  }
  launch_density(reinterpret_cast<hipStream_t>(ctx_stream(ctx)), n_e, n, weights, diag_gl, density);
  const hipError_t e = hipGetLastError();
  if (e != hipSuccess) {
    set_error(std::string("HIP error in hsc_density: ") + hipGetErrorString(e));
    return HSC_E_HIP;
  }
  return HSC_OK;
}

}  // extern "C"
