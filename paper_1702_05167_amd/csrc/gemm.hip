// Grouped complex128 GEMM on CDNA4 FP64 matrix cores (v_mfma_f64_16x16x4_f64).
//
// Every Schur update, multiplier, extraction and fold product of Algorithms 1
// and 2 is a dense complex product of blocks of uneven size.  One launch
// covers all problems of one tree level (over clusters and energies): each
// workgroup owns one output tile of one problem (host-built tile -> problem
// map), so uneven sizes share the chip.
//
// Complex product on real matrix cores, interleaved (re, im) storage:
//   Re += Ar*Br + Ai*(-Bi),   Im += Ar*Bi + Ai*Br   (4 real MFMAs per block step),
// or, with the three-multiplication form (Gauss):
//   T1 += Ar*Br, T2 += Ai*Bi, T3 += (Ar+Ai)*(Br+Bi);  Re = T1 - T2, Im = T3 - T1 - T2
// (3 real MFMAs per block step; the imaginary part's error bound grows with |A||B| rather
// than with |Ar||Bi| + |Ai||Br|).
// Layout of v_mfma_f64_16x16x4_f64 (one wave, 64 lanes):
//   A 16x4: lane l holds A[l%16][l/16];  B 4x16: lane l holds B[l/16][l%16];
//   D 16x16: lane l, register r holds D[l/16 + 4*r][l%16].
// Layout of v_mfma_f64_4x4x4_f64 (four independent 4x4x4 products, blk = (l>>2)&3):
//   A_blk[l&3][l>>4], B_blk[l>>4][l&3], D_blk[l>>4][l&3].
// A 16x16x4 block step is also four of these (I = 0..3): B as above (B[l>>4][l&15]),
// A[4I + (l&3)][l>>4] (the same for the four blks), D rows 4I + (l>>4), column l&15.
// On this chip the 4x4x4 form sustains a higher FP64 rate (about 71 vs 50 TFLOP/s in an
// MFMA-only stream), at the price of four times the A operand reads.
#include <hip/hip_runtime.h>

#include "kern.h"

namespace hsc {

typedef double v4d __attribute__((ext_vector_type(4)));

namespace {

constexpr int NT = 256;   // default: 4 waves, arranged 2 x 2 over the tile

// Load the logical tile X'(r, k), r in [r0, r0+R), k in [k0, k0+KS), into
// registers.  KCONTIG: X'(r,k) = src[r*ld + k]; otherwise X'(r,k) = src[k*ld + r].
template <int R, int KS, bool KCONTIG, int NTH = NT>
struct TileLoader {
  static constexpr int PER = R * KS / NTH;   // elements per thread (multiple of 4)
  static_assert(PER % 4 == 0, "tile too small");
  double2 v[PER];

  __device__ inline void load(const double2* __restrict__ src, int ld, int r0, int k0, int Rmax,
                              int Kmax, bool conj, int t) {
    if (KCONTIG) {
      constexpr int TPR = KS / 4, RPP = NTH / TPR;
#pragma unroll
      for (int p = 0; p < PER / 4; ++p) {
        int r = r0 + p * RPP + t / TPR;
        int k = k0 + (t % TPR) * 4;
#pragma unroll
        for (int u = 0; u < 4; ++u) {
          double2 x = make_double2(0.0, 0.0);
          if (r < Rmax && k + u < Kmax) x = src[(int64_t)r * ld + k + u];
          if (conj) x.y = -x.y;
          v[p * 4 + u] = x;
        }
      }
    } else {
      constexpr int TPK = R / 4, KPP = NTH / TPK;
#pragma unroll
      for (int p = 0; p < PER / 4; ++p) {
        int k = k0 + p * KPP + t / TPK;
        int r = r0 + (t % TPK) * 4;
#pragma unroll
        for (int u = 0; u < 4; ++u) {
          double2 x = make_double2(0.0, 0.0);
          if (r + u < Rmax && k < Kmax) x = src[(int64_t)k * ld + r + u];
          if (conj) x.y = -x.y;
          v[p * 4 + u] = x;
        }
      }
    }
  }

  // store as S[k][r] (row stride RS)
  template <int RS>
  __device__ inline void store(double2* S, int t) const {
    if (KCONTIG) {
      constexpr int TPR = KS / 4, RPP = NTH / TPR;
#pragma unroll
      for (int p = 0; p < PER / 4; ++p) {
        int r = p * RPP + t / TPR;
        int k = (t % TPR) * 4;
#pragma unroll
        for (int u = 0; u < 4; ++u) S[(k + u) * RS + r] = v[p * 4 + u];
      }
    } else {
      constexpr int TPK = R / 4, KPP = NTH / TPK;
#pragma unroll
      for (int p = 0; p < PER / 4; ++p) {
        int k = p * KPP + t / TPK;
        int r = (t % TPK) * 4;
#pragma unroll
        for (int u = 0; u < 4; ++u) S[k * RS + r + u] = v[p * 4 + u];
      }
    }
  }
};

template <int BM, int BN, int BK, int OPA, int OPB, bool M3, bool MF4 = false, int WGM = 2, int WGN = 2>
__global__ __launch_bounds__(64 * WGM * WGN) void k_zgemm(const GemmProb* __restrict__ probs,
                                                         const int32_t* __restrict__ tile_prob, int total_tiles,
                                                         double alpha_re, double alpha_im, int beta) {
  constexpr int NTH = 64 * WGM * WGN;                // WGM x WGN waves over the tile
  constexpr int WTM = BM / WGM, WTN = BN / WGN;      // wave tile
  constexpr int MB = WTM / 16, NB = WTN / 16;        // 16x16 blocks per wave
  constexpr int AS = BM + 1, BS = BN + 1;            // padded LDS row strides
  constexpr bool A_KC = (OPA == OP_N);               // A'(m,k) = A[m*lda+k]
  constexpr bool B_KC = (OPB != OP_N);               // B'(k,n) = B[n*ldb+k]
  __shared__ double2 As[2][BK * AS];
  __shared__ double2 Bs[2][BK * BS];

  // XCD-aware order: consecutive logical tiles on the same XCD (round-robin dispatch over 8)
  const int per = (total_tiles + 7) >> 3;
  const int tile = (blockIdx.x & 7) * per + (blockIdx.x >> 3);
  if (tile >= total_tiles) return;
  const GemmProb& pr = probs[tile_prob[tile]];
  const int local = tile - pr.tile_off;
  const int m0 = (local / pr.tiles_n) * BM, n0 = (local % pr.tiles_n) * BN;
  const int M = pr.M, N = pr.N, K = pr.K;

  const int t = threadIdx.x, lane = t & 63, w = t >> 6;
  const int wm = w / WGN, wn = w % WGN;

  // 16x16x4 form: v4d accumulators; 4x4x4 form: the same registers as four doubles (one per I)
  v4d cr[MB][NB], ci[MB][NB], cs[M3 ? MB : 1][M3 ? NB : 1];   // cs: T3 of the 3-product form
#pragma unroll
  for (int i = 0; i < MB; ++i)
#pragma unroll
    for (int j = 0; j < NB; ++j) {
      cr[i][j] = v4d{0, 0, 0, 0};
      ci[i][j] = v4d{0, 0, 0, 0};
      if (M3) cs[i][j] = v4d{0, 0, 0, 0};
    }

  TileLoader<BM, BK, A_KC, NTH> la;
  TileLoader<BN, BK, B_KC, NTH> lb;
  const int nk = (K + BK - 1) / BK;
  if (nk > 0) {
    la.load(pr.A, pr.lda, m0, 0, M, K, OPA == OP_C, t);
    lb.load(pr.B, pr.ldb, n0, 0, N, K, OPB == OP_C, t);
    la.template store<AS>(As[0], t);
    lb.template store<BS>(Bs[0], t);
  }
  __syncthreads();
  for (int kt = 0; kt < nk; ++kt) {
    const int cur = kt & 1;
    if (kt + 1 < nk) {
      la.load(pr.A, pr.lda, m0, (kt + 1) * BK, M, K, OPA == OP_C, t);
      lb.load(pr.B, pr.ldb, n0, (kt + 1) * BK, N, K, OPB == OP_C, t);
    }
    const double2* __restrict__ as = As[cur];
    const double2* __restrict__ bs = Bs[cur];
#pragma unroll
    for (int kk = 0; kk < BK / 4; ++kk) {
      const int k = kk * 4 + (lane >> 4);
      if (MF4) {
        double2 b[NB], a4[MB][4];
#pragma unroll
        for (int j = 0; j < NB; ++j) b[j] = bs[k * BS + wn * WTN + j * 16 + (lane & 15)];
#pragma unroll
        for (int i = 0; i < MB; ++i)
#pragma unroll
          for (int I = 0; I < 4; ++I) a4[i][I] = as[k * AS + wm * WTM + i * 16 + 4 * I + (lane & 3)];
#pragma unroll
        for (int i = 0; i < MB; ++i)
#pragma unroll
          for (int j = 0; j < NB; ++j)
#pragma unroll
            for (int I = 0; I < 4; ++I) {
              const double2 x = a4[i][I], y = b[j];
              if (M3) {
                cr[i][j][I] = __builtin_amdgcn_mfma_f64_4x4x4f64(x.x, y.x, cr[i][j][I], 0, 0, 0);
                ci[i][j][I] = __builtin_amdgcn_mfma_f64_4x4x4f64(x.y, y.y, ci[i][j][I], 0, 0, 0);
                cs[i][j][I] = __builtin_amdgcn_mfma_f64_4x4x4f64(x.x + x.y, y.x + y.y, cs[i][j][I], 0, 0, 0);
              } else {
                cr[i][j][I] = __builtin_amdgcn_mfma_f64_4x4x4f64(x.x, y.x, cr[i][j][I], 0, 0, 0);
                ci[i][j][I] = __builtin_amdgcn_mfma_f64_4x4x4f64(x.x, y.y, ci[i][j][I], 0, 0, 0);
                cr[i][j][I] = __builtin_amdgcn_mfma_f64_4x4x4f64(x.y, -y.y, cr[i][j][I], 0, 0, 0);
                ci[i][j][I] = __builtin_amdgcn_mfma_f64_4x4x4f64(x.y, y.x, ci[i][j][I], 0, 0, 0);
              }
            }
        continue;
      }
      double2 a[MB], b[NB];
      double nbi[NB];
#pragma unroll
      for (int i = 0; i < MB; ++i) a[i] = as[k * AS + wm * WTM + i * 16 + (lane & 15)];
#pragma unroll
      for (int j = 0; j < NB; ++j) {
        b[j] = bs[k * BS + wn * WTN + j * 16 + (lane & 15)];
        nbi[j] = -b[j].y;
      }
      if (M3) {
        // cr = T1 (Ar Br), ci = T2 (Ai Bi), cs = T3 ((Ar + Ai)(Br + Bi))
#pragma unroll
        for (int i = 0; i < MB; ++i)
#pragma unroll
          for (int j = 0; j < NB; ++j) {
            cr[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[i].x, b[j].x, cr[i][j], 0, 0, 0);
            ci[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[i].y, b[j].y, ci[i][j], 0, 0, 0);
            cs[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[i].x + a[i].y, b[j].x + b[j].y, cs[i][j], 0, 0, 0);
          }
      } else {
#pragma unroll
        for (int i = 0; i < MB; ++i)
#pragma unroll
          for (int j = 0; j < NB; ++j) {
            cr[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[i].x, b[j].x, cr[i][j], 0, 0, 0);
            ci[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[i].x, b[j].y, ci[i][j], 0, 0, 0);
          }
#pragma unroll
        for (int i = 0; i < MB; ++i)
#pragma unroll
          for (int j = 0; j < NB; ++j) {
            cr[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[i].y, nbi[j], cr[i][j], 0, 0, 0);
            ci[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[i].y, b[j].x, ci[i][j], 0, 0, 0);
          }
      }
    }
    if (kt + 1 < nk) {
      la.template store<AS>(As[cur ^ 1], t);
      lb.template store<BS>(Bs[cur ^ 1], t);
    }
    __syncthreads();
  }

  // epilogue: D = alpha * acc + beta * C
#pragma unroll
  for (int i = 0; i < MB; ++i)
#pragma unroll
    for (int j = 0; j < NB; ++j)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int row = m0 + wm * WTM + i * 16 + (MF4 ? 4 * r + (lane >> 4) : (lane >> 4) + 4 * r);
        const int col = n0 + wn * WTN + j * 16 + (lane & 15);
        if (row < M && col < N) {
          double xr = cr[i][j][r], xi = ci[i][j][r];
          if (M3) {
            const double t1 = xr, t2 = xi;
            xr = t1 - t2;
            xi = cs[i][j][r] - t1 - t2;
          }
          double2 o = make_double2(alpha_re * xr - alpha_im * xi, alpha_re * xi + alpha_im * xr);
          if (beta) {
            const double2 c = pr.C[(int64_t)row * pr.ldc + col];
            o.x += c.x;
            o.y += c.y;
          }
          pr.D[(int64_t)row * pr.ldd + col] = o;
        }
      }
}

template <int BM, int BN, int BK, bool M3, bool MF4 = false, int WGM = 2, int WGN = 2>
void dispatch(hipStream_t st, int opA, int opB, const GemmProb* probs, const int32_t* tile_prob,
              int total, double ar, double ai, int beta) {
  const int per = (total + 7) / 8;
  dim3 grid(per * 8), block(64 * WGM * WGN);
#define HSC_GEMM_CASE(OA, OB)                                                                       \
  if (opA == OA && opB == OB) {                                                                     \
    hipLaunchKernelGGL((k_zgemm<BM, BN, BK, OA, OB, M3, MF4, WGM, WGN>), grid, block, 0, st, probs, tile_prob, total, \
                       ar, ai, beta);                                                               \
    return;                                                                                         \
  }
  HSC_GEMM_CASE(OP_N, OP_N)
  HSC_GEMM_CASE(OP_N, OP_T)
  HSC_GEMM_CASE(OP_N, OP_C)
  HSC_GEMM_CASE(OP_T, OP_N)
  HSC_GEMM_CASE(OP_T, OP_T)
  HSC_GEMM_CASE(OP_T, OP_C)
  HSC_GEMM_CASE(OP_C, OP_N)
  HSC_GEMM_CASE(OP_C, OP_T)
  HSC_GEMM_CASE(OP_C, OP_C)
#undef HSC_GEMM_CASE
}

__global__ void k_mfma_probe(double* out) {
  const int l = threadIdx.x;
  const double a = 1.0 + l;            // A[l%16][l/16]
  const double b = 0.5 * ((l * 7) % 13) - 1.0;   // B[l/16][l%16]
  v4d c = v4d{0, 0, 0, 0};
  c = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
  for (int r = 0; r < 4; ++r) out[l * 4 + r] = c[r];
}

// MFMA-only stream: 8 independent v_mfma_f64_16x16x4_f64 accumulators per wave, no memory
// traffic but one store per lane at the end (the achievable FP64 matrix rate of the chip)
__global__ __launch_bounds__(256) void k_mfma_rate(double* out, int iters) {
  v4d c[8];
#pragma unroll
  for (int i = 0; i < 8; ++i) c[i] = v4d{0, 0, 0, 0};
  const double a = 1.0 + threadIdx.x * 1e-9, b = 1e-3;
  for (int it = 0; it < iters; ++it) {
#pragma unroll
    for (int i = 0; i < 8; ++i) c[i] = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c[i], 0, 0, 0);
  }
  double s = 0;
#pragma unroll
  for (int i = 0; i < 8; ++i) s += c[i][0] + c[i][1] + c[i][2] + c[i][3];
  out[(int64_t)blockIdx.x * blockDim.x + threadIdx.x] = s;
}

}  // namespace

void launch_mfma_rate(hipStream_t st, double* out, int blocks, int iters) {
  hipLaunchKernelGGL(k_mfma_rate, dim3(blocks), dim3(256), 0, st, out, iters);
}

// tile shapes (BM x BN x BK) the launcher offers; 4 waves in a 2 x 2 grid over the tile
static const int kTileM[] = {64, 128, 64, 32, 64, 32, 64, 64, 128};
static const int kTileN[] = {64, 64, 128, 32, 64, 32, 64, 64, 128};

int gemm_tile_kinds() { return 9; }
int gemm_tile_m(int kind) { return kTileM[kind]; }
int gemm_tile_n(int kind) { return kTileN[kind]; }

// tile_kind 0-3 as above with four real products per complex block step; 4 and 5: the 64x64
// and 32x32 tiles with the three-product form; 6 and 7: the 64x64 tile on the 4x4x4 MFMA with
// four and three real products; 8: a 128x128 tile over 8 waves (2 x 4, 64 x 32 each)
void launch_gemm(hipStream_t st, int opA, int opB, const GemmProb* probs, const int32_t* tile_prob,
                 int total_tiles, double alpha_re, double alpha_im, int beta, int tile_kind) {
  if (total_tiles <= 0) return;
  switch (tile_kind) {
    case 1: dispatch<128, 64, 16, false>(st, opA, opB, probs, tile_prob, total_tiles, alpha_re, alpha_im, beta); break;
    case 2: dispatch<64, 128, 16, false>(st, opA, opB, probs, tile_prob, total_tiles, alpha_re, alpha_im, beta); break;
    case 3: dispatch<32, 32, 32, false>(st, opA, opB, probs, tile_prob, total_tiles, alpha_re, alpha_im, beta); break;
    case 4: dispatch<64, 64, 16, true>(st, opA, opB, probs, tile_prob, total_tiles, alpha_re, alpha_im, beta); break;
    case 5: dispatch<32, 32, 32, true>(st, opA, opB, probs, tile_prob, total_tiles, alpha_re, alpha_im, beta); break;
    case 6: dispatch<64, 64, 16, false, true>(st, opA, opB, probs, tile_prob, total_tiles, alpha_re, alpha_im, beta); break;
    case 7: dispatch<64, 64, 16, true, true>(st, opA, opB, probs, tile_prob, total_tiles, alpha_re, alpha_im, beta); break;
    case 8: dispatch<128, 128, 16, false, false, 2, 4>(st, opA, opB, probs, tile_prob, total_tiles, alpha_re, alpha_im, beta); break;
    default: dispatch<64, 64, 16, false>(st, opA, opB, probs, tile_prob, total_tiles, alpha_re, alpha_im, beta); break;
  }
}

void launch_mfma_probe(hipStream_t st, double* out) {
  hipLaunchKernelGGL(k_mfma_probe, dim3(1), dim3(64), 0, st, out);
}

}  // namespace hsc
