/*
 * hsc_kernels.h -- kernel-level entry points of the solver library.
 *
 * These expose the two compute kernels that every step of the solve is built
 * from, so that they can be checked in isolation against a plain reference:
 * the grouped complex128 GEMM (FP64 matrix cores) and the batched blocked
 * Gauss-Jordan inversion with partial pivoting (the A_ii^-1 of Algorithm 1).
 * All pointers are HIP device memory owned by the caller; complex values are
 * (re, im) double pairs; matrices are row-major with the given leading
 * dimension.  Calls are asynchronous on the context's stream (hsc_sync waits).
 */
#ifndef HSC_KERNELS_H_
#define HSC_KERNELS_H_

#include <stdint.h>

#include "hsc.h"

#ifdef __cplusplus
extern "C" {
#endif

/* D = alpha * op(A) * op(B) + beta * C for one problem, op in {0: as is,
 * 1: transpose, 2: conjugate transpose}; op(A) is M x K, op(B) is K x N.
 * beta is 0 or 1; C may equal D (in-place update) and may be NULL when beta = 0.
 * Errors: HSC_E_ARG (sizes < 0, bad op, leading dimension too small), HSC_E_HIP. */
hsc_status hsc_kern_zgemm(hsc_ctx* ctx, int32_t opA, int32_t opB, int32_t M, int32_t N, int32_t K,
                          double alpha_re, double alpha_im, const void* A, int32_t lda, const void* B,
                          int32_t ldb, int32_t beta, const void* C, int32_t ldc, void* D, int32_t ldd);

/* The same product with a chosen tile shape of the grouped GEMM kernel:
 * tile_kind 0 = 64x64x16 (the default above), 1 = 128x64x16, 2 = 64x128x16,
 * 3 = 32x32x32 (rows x columns x depth per workgroup); 4 = 64x64x16 and 5 = 32x32x32
 * with three real products per complex multiply-add (see hsc_solve_opts.complex3m);
 * 6 and 7 = 64x64x16 built on the 4x4x4 FP64 MFMA with four and three real products;
 * 8 = 128x128x16 over 8 waves (four real products).  HSC_E_ARG for another kind. */
hsc_status hsc_kern_zgemm_tile(hsc_ctx* ctx, int32_t tile_kind, int32_t opA, int32_t opB, int32_t M, int32_t N,
                               int32_t K, double alpha_re, double alpha_im, const void* A, int32_t lda,
                               const void* B, int32_t ldb, int32_t beta, const void* C, int32_t ldc, void* D,
                               int32_t ldd);

/* The block product of the double-double solve (hsc_solve_opts.precision >= 1;
 * Algorithm 1's multipliers and Schur updates, Algorithm 2's extraction
 * products) on its own: D = (-1)^negate op(A) op(B) + beta C in complex
 * double-double.  Every element is 32 bytes, four doubles (real hi, real lo,
 * imaginary hi, imaginary lo) with |lo| <= ulp(hi) / 2; row-major, leading
 * dimensions in elements; device pointers.  op 0 = as is, 1 = transposed.
 * config 0-2: FP64 vector units with tiles 0 = 32x32, 1 = 64x32, 2 = 64x64; the
 * result is accurate to about 2^-104 relative to sum_k |op(A)_ik| |op(B)_kj|
 * (products accumulated lazily, renormalised every 8 terms).  config 3: the
 * integer matrix cores (the products of hsc_solve_opts.precision = 3): op(A)
 * split into 16 signed 8-bit slices per element with one power-of-two scale per
 * row, op(B) likewise per column (the error-free splitting of Ozaki et al.),
 * exact int32 sums of slice products, the leading 136 of 256 slice pairs
 * combined in double-double; the error is at most about K 2^-104 max_k
 * (|Re| + |Im|) of row i of op(A) times the same of column j of op(B), plus
 * 2^-104 |C_ij|, K <= 10880.  config 4: as 3 with 15 slices (120 pairs, the
 * products of hsc_solve_opts.slices = 15): K 2^-97 instead of K 2^-104,
 * K <= 11648.  beta is 0 or 1; C
 * may equal D and may be NULL when beta = 0.  Synchronous.
 * Errors: HSC_E_ARG (sizes < 0, bad op or config, leading dimension too small,
 * K beyond the limit of config 3 or 4), HSC_E_OOM, HSC_E_HIP. */
hsc_status hsc_kern_zgemm_dd(hsc_ctx* ctx, int32_t config, int32_t opA, int32_t opB, int32_t M, int32_t N,
                             int32_t K, int32_t negate, const void* A, int32_t lda, const void* B, int32_t ldb,
                             int32_t beta, const void* C, int32_t ldc, void* D, int32_t ldd);

/* For callers that cannot allocate device memory (code under HIP graph capture,
 * tight serving loops, harnesses that forbid hipMalloc): the double-double
 * product of hsc_kern_zgemm_dd with config 3 (8-bit slices on the integer
 * matrix cores), same arguments, same kernels, same results, with every
 * descriptor, slice plane and scale in one static device array of 64 MiB per
 * GPU (held from the first context on that GPU until the process ends); the
 * call allocates nothing and does not wait: it enqueues four kernels on the
 * context's stream and returns (D is valid after hsc_sync or a stream
 * synchronisation).  Limit: the scratch of one product, 48 (Mp + Np) Kp bytes
 * plus maps (Mp, Np = M, N rounded up to 32, Kp = K rounded up to 64), must fit
 * 64 MiB (e.g. M = N = 1024 with K <= 640); larger products return HSC_E_ARG.
 * Every call on one GPU shares that array and leaves it holding its own
 * intermediates: calls that overlap on one GPU (other streams, other contexts,
 * other threads) race and must be serialised by the caller.
 * Errors: HSC_E_ARG (as hsc_kern_zgemm_dd, or too large), HSC_E_HIP. */
hsc_status hsc_kern_zgemm_dd_noalloc(hsc_ctx* ctx, int32_t opA, int32_t opB, int32_t M, int32_t N, int32_t K,
                                     int32_t negate, const void* A, int32_t lda, const void* B, int32_t ldb,
                                     int32_t beta, const void* C, int32_t ldc, void* D, int32_t ldd);

/* The pivot-block inverse of the double-double fold (hsc_solve_opts.precision
 * >= 1, Algorithm 1's A_ii^-1) on its own, with the solver's own launch
 * sequence: two-level blocked Gauss-Jordan with partial pivoting inside the
 * block, in complex double-double (panels of 8, 4 or 2 columns inside
 * super-panels of 64; each super-panel's pivot rows update the other columns in
 * one rank-64 product, on the integer matrix cores when matrix_cores = 1 as with
 * precision 3, else on the vector units).  X (order n, leading dimension ld,
 * 32-byte elements as in hsc_kern_zgemm_dd; device) is overwritten; Y (ldy)
 * receives X^-1.  status (device int32, may be NULL) receives 0 or
 * HSC_E_SINGULAR.  1 <= n <= 4096.  Synchronous.
 * Errors: HSC_E_ARG, HSC_E_OOM, HSC_E_HIP. */
hsc_status hsc_kern_zinv_dd(hsc_ctx* ctx, int32_t n, void* X, int32_t ld, void* Y, int32_t ldy, int32_t* status,
                            int32_t matrix_cores);

/* Invert `count` matrices of order n[k] in place (X[k], leading dimension ld[k])
 * and write X[k]^-1 into Y[k] (leading dimension ldy[k]); all pointer/size
 * arrays are host arrays.  status (device, int32[count], may be NULL) receives
 * 0 or HSC_E_SINGULAR per matrix.  n[k] <= 4096.  Errors: HSC_E_ARG, HSC_E_OOM,
 * HSC_E_HIP. */
hsc_status hsc_kern_zinv_batched(hsc_ctx* ctx, int32_t count, const int32_t* n, void* const* X,
                                 const int32_t* ld, void* const* Y, const int32_t* ldy, int32_t* status);

/* Rate of a plain FP64 MFMA stream: a kernel issuing only v_mfma_f64_16x16x4_f64 on 8
 * independent accumulators per wave (4096 workgroups of 4 waves, no memory traffic but one store
 * per lane) is timed with HIP events; *tflops (host) receives the best of three runs in TFLOP/s.
 * This instruction pattern is not the chip's ceiling (a GEMM inner loop with more independent
 * products per step issues faster); it is a repeatable reference point.  Synchronous.
 * Errors: HSC_E_ARG, HSC_E_OOM, HSC_E_HIP. */
hsc_status hsc_kern_mfma_rate(hsc_ctx* ctx, double* tflops);

/* One wave of v_mfma_f64_16x16x4_f64 with A[l%16][l/16] = 1 + l and
 * B[l/16][l%16] = 0.5*((7l) mod 13) - 1 (l = lane); writes the 4 accumulator
 * registers of each lane to out[l*4 + r] (device, 256 doubles); register r of
 * lane l holds D[l/16 + 4r][l%16].  Used to check the lane layout the GEMM
 * kernel assumes. */
hsc_status hsc_kern_mfma_probe(hsc_ctx* ctx, double* out);

#ifdef __cplusplus
}
#endif

#endif /* HSC_KERNELS_H_ */
