/*
 * lmag_debug.h -- test and instrumentation entry points of liblmag.so.
 *
 * Not part of the propagator's interface (include/lmag.h): unit-test kernels
 * on single 64 x 64 tiles, used by the library's own tests to check the tile
 * product, the unpivoted inverse and the scaled Pade exponential in isolation,
 * the block-tiled product kernels at any supported size, and a per-phase cycle
 * counter of the slice kernels used to place memory
 * traffic inside the products. Same conventions and status codes as lmag.h.
 */
#ifndef LMAG_DEBUG_H
#define LMAG_DEBUG_H

#include "lmag.h"

#ifdef __cplusplus
extern "C" {
#endif

/* Instrumentation: per-phase shader-clock cycles of workgroup 0 of the slice
 * kernels, summed over the calls made while enabled. enable = 1 clears and
 * starts recording, 0 stops, -1 leaves the state; out (if not NULL) receives
 * 32 counters (0-6 forward phases, 16-25 backward phases). Blocks. */
lmag_status lmag_debug_phase_cycles(lmag_ctx *ctx, int enable, int64_t *out /*[32]*/);

/* Unit-test kernels on single 64 x 64 complex tiles of the given precision,
 * DEVICE pointers, row-major. C = op(A) B (op = transpose when transA != 0);
 * C = A^{-1} (no pivoting; A must be column diagonally dominant);
 * C = exp(A) by the library's scaled Pade path, ms_out[0..1] = (m, s). */
lmag_status lmag_debug_tile_gemm(lmag_ctx *ctx, int precision, const void *A, const void *B,
                                 void *C, int transA, void *hip_stream);
lmag_status lmag_debug_tile_inverse(lmag_ctx *ctx, int precision, const void *A, void *C,
                                    void *hip_stream);
lmag_status lmag_debug_tile_expm(lmag_ctx *ctx, int precision, const void *A, void *C,
                                 int8_t *ms_out, void *hip_stream);

/* The block-tiled product kernels on their own: C_b = A_b B_b for b < batch,
 * complex FP32 n x n matrices (n a multiple of 64, 64 <= n <= 4096), DEVICE
 * pointers to batch contiguous row-major matrices each, C distinct from A and
 * B. variant selects the product kernel as the autotuner does (0..8; a kernel
 * whose shape condition fails runs kernel 0). Asynchronous on hip_stream. */
lmag_status lmag_debug_block_gemm(lmag_ctx *ctx, int n, int batch, const void *A, const void *B,
                                  void *C, int variant, void *hip_stream);

#ifdef __cplusplus
}
#endif

#endif /* LMAG_DEBUG_H */
