// Declarations of the block-tiled path (superoperators of n = 64 T > 64),
// shared by its kernels and the host library; kept apart from the slice
// kernels' declarations in internal.hpp.
#pragma once
#include "internal.hpp"

namespace lmag {

constexpr int MAX_BIG_NB = 64;
// consecutive slices per workgroup in the basis assembly and trace kernels of
// the block-tiled path (each basis tile is fetched once for all of them)
constexpr int kBigSlicesPerGroup = 4;
// Block-tiled path: Neumann levels of the Pade-3 denominator inverse (the
// single-precision bound of neumann_levels; a slice whose bound does not hold
// takes all of them) and the largest supported scaling exponent.
constexpr int kBigNeumannLevels = 4;
constexpr int kBigMaxSquarings = 64;

struct BigGemmArgs {
  int n, batch;
  const void* A; const int32_t* Ai;
  const void* B; const int32_t* Bi;
  const void* C; const int32_t* Ci;      // output
  const void* D; const int32_t* Di;      // epilogue addend (may alias C)
  const void* D2; const int32_t* D2i;    // second addend (may be null)
  double alpha, beta, gamma, beta2;
  int transA, transB;
  const int8_t* pred; int pred_stride; int pred_thresh;   // active if pred[i*stride] > thresh
  int variant;   // FP32 product kernel (autotuned): 0 register-B tiles, 16x16x4 MFMA;
                 // 1 quadrant per wave, 16x16x4; 2 quadrant per wave, 32x32x2;
                 // 3 quadrant per wave, FP32 operands split into three bf16 pieces
                 // on the 16x16x32 bf16 MFMA; 4 as 0 with two output tiles (eight
                 // waves) per workgroup sharing each staged A tile (n / 64 even);
                 // 5 as 0 with every product's tiles on one XCD (n <= 1024);
                 // 6 as 0 without the operand pipeline, three workgroups per CU;
                 // 7 as 6 with every product's tiles on one XCD (n <= 1024);
                 // 8 as 0 with the A tiles double-buffered in LDS by direct
                 // global-to-LDS loads (with the XCD grouping where n <= 1024)
  // optional second output of the same tile (kernels 0, 5, 6, 7, 8; not with
  // pred): C2 = c2_c C + c2_e E2 + c2_gamma I, E2 may be null
  const void* C2; const int32_t* C2i;
  const void* E2; const int32_t* E2i;
  double c2_c, c2_e, c2_gamma;
};
constexpr int kBigGemmVariants = 9;
constexpr int kBigGemmDefault = 0;   // product kernel of an untuned block-tiled call
struct BigAxpbyArgs {
  int n, batch;
  const void* X; const int32_t* Xi;
  const void* Z; const int32_t* Zi;
  void* Y; const int32_t* Yi;
  double a, c, d;
  const int8_t* ms;         // if set: a *= 2^-s of entry Yi[b] (ms[2 i + 1])
};
// Tile lists of the basis (block-tiled path): the basis elements whose 64 x 64
// tile at position t = ti * Tn + tj is not all zero are tile_j[tile_ptr[t] ..
// tile_ptr[t + 1]), ascending; null pointers mean every element.
struct BigOmegaArgs {
  int n, n_slices, nb;
  const void* basis; const double* alpha;
  void* omega; double* part;
  int8_t* ms; int8_t* nlev;
  double b3[4];
  const int32_t* tile_ptr; const int32_t* tile_j;
};
struct BigTraceArgs {
  int n, n_slices, nb, first_slice, trans_basis;
  const void* K; const void* basis;
  double* part; double* gtrace;
  const int32_t* tile_ptr; const int32_t* tile_j;
};
// flags[j][t] = 1 if tile t of basis element j has a nonzero entry (FP64 basis)
hipError_t launch_tile_flags(const double* basis, int nb, int n, uint8_t* flags, hipStream_t s);
struct BigFidArgs {
  int n, n_items, d;
  const void* U; const int32_t* U_index;
  const double* st64; const int32_t* target;
  double* F; const int32_t* F_index;
};
hipError_t launch_bgemm(int prec, const BigGemmArgs& g, hipStream_t s);
hipError_t launch_baxpby(int prec, const BigAxpbyArgs& g, hipStream_t s);
hipError_t launch_bomega(int prec, const BigOmegaArgs& g, hipStream_t s);
hipError_t launch_bnorm_dense(int prec, const BigOmegaArgs& g, hipStream_t s);
hipError_t launch_btraces(int prec, const BigTraceArgs& g, hipStream_t s);
hipError_t launch_bfidelity(int prec, const BigFidArgs& g, hipStream_t s);
hipError_t launch_blift(const double* H, int d, double* out, hipStream_t s);
hipError_t launch_bdissipator(const double* Ls, int n_jump, int d, double* ldl, double* out, hipStream_t s);
hipError_t launch_btargets(const double* U, int n_targets, int d, double* st64, float* st32, hipStream_t s);
hipError_t launch_btraces_sum(const BigTraceArgs& g, hipStream_t s);

// the same path in the real basis of Hermitian operators (k_real.hip): real FP32
// matrices of n x n floats behind the same argument structures
hipError_t launch_rgemm(const BigGemmArgs& g, hipStream_t s);
hipError_t launch_raxpby(const BigAxpbyArgs& g, hipStream_t s);
hipError_t launch_romega(const BigOmegaArgs& g, hipStream_t s);
hipError_t launch_rnorm_dense(const BigOmegaArgs& g, hipStream_t s);
hipError_t launch_rtraces(const BigTraceArgs& g, hipStream_t s);
hipError_t launch_rfidelity(const BigFidArgs& g, hipStream_t s);
// R = T S T^dag for nmat complex FP64 superoperators (column stacking) -> real FP64
hipError_t launch_to_real(const double* S, int d, int nmat, double* R, hipStream_t s);
// out[Yi[b]] = T^dag (I + R[Xi[b]]) T, complex FP32 (column stacking)
hipError_t launch_from_real(const float* R, const int32_t* Xi, int d, int batch, void* out, const int32_t* Yi,
                            hipStream_t s);
hipError_t launch_rtile_flags(const double* basis, int nb, int n, uint8_t* flags, hipStream_t s);
hipError_t launch_rcast(const double* in, float* out, size_t count, hipStream_t s);

// The 64 x 64 path in the same basis (d <= 8, complex tiles with zero
// imaginary parts). In place on count row-major 64 x 64 complex FP64 tiles:
// S <- (Re(T S T^dag), 0), also written as complex FP32 into out32 if given.
hipError_t launch_tile_to_real(double* tiles, int count, int d, float* out32, hipStream_t s);
// In place on the n x n complex FP32 outputs (n = d^2) of the items' sources:
// (R, .) <- T^dag R T.
hipError_t launch_out_from_real(void* out, const Item* items, int n_items, int d, hipStream_t s);

}  // namespace lmag
