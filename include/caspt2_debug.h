/*
 * caspt2_debug.h -- inspection entry points of the caspt2 library, for tests.
 * They expose intermediates of the set-up so that each can be compared with
 * an independent evaluation; none is needed to use the library.
 */
#ifndef CASPT2_DEBUG_H
#define CASPT2_DEBUG_H
#include "caspt2.h"
#ifdef __cplusplus
extern "C" {
#endif

/* C = A * op(B) with the library's FP64 MFMA GEMM.  A [M][K]; B [N][K] when
 * b_is_nk, else [K][N]; C [M][N]; all device, row major. */
CASPT2_API int caspt2_debug_gemm(int32_t b_is_nk, int64_t M, int64_t N, int64_t K, const double* A,
                                 const double* B, double* C);

/* The FP32 operator of the mixed-precision inner solver: sigma = A_L x
 * (Eq. 10 without the source) in FP32, packed layout, device x and sigma of
 * caspt2_vector_length floats.  E_STATE unless the handle holds the FP32
 * operands (created with, or switched to, CASPT2_MIXED). */
CASPT2_API int caspt2_debug_residual_f32(caspt2_handle* h, int32_t L, const float* x, float* sigma);

/* Diagnostics on stderr: 0 off, 1 set-up progress, 2 also per-stage timings
 * of the coupling terms in every residual. */
CASPT2_API int caspt2_set_verbose(caspt2_handle* h, int32_t level);

/* C = A * op(B) with the library's FP32 GEMM (same layout, float data). */
CASPT2_API int caspt2_debug_gemm_f32(int32_t b_is_nk, int64_t M, int64_t N, int64_t K, const float* A,
                                     const float* B, float* C);

/* Copy an intermediate of layout entry k of function set `set` (0 for MS-MR,
 * L for SS-SR) into host memory `out`: which = 0 overlap metric S [na][na],
 * 1 Fock metric F [na][na], 2 row energies [rows], 3 kept count (one
 * double), 4 X [na][nkeep], 5 mu [nkeep]; na = nalpha of the entry. */
CASPT2_API int caspt2_debug_entry(const caspt2_handle* h, int32_t set, int32_t k, int32_t which,
                                  double* out);

/* Source <M~|E_Omega^+ H|N~> for ket N in the function set `set` (packed,
 * device out). */
CASPT2_API int caspt2_debug_source(const caspt2_handle* h, int32_t set, int32_t N, double* out);

/* Symmetric eigendecomposition with the library's Jacobi solver: A [n][n]
 * device (overwritten), w host [n] (unsorted), V device [n][n] (columns). */
CASPT2_API int caspt2_debug_eigh(int32_t n, double* A, double* w, double* V);

/* The same with the solver form chosen: method 0 by size, 1 one workgroup
 * with the matrices in LDS (n <= 64), 2 one workgroup on global memory
 * (n <= 512), 3 one launch pair per rotation step over the whole device, 4
 * one launch per rotation step (alternating matrix buffers), 5 block Jacobi
 * (pairs of 16-index blocks diagonalised in LDS, their rotations applied to
 * the whole matrix by one launch per step of the block tournament); sweeps (host,
 * may be NULL) receives the number of sweeps.  E_ARG for a form that does
 * not take this n. */
CASPT2_API int caspt2_debug_eigh_method(int32_t n, double* A, double* w, double* V, int32_t method,
                                        int32_t* sweeps);

/* The same with an absolute stopping bound for the whole-device forms:
 * sweeps continue until the off-diagonal norm is also <= abs_tol (or stops
 * decreasing).  The set-up solves each block metric this way with abs_tol =
 * 0.1 times the overlap threshold (Sec. II.B), so that no eigenvalue outside
 * 0.9..1.1 times the threshold is misjudged.  method 0 picks the form by size exactly as
 * the set-up does.  E_ARG for a negative or non-finite abs_tol. */
CASPT2_API int caspt2_debug_eigh_abs(int32_t n, double* A, double* w, double* V, int32_t method,
                                     double abs_tol, int32_t* sweeps);

/* Coupling terms applied in packed rows (Eq. 10 with the f of Eq. 11): 1
 * (default) applies the up terms into ccvv in two packed-row passes, the
 * down terms out of ccvv into cavv, caav and ccav in two, and the terms
 * between cavv and aavv/aaav in one, for handles created from now on; 0 runs
 * them term by term through the all-orderings tensors, as every other
 * coupling (for comparing the two).  Returns the previous setting.  Not
 * thread-safe against concurrent caspt2_create. */
CASPT2_API int caspt2_debug_ccvv_passes(int32_t on);

/* For function set `set` of the handle: bit 0 set if its up terms into
 * ccvv run in the packed-row passes, bit 1 if its down terms out of ccvv do,
 * bit 2 if its terms between cavv and aavv/aaav do; 0 if all run term by
 * term; E_ARG for a bad set. */
CASPT2_API int caspt2_debug_ccvv_passes_used(const caspt2_handle* h, int32_t set);

#ifdef __cplusplus
}
#endif
#endif
