// Launchers of the HIP kernels (gfx950).  All take a stream and return
// hipError_t from the launch.
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>
#include <vector>

namespace caspt2 {

// Y[r][lead][t] = sign[r][t] * X[lead][src[r][t]] (0 where src < 0)
hipError_t launch_gather_apply(const double* X, int64_t nlead, int64_t dim_from,
                               const int32_t* src, const double* sign, int na, int64_t dim_to,
                               double* Y, hipStream_t s);

// C = alpha * A * op(B) + beta * C, FP64 on MFMA.
//   A: [M][K] row major, lda;  B: NT -> [N][K] (ldb), NN -> [K][N] (ldb)
//   C: [M][N] row major, ldc.  batch with element strides sA, sB, sC.
hipError_t gemm_f64(bool b_is_nk, int64_t M, int64_t N, int64_t K, double alpha, const double* A,
                    int64_t lda, int64_t sA, const double* B, int64_t ldb, int64_t sB, double beta,
                    double* C, int64_t ldc, int64_t sC, int batch, hipStream_t s);
// the same product (batch 1, no strides) split over K when it has fewer than
// 512 tiles of 64 x 64 and K >= 128: partial products in ws (ws_n doubles;
// split count reduced to fit, plain product if none fits), then one summing
// pass, C = alpha sum + beta C.  Deterministic: the split count depends on
// the shape and ws_n only.
hipError_t gemm_f64_ws(bool b_is_nk, int64_t M, int64_t N, int64_t K, double alpha, const double* A, int64_t lda,
                       const double* B, int64_t ldb, double beta, double* C, int64_t ldc, double* ws, int64_t ws_n,
                       hipStream_t s);
// batched C_p = A_p B_p (B_p [K][N], beta 0), tile order for few m tiles
hipError_t gemm_f64_batched(int64_t M, int64_t N, int64_t K, const double* A, int64_t lda, int64_t sA,
                            const double* B, int64_t ldb, int64_t sB, double* C, int64_t ldc, int64_t sC,
                            int batch, hipStream_t s);

// Launch choices of a residual entry; a field left at its default means
// "by rule" (the launcher's built-in choice for the shape).  The autotuner
// sets them per entry from timings.
constexpr int BK_RESIDUAL = 16;   // K tile of the residual GEMM (split ranges are multiples)
struct LaunchTune {
  int splitk = -1;     // residual GEMM: K splits (1 = none)
  int order = -1;      // residual GEMM tile order: 0/1 plain (n or m tiles on
                       // grid x), 2 XCD-grouped
  unsigned grid = 0;   // streaming residual kernels: cap on the workgroup count
  int tile = 0;        // residual GEMM tile rows: 64 or 128 (without K splits)
  int kb = 0;          // residual GEMM K tile: 16 or 32 (without K splits)
  int occ = 0;         // residual GEMM without K splits: waves per SIMD asked of
                       // the compiler (1, 2 with 128-row tiles, 3 with 64-row tiles)
  int plain = 0;       // streaming MFMA residual: 1 = without the X prefetch
  int breg = 0;        // streaming MFMA residual (nalpha <= 32): 1 = S, F operands in registers
};

// Residual of one packed entry on MFMA:
//   C[m][n] = V[m][n] + d[m] * (X S)[m][n] + (X F)[m][n]   (V may be null)
// X [M][K], S and F [K][N] row major (symmetric in use), d [M].
// With few output tiles (small M) the K range is split over workgroups
// (residual_splitk(M, N, K) splits, workspace ws of >= splits * 2 * M * N
// doubles; without it the plain kernel runs).
hipError_t residual_gemm_f64(int64_t M, int64_t N, int64_t K, const double* X, int64_t ldx,
                             const double* S, const double* F, const double* d, double dshift,
                             const double* V, int64_t ldv, double* C, int64_t ldc, hipStream_t s,
                             double* ws = nullptr, int64_t ws_len = 0, LaunchTune tune = {});
// number of K splits residual_gemm_f64 uses by rule for this shape (1: none)
int residual_splitk(int64_t M, int64_t N, int64_t K);
// Same for small K = N (<= 64): streaming kernel with S, F staged in LDS.
hipError_t residual_small_f64(int64_t M, int64_t N, const double* X, const double* S,
                              const double* F, const double* d, double dshift, const double* V,
                              double* C, hipStream_t s, LaunchTune tune = {});

// FP32 form of residual_small_f64 for K = N <= 64 (SIMT, S and F in LDS).
hipError_t residual_small_f32(int64_t M, int64_t N, const float* X, const float* S, const float* F,
                              const float* d, float dshift, const float* V, float* C,
                              hipStream_t s);

// Row energies of a packed entry in separable form: eps(m) = A[m / nB] +
// B[m % nB] (first orbital unit of the row / the remaining units).
template <typename T>
struct RowEnergy {
  const T* A;
  const T* B;
  uint32_t nB;
};
// A[a] = eps[a nB], B[b] = eps[b] - eps[0]  (a < nA, b < nB)
hipError_t split_energies(int64_t nA, int64_t nB, const double* eps, double* A, double* B,
                          hipStream_t s);

// Streaming residual of two consecutive packed entries with nalpha = nst
// (<= 4), e.g. ccvv '+' and '-': rows [0, M0) use (S0, F0, d0), rows
// [M0, M0+M1) use (S1, F1, d1).  X, V, C are [M0+M1][nst].  T: double, float.
template <typename T>
hipError_t residual_rows(int nst, int64_t M0, int64_t M1, const T* X, const T* S0, const T* F0,
                         const T* S1, const T* F1, RowEnergy<T> d0, RowEnergy<T> d1, T dshift,
                         const T* V, T* C, hipStream_t s, LaunchTune tune = {});

// C = alpha * A * op(B) + beta * C in FP32 (SIMT FMA, 64 x 64 tiles); same
// operand conventions as gemm_f64.
hipError_t gemm_f32(bool b_is_nk, int64_t M, int64_t N, int64_t K, float alpha, const float* A,
                    int64_t lda, int64_t sA, const float* B, int64_t ldb, int64_t sB, float beta,
                    float* C, int64_t ldc, int64_t sC, int batch, hipStream_t s);
// FP32 form of residual_gemm_f64.
hipError_t residual_gemm_f32(int64_t M, int64_t N, int64_t K, const float* X, int64_t ldx,
                             const float* S, const float* F, const float* d, float dshift,
                             const float* V, int64_t ldv, float* C, int64_t ldc, hipStream_t s);

// out[m][j] = sum_i in[m][i] W[i * ws_in + j * ws_out] for rows of nin <= 8
// inputs and nout <= 8 outputs (in [M][nin], out [M][nout]).  T: double, float.
template <typename T>
hipError_t transform_rows(int64_t M, int nin, int nout, const T* in, const T* W, int ws_in,
                          int ws_out, T* out, hipStream_t s);

// dst[sum_k idx_k * dstride_k] += c * src[flat], src dims dims[0..nd)
hipError_t permute_axpy(int nd, const int64_t* dims, const int64_t* dstride, double c,
                        const double* src, double* dst, hipStream_t s);
// dst[sum_k i_k dstride[k]] = src[(i_0, .., i_{nd-1})]: a permuted copy of
// all elements (nd <= 10)
template <typename T>
hipError_t permute_copy(int nd, const int64_t* dims, const int64_t* dstride, const T* src, T* dst, hipStream_t s);

// y[j] += sum_i c[i] * G[i][j], i < ni, j < nj   (c on device)
hipError_t contract_lead(int64_t ni, int64_t nj, const double* c, const double* G, double* y,
                         hipStream_t s);

// B [Q][nmo][nmo] -> Bt [p-range x q-range][Q] for a block of orbitals
hipError_t df_pack(const double* B, int naux, int nmo, int p0, int np, int q0, int nq, double* Bt,
                   hipStream_t s);

// Packed term contraction (sources and couplings); see kernels.hip.
struct TermDesc {
  int block;            // output block id
  int nslot;            // number of external slots of the output block
  int slot_dim[4];      // dimension of each slot (nc or nv)
  int swap_k[2], swap_l[2], nswap;
  int chi[2];           // character of this output entry
  int strict[2];        // 1 where chi = -1 (strict pair)
  int64_t nrow, nalpha;
  int64_t ldo;          // row stride of the output (== nalpha)
  // coefficient tensor: up to 4 axes; axis a takes its index from
  // slot c_slot[a] (>= 0) or from active label -1-c_slot[a]
  int ncax;
  int c_slot[4];
  int64_t c_stride[4];
  // active labels summed: nopact (0..3), each of range na
  int nopact, na;
  // G layout: [opact (na^nopact)][nalpha][gcols], ket column gcol
  int64_t gcols;
  int gcol;
  int64_t galpha;       // alpha extent of G (>= nalpha) and offset of column 0
  int64_t goff;
  int mode_avg;         // 1: evaluate on the representative only, weight 1
  double scale;
};
hipError_t term_source(const TermDesc& d, const double* C, const double* G, double* out,
                       hipStream_t s);

// Packed representation of one block (for gathering all-orderings values):
// entries (characters) with their offsets relative to a base pointer.
struct PackInfo {
  int nslot;
  int slot_dim[4];
  int nswap;
  int swap_k[2], swap_l[2];
  int nent;               // character entries present (1 or 2)
  int chi[2][2];          // chi[entry][swap]
  int64_t offset[2];      // entry offsets (doubles) from the base pointer
  int64_t rowlen;         // doubles per packed row
};

// All-orderings tensors of a block: rows are the external index tuples in
// row-major slot order (dims slot_dim), rowlen doubles per row.
struct AllDesc {
  int nslot;
  int slot_dim[4];
};

// out_all[e][c] = x_all[e][c] for every tuple e (unpack packed rows)
template <typename T>
hipError_t unpack_all(const PackInfo& p, const AllDesc& a, const T* packed, T* out_all,
                      hipStream_t s);
// packed[row][c] += sum_{images e of the orbit} w chi(pi_e) in_all[e][c] for
// one packed entry described by d (decode, images, character; d.ldo = row
// stride, d.nalpha = columns)
template <typename T>
hipError_t pack_acc(const TermDesc& d, const AllDesc& a, const T* in_all, T* packed,
                    hipStream_t s);
// the same for the two ccvv entries at once (all-orderings [nc][nc][nv][nv]
// rows of ncol <= 4; plus: entry (+,+), minus: entry (-,-) or null),
// LDS-tiled so that the (a,b)-swapped images are read along rows
template <typename T>
hipError_t pack_ccvv(int nc, int nv, int ncol, const T* in_all, T* plus, T* minus, hipStream_t s);
// the transpose: packed ccvv + and - entries (minus may be NULL) into the
// all-orderings tensor [i][j][a][b][ncol], every element written
template <typename T>
hipError_t unpack_ccvv(int nc, int nv, int ncol, const T* plus, const T* minus, T* out_all, hipStream_t s);

// Index sources of the coupling kernels: a value >= 0 is a bra slot, -1 - s
// is summed external label s, -10 is the operator's active label y.
struct CoupleDesc {
  AllDesc bra, ket;
  int ket_src[4];
  int fx_src, fy_src;
  int64_t f_stride;       // row stride of f; f points at the block origin
  int nsum;
  int sum_dim[2];
  int ny;                 // 1 or na
  int64_t ncol;           // alpha columns (bra for expand, ket for reduce)
};
// expand (bra has more external slots):
//   out_all[e_b][a] += sum_y f(.) W_all[e_k(e_b)][y * ncol + a]
template <typename T>
// mode: 0 by size, 1 ket-parallel (a thread per ket row loops over the free
// bra slots), 2 output-parallel (a thread per bra row)
hipError_t couple_expand(const CoupleDesc& d, const double* f, const T* W, T* out_all,
                         hipStream_t s, int mode = 0);
// up term with the active contraction fused in (G [(y, alpha_b)][alpha_k]
// staged in LDS; X_all the ket's all-orderings rows of nak values):
//   out_all[e_b][a] += sum_y f(.) sum_k X_all[e_k(e_b)][k] G[y ncol + a][k]
// usable when couple_up_fusable (G small enough for LDS)
template <typename T>
bool couple_up_fusable(const CoupleDesc& d, int64_t nak);
template <typename T>
hipError_t couple_up_fused(const CoupleDesc& d, const double* f, const T* X_all, int64_t nak, const T* G,
                           T* out_all, hipStream_t s);
// reduce (bra has fewer external slots):
//   Y_all[e_b][y * ncol + a] = sum_z f(.) X_all[e_k(e_b, z)][a]
template <typename T>
hipError_t couple_reduce(const CoupleDesc& d, const double* f, const T* X, T* Y,
                         hipStream_t s);
// reduce reading the ket from its packed rows (pk: packed layout of the ket
// block, offsets relative to x) instead of an all-orderings copy
template <typename T>
hipError_t couple_reduce_packed(const CoupleDesc& d, const PackInfo& pk, const double* f, const T* x,
                                T* Y, hipStream_t s);
// out[r][a] += sum_c Y[r][c] G[a][c] for rows r < nrows, a < nab, c < width
// (G [nab][width]); one thread per row, for nab, width <= 8 (the contraction
// of a down term's reduce with its active tensor when both are narrow)
template <typename T>
hipError_t rows_small_gemm(int64_t nrows, int nab, int width, const T* Y, const T* G, T* out, hipStream_t s);

// The up coupling terms into ccvv added straight into its packed rows
// (couple_ccvv.hip).  Absent terms are NULL.  Row layouts are the
// all-orderings ones: X_cavv [i][a][b][nak], W5/W6 (caav) [i][a][ncol],
// W3/W4 (ccav) [i][j][a][ny * ncol]; G1/G2 [ny * ncol][nak] (nak = ny * ncol).
// f(y, j) = fA[y * fA_stride + j], f(v, j) = fC[v * fC_stride + j],
// f(v, y) = fV[v * fV_stride + y].  plus/minus: the packed + and - entries
// (rows of ncol values; minus may be NULL).
template <typename T>
struct CcvvUpArgs {
  int nc = 0, nv = 0, ncol = 0, ny = 0, nak = 0;
  const T* X = nullptr;
  const T* G1 = nullptr;
  const T* G2 = nullptr;
  const double* fA = nullptr;
  int64_t fA_stride = 0;
  const T* W5 = nullptr;
  const T* W6 = nullptr;
  const double* fC = nullptr;
  int64_t fC_stride = 0;
  const T* W3 = nullptr;
  const T* W4 = nullptr;
  const double* fV = nullptr;
  int64_t fV_stride = 0;
  T* plus = nullptr;
  T* minus = nullptr;
};
bool ccvv_up_supported(int nc, int nv, int ncol, int ny, int nak);
// virtual pairs per workgroup of the virtual-pair passes (ccvv and cavv)
constexpr int VPAIR_GROUP = 3;
// workgroup table of the virtual-pair passes: a << 16 | b0 per group of
// VPAIR_GROUP pairs (a, b0 ..)
// b_major: b0 outermost, in per-XCD runs (the cavv pass reads rows of the
// pair's second index); else a outermost
std::vector<uint32_t> ccvv_up_groups(int nv, bool b_major = false);
template <typename T>
hipError_t ccvv_up_apply(const CcvvUpArgs<T>& p, const uint32_t* groups, int64_t ngroups, hipStream_t s);

// The down terms out of ccvv into cavv, caav and ccav read straight from the
// packed ccvv rows (couple_ccvv.hip).  xp/xm: packed ccvv + and - (xm may be
// NULL); G1/G2 [nab][ny * ncol] of the two cavv terms (NULL if absent);
// f(z, y) = fA[z * fA_stride + y] (closed, active); sp/sm: packed cavv + and
// - sigma, added to; f(z, w) = fC[z * fC_stride + w] (closed, virtual);
// Tw: work [2][nc][nv][nv][ncol]; Y [2][nc][nv][ncol] receives the two caav
// reductions (caav rows (i, v)), to be contracted with the terms' G.
template <typename T>
struct CcvvDownArgs {
  int nc = 0, nv = 0, ncol = 0, ny = 0, nab = 0;
  const T* xp = nullptr;
  const T* xm = nullptr;
  const T* G1 = nullptr;
  const T* G2 = nullptr;
  const double* fA = nullptr;
  int64_t fA_stride = 0;
  T* sp = nullptr;
  T* sm = nullptr;
  const double* fC = nullptr;
  int64_t fC_stride = 0;
  T* Tw = nullptr;
  T* Y = nullptr;
  // into ccav: G3/G4 [nab3][ny * ncol]; f(y, w) = fV[y * fV_stride + w]
  // (active, virtual); cp/cm: packed ccav + and - sigma, added to
  int nab3 = 0;
  const T* G3 = nullptr;
  const T* G4 = nullptr;
  const double* fV = nullptr;
  int64_t fV_stride = 0;
  T* cp = nullptr;
  T* cm = nullptr;
};
bool ccvv_down_supported(int nc, int nv, int ncol, int ny, int nab);
template <typename T>
// groups: the workgroup table of ccvv_up_groups (device), ngroups its length
hipError_t ccvv_down_apply(const CcvvDownArgs<T>& p, const uint32_t* groups, int64_t ngroups, hipStream_t s);

// Coupling terms of cavv with aavv and aaav in the packed rows
// (couple_cavv.hip).  nak: cavv columns; ny: active orbitals.  Absent parts
// are NULL.  Q+-: [aavv +/- rows][ny * nak] (packed aavv rows times the
// summed and differenced G of the two up terms); f(y, i) = fAC[y * stride + i];
// B+-: [nv][nak] (aaav rows times the G sum and difference); f(v, i) =
// fVC[v * stride + i]; sp/sm: packed cavv sigma (added to); xp/xm: packed
// cavv x; f(z, y) = fCA[z * stride + y]; Zp/Zm: [aavv +/- rows][ny * nak]
// (written) for the down terms into aavv.
template <typename T>
struct CavvArgs {
  int nc = 0, nv = 0, nak = 0, ny = 0;
  const T* Qp = nullptr;
  const T* Qm = nullptr;
  const double* fAC = nullptr;
  int64_t fAC_stride = 0;
  const T* Bp = nullptr;
  const T* Bm = nullptr;
  const double* fVC = nullptr;
  int64_t fVC_stride = 0;
  T* sp = nullptr;
  T* sm = nullptr;
  const T* xp = nullptr;
  const T* xm = nullptr;
  const double* fCA = nullptr;
  int64_t fCA_stride = 0;
  T* Zp = nullptr;
  T* Zm = nullptr;
  // up from caav: C+- [nc * nv][ny * nak] (caav rows times the G sum and
  // difference); f(v, y) = fVA[v * stride + y]
  const T* Cp = nullptr;
  const T* Cm = nullptr;
  const double* fVA = nullptr;
  int64_t fVA_stride = 0;
  // down into caav and aaav (closed-index pass over the packed cavv x):
  // Sb, Db [nc * nv][ny * nak] (written), f(y, w) = fAV[y * stride + w];
  // Scd [2][nc][nv][nak] (written: per closed index, summed afterwards into
  // Sc, Dc [2][nv][nak]), f(z, w) = fCV[z * stride + w]
  T* Sb = nullptr;
  T* Db = nullptr;
  const double* fAV = nullptr;
  int64_t fAV_stride = 0;
  T* Scd = nullptr;
  T* Sc = nullptr;
  const double* fCV = nullptr;
  int64_t fCV_stride = 0;
};
bool cavv_pass_supported(int nc, int nv, int nak, int ny);
// groups: the table of ccvv_up_groups
template <typename T>
hipError_t cavv_pass_apply(const CavvArgs<T>& p, const uint32_t* groups, int64_t ngroups, hipStream_t s);

// X0[i][k] = Q[i][idx[k]] * scale[k]  (Q is n x ncq, X0 is n x nk)
hipError_t select_scale_cols(int64_t n, int64_t ncq, const double* Q, const int32_t* idx,
                             const double* scale, int64_t nk, double* X0, hipStream_t s);

// Jacobi eigensolver of a symmetric n x n matrix A (destroyed; diagonal ->
// eigenvalues, unsorted); V receives eigenvectors (columns).  ws: device
// workspace of >= jacobi_ws_doubles(n) doubles. sweeps: max sweeps.  method: 0
// by size (the LDS form up to 64, the block form above), 1 one workgroup with A and V in LDS (n <= 64), 2 one
// workgroup on global memory (n <= 512), 3 launches over the whole chip per
// rotation step: one per step when A2 (a second n x n device buffer) is
// given, else a parameter launch and a rotation launch; 5 block Jacobi over
// pairs of 16-index blocks (two launches per step of the block tournament).  hpin: page-locked
// host memory (hipHostMalloc) of >= 2 doubles, the target of the per-sweep
// convergence norms and of the sweep count (required).  The whole-device
// forms stop when the off-diagonal Frobenius norm is <= tol |A|_F and, if
// abs_tol > 0, also <= abs_tol (an absolute bound on how far a diagonal
// element can be from an eigenvalue, for decisions against a fixed
// threshold), or when it no longer decreases (the round-off floor).
constexpr int JACOBI_WG_AUTO = 64;   // largest n solved by one workgroup (LDS form) by default
constexpr int JACOBI_BLOCK_MIN = 65;   // smallest n the block form takes by default
// pairs of 16-index blocks of the block form (its rotations: 1024 doubles each)
inline int64_t bjac_pairs(int64_t n) {
  const int64_t nb = (n + 15) / 16;
  return (nb + (nb & 1)) / 2;
}
inline int64_t jacobi_ws_doubles(int64_t n) { return 4 * n + 16 + 2 * 256 + 1024 * bjac_pairs(n); }
hipError_t jacobi_eigh(int n, double* A, double* V, double* ws, int max_sweeps, double tol,
                       hipStream_t s, int* sweeps_done, int method, double* A2, double* hpin,
                       double abs_tol = 0.0);

// vector kernels (element types as instantiated in kernels.hip)
template <typename T>  // FP64 accumulation; out on device (1 double); partial >= 1024 doubles
hipError_t vec_dot(int64_t n, const T* x, const T* y, double* partial, double* out, hipStream_t s);
template <typename X, typename Y>  // y += a x
hipError_t vec_axpy(int64_t n, double a, const X* x, Y* y, hipStream_t s);
template <typename T>  // y = x + a y
hipError_t vec_xpay(int64_t n, const T* x, double a, T* y, hipStream_t s);
template <typename T>  // y = x / d
hipError_t vec_div(int64_t n, const T* x, const T* d, T* y, hipStream_t s);
template <typename X, typename Y>  // y = a x (converting)
hipError_t vec_scale_copy(int64_t n, double a, const X* x, Y* y, hipStream_t s);
template <typename T>
hipError_t vec_fill(int64_t n, double v, T* y, hipStream_t s);
// y = -(x + y)
hipError_t vec_negsum(int64_t n, const double* x, double* y, hipStream_t s);
hipError_t vec_min(int64_t n, const double* x, double* partial, double* out, hipStream_t s);

// ---------------------------------------------------------------------------
// grouped PCG over many linear systems with device-resident scalars
// ---------------------------------------------------------------------------
constexpr int PCG_THREADS = 256;
constexpr int64_t PCG_CHUNK = 16384;   // elements of one system per block
enum { PCG_T = 0, PCG_R = 1, PCG_P = 2, PCG_Q = 3, PCG_D = 4, PCG_NVEC = 5 };
enum { PCG_IDLE = 0, PCG_RUNNING = 1, PCG_CONVERGED = 2, PCG_INDEFINITE = 3, PCG_MAXITER = 4 };
// per-system vectors (orthonormal basis, length n): solution t, residual r,
// search direction p, q = A p, preconditioner denominators D
template <typename T>
struct PcgVecs {
  T* vec[PCG_NVEC];
};
// per-system scalars (device); tol2 = tolerance on |r|^2
struct PcgScalars {
  double rz, rr, alpha, beta, tol2, pap;   // pap: last p.Ap
  int32_t iters, maxiter, status, active;
};
// block table: block b works on elements [blk_start, blk_end) of system blk_sys
struct PcgTable {
  int nblk;
  const int32_t* blk_sys;
  const int64_t* blk_start;
  const int64_t* blk_end;
};
// per-system view of the same table: system sys_id[k] owns blocks [b0[k], b1[k])
struct PcgSysTable {
  int nsys;
  const int32_t* sys_id;
  const int32_t* b0;
  const int32_t* b1;
};
// z = r / D, p = z, rz = r.z, rr = r.r; running unless rr <= tol2
template <typename T>
hipError_t pcg_init(const PcgTable& tab, const PcgSysTable& st, const PcgVecs<T>* v, PcgScalars* sc,
                    double* part_rr, double* part_rz, hipStream_t s);
// one PCG step after q = A p: alpha, t += alpha p, r -= alpha q, z = r / D,
// convergence test, beta, p = z + beta p (systems no longer active keep t)
template <typename T>
hipError_t pcg_step(const PcgTable& tab, const PcgSysTable& st, const PcgVecs<T>* v, PcgScalars* sc,
                    double* part_a, double* part_b, hipStream_t s);

// small dense symmetric eigenproblem on one thread (n <= 16): A -> values w
// ascending, vectors R (columns, largest-magnitude entry positive)
hipError_t small_eigh(int n, const double* A, double* w, double* R, hipStream_t s);
// Correlated densities (Sec. II.D): the source contraction transposed,
//   D[idx(e, y)] += scale w chi sum_N sum_alpha W[N wstride + row ldo + alpha]
//                   G[(y galpha + goff + alpha) gcols + N]
// over the images e of every packed row of entry d (D is the coefficient
// tensor's layout, d.c_slot / d.c_stride index it; atomic adds)
hipError_t term_density(const TermDesc& d, double* D, const double* G, const double* W, int64_t wstride,
                        int nst, hipStream_t s);
// u[row] = Y[row] . X[row] over the packed rows of entry d: sum into *nsum;
// +u (virtual slot, bit k of virt_mask) or -u (closed slot) onto the
// diagonal of gdiag at orbital (nvoff +) slot value; nmo <= 2048
hipError_t row_metric(const TermDesc& d, const double* Y, const double* X, int virt_mask, int nvoff, int nmo,
                      double* gdiag, int64_t ld, double* nsum, hipStream_t s);
// transposed Fock coupling term: gf[fx][fy] += sum_{e_b, z, y} sum_a
// A[e_b][y ay + a] B[e_k(e_b, z)][y by + a] with the term's index maps
// (fx, fy from a bra slot, a summed label or y); skip_diag drops fx == fy
hipError_t fock_grad(const CoupleDesc& d, const double* A, int64_t arow, int64_t ay, const double* B,
                     int64_t brow, int64_t by, int64_t ncol, double* gf, int64_t fstride, int skip_diag,
                     hipStream_t s);
// dst (row stride ld) += src (n x n, row major) or src^T; diagonal skipped
// when skip_diag
hipError_t add_block(int n, const double* src, double* dst, int64_t ld, int transpose, int skip_diag,
                     hipStream_t s);
// Q[a][b] += sum_r X[r][a] Y[r][b] (row-major [nrow][n], row stride ld)
hipError_t outer_rows(int64_t nrow, int64_t n, int64_t ld, const double* X, const double* Y, double* Q,
                      hipStream_t s);
// in place: gf[i][i] += 2 sum_L NL[L] (closed i); d2 = gf - sum_L NL[L]
// gam[L] on the active block, gf elsewhere (n x n, device)
hipError_t density_finish(int n, int nc, int na, int nst, const double* NL, const double* gam, double* gf,
                          double* d2, hipStream_t s);
// F [nst][nst] = sym(sum_rs f[r][s] G[M][N][r][s]) (Eq. 3 in the reference space)
hipError_t xms_fref(int na, int nst, const double* f, const double* G, double* F, hipStream_t s);

}  // namespace caspt2
