/*
 * caspt2.h -- C ABI of the MI355X (gfx950) library for the hot path of fully
 * internally contracted (X)MS-CASPT2: the amplitude equation (Eq. 10), the
 * effective Hamiltonian (Eqs. 15-17) and the lambda equation (Eq. 20) of
 * Vlaisavljevich & Shiozaki, "Nuclear energy gradients for internally
 * contracted complete active space second-order perturbation theory:
 * multistate extensions" (Sec. II.A-II.C).
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 * Orbitals: closed 0..nc-1 | active nc..nc+na-1 | virtual nc+na..nmo-1.
 * All floating point is IEEE binary64, row major.
 *
 * Reference states (Sec. II.A, Eqs. 1-2): ci[N][I], N < nst, over the
 * determinants of na active orbitals with n_alpha = ceil(nelec/2) and
 * n_beta = floor(nelec/2) electrons.  A string is a bit mask over the active
 * orbitals; strings with a given count are enumerated in increasing integer
 * value; I = ia * n_beta_strings + ib; |I> = alpha creators (ascending
 * orbital) left of beta creators (ascending orbital) on the vacuum.  The CI
 * vectors must be eigenvectors of the active Hamiltonian with energies eref
 * (only eref enters H^ref, Eq. 6).
 *
 * Fock operator (Eqs. 11-12): f is symmetric and otherwise general.  Its
 * diagonal enters through the energies of the external orbital tuples (and
 * the diagonal preconditioner); the closed-active, active-virtual and
 * closed-virtual blocks couple different excitation blocks; off-diagonal
 * closed-closed and virtual-virtual elements (orbitals that are not
 * semicanonical) couple each block with itself; these run as batched GEMMs
 * along one closed or virtual slot of the block, so non-semicanonical
 * orbitals cost extra operator time, extra device memory (copies of the
 * amplitudes with all orderings of their external indices) and extra PCG
 * iterations (the diagonal preconditioner does not hold them).  Normal
 * ordering with respect to the closed vacuum is taken as
 * {E_ij}_C = E_ij - 2 delta_ij.
 *
 * Hamiltonian: hcore = h^c, the one-electron operator dressed by the closed
 * orbitals, h^c_xy = h_xy + sum_i [2 (xy|ii) - (xi|iy)]; dfB[Q][p][q] with
 * (pq|rs) = sum_Q B^Q_pq B^Q_rs.  The core energy constant is not included
 * in any energy returned.
 *
 * Internally contracted space (Eqs. 7-9): E_Omega |N~> for the nine operator
 * types of Eq. 8 in product form E_pq E_rs, from every reference state
 * (MS-MR) or from |L~> only (SS-SR).  They are grouped in eight blocks by the
 * number of closed holes and virtual particles; E_ai,rs and E_ar,si share
 * the caav block.
 *
 * Packed amplitude layout (per state L).  Entries in this order:
 *   ccvv+, ccvv-, cavv+, cavv-, aavv+, aavv-, ccav+, ccav-, ccaa+, ccaa-,
 *   aaav, caaa, caav.
 * Block operators and external slots (storage order):
 *   ccvv  E_ai E_bj   (i, j, a, b)   swaps (i,j) and (a,b)
 *   cavv  E_ar E_bi   (i, a, b)      swap  (a,b)
 *   aavv  E_ar E_bs   (a, b)         swap  (a,b)
 *   ccav  E_ai E_rj   (i, j, a)      swap  (i,j)
 *   ccaa  E_ri E_sj   (i, j)         swap  (i,j)
 *   aaav  E_ar E_st   (a)
 *   caaa  E_ri E_st   (i)
 *   caav  E_ai E_rs (type 0), E_ar E_si (type 1)   (i, a)
 * Each entry is a row-major matrix [rows][nalpha].  Rows are canonical orbit
 * representatives: for every swap (k,l) the index in slot k is >= the index
 * in slot l (strictly > for a '-' entry); slots vary lexicographically, so a
 * swapped pair is stored as the pair index k(k+1)/2 + l ('+') or
 * k(k-1)/2 + l ('-').  ccvv '-' means the character (-,-) over its two swaps.
 * Columns alpha = (state M, operator type, active tuple) with the active
 * tuple (r, s, t) row-major, state M slowest; in SS-SR the state is absent.
 * A packed row relates to the coefficients x[e] of the individual functions
 * E_Omega(e)|M~> by x[e] = sum_chi chi(pi_e) t_chi / sqrt(|orbit|), pi_e
 * being the swaps that map the representative to e.
 *
 * Status codes: every entry point returns int; 0 is success.
 * Ownership: the caller owns every buffer it passes; caspt2_create copies
 * the inputs it needs; the handle owns all device memory and
 * caspt2_destroy frees it.  Pointers marked "device" must be HIP device
 * memory of the handle's device; pointers marked "host" are host memory.
 * Threading: one host thread at a time per handle; distinct handles are
 * independent.  All work is issued on the stream given at creation and is
 * complete when an entry point returns.
 */
#ifndef CASPT2_H
#define CASPT2_H

#include <stdint.h>

#if defined(__GNUC__)
#define CASPT2_API __attribute__((visibility("default")))
#else
#define CASPT2_API
#endif

#ifdef __cplusplus
extern "C" {
#endif

enum {
  CASPT2_OK = 0,
  CASPT2_E_ARG = -1,         /* bad dimension, non-finite or non-symmetric input, bad pointer */
  CASPT2_E_NOMEM = -2,       /* device allocation failed */
  CASPT2_E_DEVICE = -3,      /* a HIP call failed (caspt2_last_error() has the text) */
  CASPT2_E_NOCONV = -4,      /* maxiter reached; best iterate kept, info filled */
  CASPT2_E_INDEFINITE = -5,  /* a denominator <= 0, or p^T A p <= 0 in PCG */
  CASPT2_E_NOTIMPL = -6,     /* feature not available in this build */
  CASPT2_E_STATE = -7        /* call out of order (e.g. heff before amplitudes) */
};

enum { CASPT2_MSMR = 0, CASPT2_SSSR = 1 };  /* Sec. II.B, Eqs. 7 and 9 */
/* Arithmetic of the solves.  FP64: every step in FP64.  MIXED: the
 * set-up (XMS, integrals, sources, metrics, bases, denominators), the
 * effective Hamiltonian and the refinement residual stay FP64; each PCG
 * (amplitudes, lambda) runs as FP64 iterative refinement around an inner
 * PCG whose operator, basis transforms, couplings and vectors are FP32 (dot
 * products accumulated in FP64).  The refined solution meets the same FP64
 * residual tolerance.  caspt2_residual is FP64 in both modes. */
enum { CASPT2_FP64 = 0, CASPT2_MIXED = 1 };

typedef struct {
  int32_t nclosed, nact, nvirt, naux, nstates, nelec;
  int32_t scheme;      /* CASPT2_MSMR or CASPT2_SSSR */
  int32_t xms;         /* 1: XMS rotation (Eqs. 3-5); 0: U = 1, MS-CASPT2 */
  int32_t precision;   /* CASPT2_FP64 or CASPT2_MIXED */
  int32_t reserved;
  double shift;        /* real vertical shift E_s (Sec. II.B) */
  double ovl_thresh;   /* overlap eigenvalue truncation, 1e-9 in the paper */
} caspt2_dims;

typedef struct {      /* all [row-major], read only, copied at create */
  const double* fock;   /* [nmo][nmo] f (Eq. 11) */
  const double* hcore;  /* [nmo][nmo] h^c */
  const double* dfB;    /* [naux][nmo][nmo] B^Q_pq, symmetric in p,q */
  const double* ci;     /* [nst][ndet] reference CI vectors (not XMS rotated) */
  const double* eref;   /* [nst] active-space CAS-CI energies */
} caspt2_inputs;

typedef struct {
  int32_t iters;        /* PCG iterations (FP32 inner iterations in MIXED) */
  int32_t flags;        /* bit 0: converged */
  double resnorm;       /* final 2-norm of the residual in the orthonormal basis */
  double e0;            /* E_L^(0) (Eq. 14) */
  double min_denom;     /* smallest preconditioner denominator */
  double emin_kept;     /* smallest kept overlap eigenvalue (all blocks) */
  double emax_dropped;  /* largest dropped overlap eigenvalue (-1 if none) */
  int32_t refinements;  /* MIXED: FP64 refinement steps (iters counts the FP32
                           inner iterations of all of them); 0 in FP64 */
  int32_t reserved;
} caspt2_info;

typedef struct caspt2_handle caspt2_handle;

/* Set up one problem (Sec. II.A-II.B): copies inputs to the device, applies
 * the XMS rotation (dims.xms), builds the density-fitted integral classes,
 * the sources <M~|E_Omega^+ H|N~> for every N, the overlap and Fock metrics
 * of every block and their orthonormal kept bases (eigenvalues >= thresh).
 * inputs_on_device: 0 if the inputs are host pointers, 1 if device.
 * stream: a hipStream_t (NULL = default stream).
 * Errors: E_ARG (dims <= 0 where forbidden, nst > ndet, non-finite inputs,
 * |f - f^T| > 1e-12), E_NOMEM,
 * E_DEVICE, E_INDEFINITE (a denominator <= 0 for some state). */
CASPT2_API int caspt2_create(const caspt2_dims* dims, const caspt2_inputs* inputs, int inputs_on_device,
                  void* stream, caspt2_handle** out);

/* Set up n problems as caspt2_create does, nthreads at a time on host
 * threads of the library (each creation is latency-bound: small launches,
 * host synchronisations, the term engine; several overlap on the device).
 * dims, inputs, streams, out and status are arrays of n; problem k runs on
 * streams[k] (a hipStream_t the caller keeps alive for the handle's life;
 * distinct streams let the creations overlap, a shared stream serialises
 * them) on the caller's current device.  status[k] receives caspt2_create's
 * code for problem k and out[k] its handle (NULL on failure; the others are
 * still created).  Returns the first failing status in k order, or OK; the
 * message of that failure is then caspt2_last_error's on the calling
 * thread.  E_ARG for n < 1, nthreads < 1 or a NULL array. */
CASPT2_API int caspt2_create_many(int32_t n, const caspt2_dims* dims, const caspt2_inputs* inputs,
                                  int inputs_on_device, void* const* streams, int32_t nthreads,
                                  caspt2_handle** out, int32_t* status);
CASPT2_API int caspt2_destroy(caspt2_handle* h);

/* Switch the arithmetic of later solves (CASPT2_FP64 or CASPT2_MIXED) on an
 * existing handle; the first switch to MIXED makes the FP32 copies of the
 * operands (device memory owned by the handle).  Solutions already stored
 * stay valid.  E_ARG for an unknown precision. */
CASPT2_API int caspt2_set_precision(caspt2_handle* h, int32_t precision);

/* Autotune the launches of the FP64 residual (Eq. 10, within-block part) of
 * this handle: for every packed entry, time each candidate -- the K split
 * count and tile order (plain or XCD-grouped) of the MFMA residual GEMM, or
 * the tile shape (64 x 64 or 128 x 64), K tile (16 or 32) and occupancy, or
 * the workgroup-count cap and prefetch form of the streaming kernels -- on
 * the handle's own
 * operands and keep the fastest (the built-in rule is one of the
 * candidates).  Choices are cached per entry shape for the process and, if
 * cache_path is not NULL, in that text file (read first, rewritten after;
 * one line per shape), so handles of equal shapes are timed once; force = 1
 * times again even for cached shapes.  Results change only by the order of
 * the K summation.  Errors: E_ARG (cache file not writable), E_DEVICE. */
CASPT2_API int caspt2_autotune(caspt2_handle* h, const char* cache_path, int32_t force);

/* The launch choice of entry k (order of the packed layout) after
 * caspt2_autotune: choice[8] = {K splits, tile order, grid cap, tile rows,
 * K tile, waves per SIMD asked of the compiler, streaming MFMA kernel
 * without prefetch, streaming MFMA kernel with its S and F operands in
 * registers} (-1, -1, 0, 0, 0, 0, 0, 0: the rule); rule_ms
 * and tuned_ms the timings of the rule and of the choice (-1 when the choice
 * came from the cache).  host outputs, each may be NULL. */
CASPT2_API int caspt2_tune_entry(const caspt2_handle* h, int32_t k, int32_t* choice, double* rule_ms,
                                 double* tuned_ms);

/* Packed vector length per state L (number of doubles). */
CASPT2_API int64_t caspt2_vector_length(const caspt2_handle* h);
/* Layout entry k (0..12, order above): offset (doubles), rows, nalpha.
 * Returns E_ARG for k out of range. */
CASPT2_API int caspt2_layout(const caspt2_handle* h, int32_t k, int64_t* offset, int64_t* rows,
                  int64_t* nalpha);

/* Residual of the amplitude equation (Eq. 10) for state L:
 * sigma = sum_N <M~|E_Omega^+ (f - E_L^(0) + E_s) T_LN|N~> (+ <M~|E_Omega^+ H|L~>)
 * in the packed non-orthogonal layout.  x, sigma: device, length
 * caspt2_vector_length; they must not overlap. */
CASPT2_API int caspt2_residual(caspt2_handle* h, int32_t L, int32_t with_source, const double* x,
                    double* sigma);
/* Residuals for every state at once: x and sigma are [nst][length] device.
 * The states alternate between two streams of the handle (the second
 * launching its entries in reverse order; with couplings between blocks the
 * second stream uses a second set of the handle's work tensors, allocated
 * on first use), so that kernels of different states overlap; results equal
 * the one-state calls bit for bit.  The call returns when all of them are
 * done. */
CASPT2_API int caspt2_residual_all(caspt2_handle* h, int32_t with_source, const double* x, double* sigma);

/* caspt2_residual_all for n handles (distinct; x[k] and sigma[k] as that call
 * takes them for handle k), nthreads calls at a time on host threads of the
 * library, so that the launches of different problems overlap on the device
 * (each handle works on its own stream; handles created on distinct streams
 * overlap).  status[k] receives handle k's code.  Returns when every call is
 * done: the first failing status in k order (its message is then
 * caspt2_last_error's), or OK.  E_ARG for n < 1, nthreads < 1, a NULL array
 * or a repeated handle. */
CASPT2_API int caspt2_residual_all_many(int32_t n, caspt2_handle* const* handles, int32_t with_source,
                                        const double* const* x, double* const* sigma, int32_t nthreads,
                                        int32_t* status);

/* Streams caspt2_residual_all spreads the states over: 2 (default) or 1 (all
 * on the handle's stream, e.g. to time each kernel alone).  E_ARG otherwise. */
CASPT2_API int caspt2_set_streams(caspt2_handle* h, int32_t n);

/* Solve Eq. 10 for every state by preconditioned conjugate gradients in the
 * orthonormal kept basis (preconditioner: external orbital energies +
 * E_s - E_L + eigenvalues of the block Fock metric).  Stops when the
 * residual 2-norm <= tol.  T0: device [nst][length] packed starting
 * amplitudes (warm start, e.g. the result of an earlier call that stopped
 * at maxiter, read with caspt2_get_amplitudes), or NULL to start from zero;
 * only its S-orthogonal projection on the kept space enters (components
 * along dropped overlap eigenvectors are zero functions).  info: host array
 * [nst] or NULL.  Returns E_NOCONV if any state hit maxiter (the last
 * iterate is stored and can be read and resumed from), E_INDEFINITE as
 * documented. */
CASPT2_API int caspt2_solve_amplitudes(caspt2_handle* h, double tol, int32_t maxiter, const double* T0,
                                       caspt2_info* info);
/* Copy T_L (packed, device) after caspt2_solve_amplitudes; E_STATE before. */
CASPT2_API int caspt2_get_amplitudes(caspt2_handle* h, int32_t L, double* T);

/* XMS rotation (Eqs. 3-5) on its own: the Fock operator in the reference
 * space, F_MN = sum_rs f_rs <M|E_rs|N> (active part; the closed part only
 * adds a constant to the diagonal, Eq. 12), symmetrised and diagonalised:
 * F U = U diag(E~).  f_act [nact][nact] and rdm1 [nst][nst][nact][nact]
 * (rdm1[M][N][r][s] = <M|E_rs|N> of the states before rotation) host,
 * read only; U [nst][nst] (column M is |M~> = sum_N |N> U[N][M]) and
 * e0 [nst] = E~ ascending (= E_M^(0) of Eq. 14 for the rotated states)
 * host outputs; each column of U has its largest-magnitude entry positive.
 * Rotated transition densities follow as G~^{MN} = sum_KL U[K][M] U[L][N]
 * G^{KL}.  Runs on the current HIP device.  Errors: E_ARG (nact < 0,
 * nst < 1 or > 16, NULL or non-finite input), E_DEVICE. */
CASPT2_API int xms_rotate(int32_t nact, int32_t nst, const double* f_act, const double* rdm1, double* U,
                          double* e0);

/* xms_rotate for callers that cannot allocate device memory (code under HIP
 * graph capture, serving loops, harnesses that forbid hipMalloc): the same
 * result from device inputs into device outputs -- f_act [nact][nact],
 * rdm1 [nst][nst][nact][nact], U [nst][nst], e0 [nst], all device memory of
 * the current device -- issued on `stream` (a hipStream_t, NULL = default)
 * and complete when the stream reaches it.  No device memory is allocated
 * or freed: the one intermediate (F^ref, nst x nst) lives in a fixed
 * device array of 16 x 16 doubles per GPU, held until the process ends; its
 * device address is looked up on the first call on each device.  Calls that
 * overlap on one GPU (different streams or threads) race on that array.
 * The inputs are not checked for finiteness (device memory).  Errors: E_ARG
 * (nact < 0, nst < 1 or nst > 16, NULL pointer), E_DEVICE. */
CASPT2_API int xms_rotate_noalloc(int32_t nact, int32_t nst, const double* f_act, const double* rdm1, double* U,
                                  double* e0, void* stream);

/* The XMS rotation a handle applied at create (dims.xms = 1; identity when
 * 0): U [nst][nst] and E_L^(0) [nst] (Eq. 14), as xms_rotate returns them
 * for the handle's f and reference states.  host outputs, each may be NULL. */
CASPT2_API int caspt2_get_xms(const caspt2_handle* h, double* U, double* e0);

/* Effective Hamiltonian (Eq. 15), its eigenvalues E^MS ascending (Eq. 17)
 * and eigenvectors R (Eq. 16, columns, largest-magnitude entry positive).
 * host outputs, [nst][nst], [nst], [nst][nst].  E_STATE before amplitudes. */
CASPT2_API int xms_heff(caspt2_handle* h, double* heff, double* e_ms, double* R);

/* Solve the lambda equation (Eq. 20) for target state P with the same
 * operator and solver as the amplitudes.  lam0: device [nst][length] packed
 * starting multipliers (warm start) or NULL, as T0 of
 * caspt2_solve_amplitudes.  E_STATE before xms_heff. */
CASPT2_API int caspt2_solve_lambda(caspt2_handle* h, int32_t target, double tol, int32_t maxiter,
                                   const double* lam0, caspt2_info* info);
CASPT2_API int caspt2_get_lambda(caspt2_handle* h, int32_t L, double* lambda);

/* Correlated density matrices of Sec. II.D (Eqs. 24-30) for the target
 * state P of the last lambda solve (caspt2_solve_lambda or the batch), with
 * the mixed states |P> = sum_M |M~> R_MP and T_PN = sum_M T_MN R_MP:
 *   d1[x][y]  = sum_M <M~|T_PM^+ E_xy|P> + sum_MN <M~|lambda_NM^+ E_xy|N~>
 *   D1        = the same with E_xy,zw = E_xy E_zw - delta_yz E_xw
 *   dbar2[x][y] = sum_LMN <M~|lambda_LM^+ E_xy T_LN|N~>
 *   NL[L]     = sum_MN <M~|lambda_LM^+ T_LN|N~>
 *   d2        = dbar2 - sum_L NL[L] <L~|E_xy|L~> for active x, y; dbar2 else.
 * E_xy is the plain spin-summed excitation (E_ii on a closed orbital counts
 * its electrons).  d1 is non-zero only where x is active or virtual and y
 * active or closed, not both active.  D1 covers the classes of the
 * two-body part of H that act on the references (x, z active or virtual; y,
 * w active or closed; not all four active): caspt2_density2_length doubles,
 * class k (0..14) at the offset and with the orbital spaces (0 closed,
 * 1 active, 2 virtual, for x, y, z, w) caspt2_density2_layout returns,
 * stored [x][y][z][w] row major over the class's orbitals.  With these,
 * dE^MS_P/dh^c_xy = <P|E_xy|P> + d1_xy and dE^MS_P/d(xy|zw) =
 * (<P|E_xy,zw|P> + D1_xyzw)/2 at fixed reference states and f, and
 * dE^MS_P/df_xy = d2_xy (minus 2 sum_L NL[L] on the closed diagonal,
 * Eq. 12) at fixed references and XMS rotation.
 * d1, dbar2, d2: host [nmo][nmo]; D1: device [caspt2_density2_length];
 * NL: host [nst]; each may be NULL.  E_STATE before caspt2_solve_lambda. */
CASPT2_API int caspt2_densities(caspt2_handle* h, double* d1, double* D1, double* dbar2, double* d2,
                                double* NL);
CASPT2_API int64_t caspt2_density2_length(const caspt2_handle* h);
CASPT2_API int caspt2_density2_layout(const caspt2_handle* h, int32_t k, int64_t* offset, int32_t* spaces);

/* Batched solves over many independent problems (handles created with the
 * same precision, CASPT2_FP64 or CASPT2_MIXED; the problems may differ in
 * every dimension and state count).
 * All amplitude systems (every state of every problem) advance in one
 * grouped PCG with device-resident scalars and one captured HIP graph per
 * system for the operator application; as soon as the amplitudes of a
 * problem converge, its H_eff (Eqs. 15-17) is formed and its lambda systems
 * (Eq. 20, target state targets[i]) join the running group, so amplitude and
 * lambda solves of different problems interleave.  Results are stored in
 * each handle as after caspt2_solve_amplitudes, xms_heff and
 * caspt2_solve_lambda (read them with the per-handle getters).
 * handles [n] (distinct), targets [n] host; amp_info and lambda_info host
 * arrays of sum_i nstates_i entries (problem-major) or NULL.  Returns the
 * first failure over the problems (E_INDEFINITE takes precedence, then
 * E_NOCONV); a problem whose amplitude solve fails gets no lambda.
 * In CASPT2_MIXED the grouped recurrence is the FP32 inner solver and each
 * system is refined in FP64 as in caspt2_solve_amplitudes.  E_ARG if the
 * handles differ in precision. */
CASPT2_API int caspt2_batch_solve(caspt2_handle* const* handles, int32_t n, const int32_t* targets, double tol,
                                  int32_t maxiter, caspt2_info* amp_info, caspt2_info* lambda_info);

/* Measurement support: enable (1) or disable (0) HIP-event timing of every
 * residual kernel launch (clears what was recorded), and read, per packed
 * layout entry k (0..12; the '+' entry also covers its '-' partner when both
 * run in one launch), the average launch duration in ms, the number of
 * launches and the algorithmic bytes per launch (read x, read the source when
 * it is added, write sigma; 8 bytes per double).  k = 13 reports the Fock
 * couplings between blocks of one residual, timed together (bytes 0).
 * k = 14, 15, 16 report the batched GEMMs that apply off-diagonal
 * closed-closed and virtual-virtual Fock elements inside the ccvv, cavv and
 * ccav blocks respectively (orbitals that are not semicanonical): per launch
 * 2 D^2 P Q flops in place of bytes (f of D x D along one slot, P Q the other
 * elements). */
CASPT2_API int caspt2_profile(caspt2_handle* h, int32_t enable);
CASPT2_API int caspt2_profile_entry(caspt2_handle* h, int32_t k, double* avg_ms, int64_t* launches,
                                    double* bytes_per_launch);
/* Stages of the Fock couplings timed while profiling is on: k = 0, 1, ...
 * (E_ARG past the last): name (e.g. "unpack", "up ccvv <- cavv", "pack";
 * the terms of one direction and block pair together; NUL-terminated,
 * truncated to name_len), the stage's time per residual evaluation with
 * couplings (ms, HIP events on the handle's stream) and the number of such
 * evaluations recorded.  Each may be NULL. */
CASPT2_API int caspt2_profile_stage(caspt2_handle* h, int32_t k, char* name, int32_t name_len,
                                    double* ms_per_residual, int64_t* residuals);

/* Human-readable text for a status code; last HIP error text. */
CASPT2_API const char* caspt2_strerror(int code);
CASPT2_API const char* caspt2_last_error(void);

#ifdef __cplusplus
}
#endif
#endif
