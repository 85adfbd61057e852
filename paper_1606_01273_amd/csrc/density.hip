// Kernels of the correlated density matrices (Sec. II.D): every density
// element is the derivative of a matrix element the amplitude equation
// already uses with respect to its coefficient (an integral or an element of
// f), so these kernels run the source and Fock-coupling contractions
// transposed -- the amplitudes and multipliers take the place of the
// integrals or of f and the result lands in the coefficient's position.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "device_common.hpp"
#include "kernels.hpp"

namespace caspt2 {

static inline int64_t cdiv(int64_t a, int64_t b) { return (a + b - 1) / b; }

// ---------------------------------------------------------------------------
// transposed source term (one-body or two-body part of H):
//   D[idx(e, y)] += scale * w * chi(pi_e) * sum_N sum_alpha W_N[row][alpha]
//                   * G[(y * galpha + goff + alpha) * gcols + N]
// over every image e of each packed row's orbit (the images, weights and
// characters of the source kernel).  A thread takes one (row, y); the images
// of one row land in distinct positions, rows of different threads may
// share one, so the adds are atomic.
// ---------------------------------------------------------------------------
__global__ void k_term_density(TermDesc d, double* __restrict__ D, const double* __restrict__ G,
                               const double* __restrict__ W, int64_t wstride, int nst) {
  int64_t ny = 1;
  for (int k = 0; k < d.nopact; ++k) ny *= d.na;
  const int64_t total = d.nrow * ny;
  for (int64_t g = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; g < total;
       g += (int64_t)gridDim.x * blockDim.x) {
    const int64_t row = g / ny;
    const int64_t y = g % ny;
    double base = 0.0;
    for (int N = 0; N < nst; ++N) {
      const double* wr = W + N * wstride + row * d.ldo;
      const double* gy = G + (y * d.galpha + d.goff) * d.gcols + N;
      for (int64_t al = 0; al < d.nalpha; ++al) base += wr[al] * gy[al * d.gcols];
    }
    if (base == 0.0) continue;
    int yi[3] = {0, 0, 0};
    int64_t yr = y;
    for (int k = d.nopact - 1; k >= 0; --k) {
      yi[k] = (int)(yr % d.na);
      yr /= d.na;
    }
    int e0[4] = {0, 0, 0, 0};
    decode_orbit(d, row, e0);
    int ndistinct = 0;
    for (int s = 0; s < d.nswap; ++s)
      if (e0[d.swap_k[s]] != e0[d.swap_l[s]]) ++ndistinct;
    const double w = d.mode_avg ? 1.0 : 1.0 / sqrt((double)(1 << ndistinct));
    const int nbits = d.mode_avg ? 1 : (1 << d.nswap);
    for (int bits = 0; bits < nbits; ++bits) {
      int e[4] = {e0[0], e0[1], e0[2], e0[3]};
      double sg = 1.0;
      bool dup = false;
      for (int s = 0; s < d.nswap; ++s)
        if ((bits >> s) & 1) {
          if (e0[d.swap_k[s]] == e0[d.swap_l[s]]) dup = true;
          const int t = e[d.swap_k[s]];
          e[d.swap_k[s]] = e[d.swap_l[s]];
          e[d.swap_l[s]] = t;
          sg *= d.chi[s];
        }
      if (dup) continue;
      int64_t off = 0;
      for (int a = 0; a < d.ncax; ++a) {
        const int src = d.c_slot[a];
        const int v = src >= 0 ? e[src] : yi[-1 - src];
        off += (int64_t)v * d.c_stride[a];
      }
      unsafeAtomicAdd(D + off, d.scale * w * sg * base);
    }
  }
}

hipError_t term_density(const TermDesc& d, double* D, const double* G, const double* W, int64_t wstride,
                        int nst, hipStream_t s) {
  int64_t ny = 1;
  for (int k = 0; k < d.nopact; ++k) ny *= d.na;
  const int64_t total = d.nrow * ny;
  if (total == 0) return hipSuccess;
  unsigned grid = (unsigned)std::min<int64_t>(cdiv(total, 256), 65536);
  hipLaunchKernelGGL(k_term_density, dim3(grid), dim3(256), 0, s, d, D, G, W, wstride, nst);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// metric products of packed rows: u[row] = Y[row] . X[row] (Y = lambda S,
// X = T, rows of nalpha values), summed into *nsum, and u[row] times the
// occupation change of each external orbital of the row's representative
// added to the diagonal of gdiag (row stride ld): +u for a virtual slot
// (one electron more), -u for a closed slot (one fewer).  Sums go through
// LDS (one slot per orbital) and are flushed once per workgroup.
// ---------------------------------------------------------------------------
constexpr int ROWDOT_LDS = 2048;   // orbitals an LDS accumulator holds
__global__ __launch_bounds__(256) void k_row_metric(TermDesc d, const double* __restrict__ Y,
                                                    const double* __restrict__ X, int virt_mask, int nvo,
                                                    int nmo, double* __restrict__ gdiag, int64_t ld,
                                                    double* __restrict__ nsum) {
  __shared__ double acc[ROWDOT_LDS];
  __shared__ double tot[256];
  for (int k = threadIdx.x; k < nmo; k += blockDim.x) acc[k] = 0.0;
  __syncthreads();
  double mine = 0.0;
  for (int64_t row = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; row < d.nrow;
       row += (int64_t)gridDim.x * blockDim.x) {
    const double* y = Y + row * d.ldo;
    const double* x = X + row * d.ldo;
    double u = 0.0;
    for (int64_t a = 0; a < d.nalpha; ++a) u += y[a] * x[a];
    mine += u;
    int e[4] = {0, 0, 0, 0};
    decode_orbit(d, row, e);
    for (int k = 0; k < d.nslot; ++k) {
      const bool vir = (virt_mask >> k) & 1;
      const int orb = vir ? nvo + e[k] : e[k];
      atomicAdd(&acc[orb], vir ? u : -u);
    }
  }
  tot[threadIdx.x] = mine;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (threadIdx.x < w) tot[threadIdx.x] += tot[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) unsafeAtomicAdd(nsum, tot[0]);
  for (int k = threadIdx.x; k < nmo; k += blockDim.x)
    if (acc[k] != 0.0) unsafeAtomicAdd(gdiag + (int64_t)k * ld + k, acc[k]);
}

hipError_t row_metric(const TermDesc& d, const double* Y, const double* X, int virt_mask, int nvoff, int nmo,
                      double* gdiag, int64_t ld, double* nsum, hipStream_t s) {
  if (d.nrow == 0 || d.nalpha == 0) return hipSuccess;
  if (nmo > ROWDOT_LDS) return hipErrorInvalidValue;
  const unsigned grid = (unsigned)std::min<int64_t>(cdiv(d.nrow, 256), 1024);
  hipLaunchKernelGGL(k_row_metric, dim3(grid), dim3(256), 0, s, d, Y, X, virt_mask, nvoff, nmo, gdiag, ld,
                     nsum);
  return hipGetLastError();
}

// Q[a][b] += sum_r X[r][a] Y[r][b] over rows r of two row-major matrices
// [nrow][n] (row stride ld): one thread per (a, b) and chunk of rows
// (neighbouring threads share rows), chunks meeting in atomic adds
__global__ __launch_bounds__(256) void k_outer_rows(int64_t nrow, int64_t n, int64_t ld, int64_t chunk,
                                                    const double* __restrict__ X, const double* __restrict__ Y,
                                                    double* __restrict__ Q) {
  const int64_t nn = n * n;
  const int64_t nchunk = (nrow + chunk - 1) / chunk;
  for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < nn * nchunk;
       t += (int64_t)gridDim.x * blockDim.x) {
    const int64_t pr = t % nn, c = t / nn;
    const int64_t a = pr / n, b = pr % n;
    const int64_t r0 = c * chunk, r1 = r0 + chunk < nrow ? r0 + chunk : nrow;
    double acc = 0.0;
    for (int64_t r = r0; r < r1; ++r) acc += X[r * ld + a] * Y[r * ld + b];
    if (acc != 0.0) unsafeAtomicAdd(Q + pr, acc);
  }
}

hipError_t outer_rows(int64_t nrow, int64_t n, int64_t ld, const double* X, const double* Y, double* Q,
                      hipStream_t s) {
  if (nrow == 0 || n == 0) return hipSuccess;
  const int64_t nn = n * n;
  int64_t nchunk = cdiv((int64_t)1 << 20, nn);
  nchunk = std::max<int64_t>(1, std::min<int64_t>(nchunk, cdiv(nrow, 32)));
  const int64_t chunk = cdiv(nrow, nchunk);
  nchunk = cdiv(nrow, chunk);
  const unsigned grid = (unsigned)std::min<int64_t>(cdiv(nn * nchunk, 256), 65536);
  hipLaunchKernelGGL(k_outer_rows, dim3(grid), dim3(256), 0, s, nrow, n, ld, chunk, X, Y, Q);
  return hipGetLastError();
}

// gf (n x n, the reduced one-particle density of the Fock terms) finished in
// place and d2 formed (both n x n, orbitals closed | active | virtual):
// gf[i][i] += 2 sum_L N_L for closed i (E_ii counts the two electrons of a
// closed orbital); d2 = gf - sum_L N_L gamma_L on the active block
// (gamma [nst][na][na] = <L~|E_rs|L~>), d2 = gf elsewhere
__global__ void k_density_finish(int n, int nc, int na, int nst, const double* __restrict__ NL,
                                 const double* __restrict__ gam, double* __restrict__ gf,
                                 double* __restrict__ d2) {
  const int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (t >= (int64_t)n * n) return;
  const int x = (int)(t / n), y = (int)(t % n);
  double ntot = 0.0;
  for (int L = 0; L < nst; ++L) ntot += NL[L];
  double g = gf[t];
  if (x == y && x < nc) g += 2.0 * ntot;
  gf[t] = g;
  if (x >= nc && x < nc + na && y >= nc && y < nc + na)
    for (int L = 0; L < nst; ++L) g -= NL[L] * gam[((int64_t)L * na + (x - nc)) * na + (y - nc)];
  d2[t] = g;
}

hipError_t density_finish(int n, int nc, int na, int nst, const double* NL, const double* gam, double* gf,
                          double* d2, hipStream_t s) {
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(k_density_finish, dim3((unsigned)cdiv((int64_t)n * n, 256)), dim3(256), 0, s, n, nc, na,
                     nst, NL, gam, gf, d2);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// transposed Fock coupling: for the term's index maps (bra slots, summed
// labels z, active label y of the Fock element)
//   gf[fx][fy] += sum over (e_b, z, y) with f(e_b, z, y) = f[fx][fy] of
//                 sum_a A[e_b][y * ay + a] B[e_k(e_b, z)][y * by + a]
// Up terms: A = lambda (all orderings, ay = 0), B = W = x G (by = ncol);
// down terms: A = lambda G (ay = ncol), B = x (by = 0).
// Variables: the bra slots (0..3), the summed labels (4, 5), y (6); fx and
// fy each come from one of them.  A thread owns one (fx, fy) pair and one
// chunk of the other variables' range (no race inside a thread; chunks of
// one pair meet in an atomic add).  skip_diag: leave fx == fy out (the
// diagonal of a within-space block is the row energies' derivative).
// ---------------------------------------------------------------------------
struct GradPlan {
  int dim[7];        // range of every variable (1 if absent)
  int xvar, yvar;    // variable feeding fx, fy
  int loopvar[7];    // the other variables with range > 1, slowest first
  int nloop;
  int64_t da[7], db[7];   // offset of A and of B per unit step of each variable
  int64_t loop_total;
  int64_t chunk, nchunk;
};

// A thread owns one (fx, fy) and a chunk [lo, hi) of the other variables'
// linear range: the start is decoded once, then the offsets into A and B
// advance by the variables' deltas like an odometer (no division per step).
__global__ __launch_bounds__(256) void k_fock_grad(GradPlan gp, const double* __restrict__ A,
                                                   const double* __restrict__ B, int64_t ncol,
                                                   double* __restrict__ gf, int64_t fstride, int skip_diag) {
  const int64_t npair = (int64_t)gp.dim[gp.xvar] * gp.dim[gp.yvar];
  const int64_t total = npair * gp.nchunk;
  for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < total;
       t += (int64_t)gridDim.x * blockDim.x) {
    const int64_t pairi = t / gp.nchunk, c = t % gp.nchunk;
    const int fx = (int)(pairi / gp.dim[gp.yvar]), fy = (int)(pairi % gp.dim[gp.yvar]);
    if (skip_diag && fx == fy) continue;
    const int64_t lo = c * gp.chunk;
    const int64_t hi = lo + gp.chunk < gp.loop_total ? lo + gp.chunk : gp.loop_total;
    if (lo >= hi) continue;
    int64_t oa = fx * gp.da[gp.xvar] + fy * gp.da[gp.yvar];
    int64_t ob = fx * gp.db[gp.xvar] + fy * gp.db[gp.yvar];
    int cnt[7] = {0, 0, 0, 0, 0, 0, 0};
    {
      int64_t r = lo;
      for (int k = gp.nloop - 1; k >= 0; --k) {
        const int var = gp.loopvar[k];
        const int v = (int)(r % gp.dim[var]);
        r /= gp.dim[var];
        cnt[k] = v;
        oa += v * gp.da[var];
        ob += v * gp.db[var];
      }
    }
    double acc = 0.0;
    for (int64_t q = lo; q < hi; ++q) {
      const double* pa = A + oa;
      const double* pb = B + ob;
      for (int64_t a = 0; a < ncol; ++a) acc += pa[a] * pb[a];
      // next value of the loop variables (the last one fastest)
      for (int k = gp.nloop - 1; k >= 0; --k) {
        const int var = gp.loopvar[k];
        if (++cnt[k] < gp.dim[var]) {
          oa += gp.da[var];
          ob += gp.db[var];
          break;
        }
        cnt[k] = 0;
        oa -= (int64_t)(gp.dim[var] - 1) * gp.da[var];
        ob -= (int64_t)(gp.dim[var] - 1) * gp.db[var];
      }
    }
    if (acc != 0.0) unsafeAtomicAdd(gf + (int64_t)fx * fstride + fy, acc);
  }
}

// dst (n x n block, row stride ld) += src (n x n) or its transpose, the
// diagonal left out when skip_diag
__global__ void k_add_block(int n, const double* __restrict__ src, double* __restrict__ dst, int64_t ld,
                            int transpose, int skip_diag) {
  const int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (t >= (int64_t)n * n) return;
  const int r = (int)(t / n), c = (int)(t % n);
  if (skip_diag && r == c) return;
  dst[(int64_t)r * ld + c] += transpose ? src[(int64_t)c * n + r] : src[t];
}

hipError_t add_block(int n, const double* src, double* dst, int64_t ld, int transpose, int skip_diag,
                     hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_add_block, dim3((unsigned)cdiv((int64_t)n * n, 256)), dim3(256), 0, s, n, src, dst, ld,
                     transpose, skip_diag);
  return hipGetLastError();
}

// the variable (0..3 bra slot, 4..5 summed label, 6 active y) an index
// source of a coupling descriptor names
static inline int src_var(int src) {
  if (src >= 0) return src;
  if (src == -10) return 6;
  return 4 + (-1 - src);
}

hipError_t fock_grad(const CoupleDesc& d, const double* A, int64_t arow, int64_t ay, const double* B,
                     int64_t brow, int64_t by, int64_t ncol, double* gf, int64_t fstride, int skip_diag,
                     hipStream_t s) {
  GradPlan gp{};
  for (int k = 0; k < 7; ++k) gp.dim[k] = 1;
  for (int k = 0; k < d.bra.nslot; ++k) gp.dim[k] = d.bra.slot_dim[k];
  for (int k = 0; k < d.nsum; ++k) gp.dim[4 + k] = d.sum_dim[k];
  gp.dim[6] = d.ny;
  for (int k = 0; k < 7; ++k)
    if (gp.dim[k] == 0) return hipSuccess;
  gp.xvar = src_var(d.fx_src);
  gp.yvar = src_var(d.fy_src);
  if (gp.xvar == gp.yvar) return hipErrorInvalidValue;   // both indices of f from one label
  // row strides of the all-orderings tensors
  int64_t bst[4] = {0, 0, 0, 0}, kst[4] = {0, 0, 0, 0}, st = 1;
  for (int k = d.bra.nslot - 1; k >= 0; --k) {
    bst[k] = st;
    st *= d.bra.slot_dim[k];
  }
  st = 1;
  for (int l = d.ket.nslot - 1; l >= 0; --l) {
    kst[l] = st;
    st *= d.ket.slot_dim[l];
  }
  for (int k = 0; k < 7; ++k) gp.da[k] = gp.db[k] = 0;
  for (int k = 0; k < d.bra.nslot; ++k) gp.da[k] = bst[k] * arow;
  for (int l = 0; l < d.ket.nslot; ++l) {
    const int src = d.ket_src[l];
    const int var = src >= 0 ? src : 4 + (-1 - src);
    gp.db[var] += kst[l] * brow;
  }
  gp.da[6] += ay;
  gp.db[6] += by;
  gp.nloop = 0;
  gp.loop_total = 1;
  for (int k = 0; k < 7; ++k)
    if (k != gp.xvar && k != gp.yvar && gp.dim[k] > 1) {
      gp.loopvar[gp.nloop++] = k;
      gp.loop_total *= gp.dim[k];
    }
  const int64_t npair = (int64_t)gp.dim[gp.xvar] * gp.dim[gp.yvar];
  // about 2^20 threads, each with a chunk of at least 64 loop iterations
  int64_t nchunk = cdiv((int64_t)1 << 20, npair);
  const int64_t maxchunks = cdiv(gp.loop_total, 64);
  if (nchunk > maxchunks) nchunk = maxchunks;
  if (nchunk < 1) nchunk = 1;
  gp.nchunk = nchunk;
  gp.chunk = cdiv(gp.loop_total, nchunk);
  const int64_t total = npair * nchunk;
  const unsigned grid = (unsigned)std::min<int64_t>(cdiv(total, 256), 65536);
  hipLaunchKernelGGL(k_fock_grad, dim3(grid), dim3(256), 0, s, gp, A, B, ncol, gf, fstride, skip_diag);
  return hipGetLastError();
}

}  // namespace caspt2
