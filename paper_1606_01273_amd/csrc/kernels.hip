// HIP kernels for gfx950 (CDNA4): operator application on CI vectors, FP64
// MFMA GEMMs, packed-term contractions, Jacobi eigensolver, vector ops.
#include "kernels.hpp"
#include "device_common.hpp"

#include <algorithm>
#include <cmath>
#include <cstring>
#include <vector>

namespace caspt2 {

typedef double d4 __attribute__((ext_vector_type(4)));

static inline unsigned cdiv(int64_t a, int64_t b) { return (unsigned)((a + b - 1) / b); }

// grid of tiles: the dimension with more tiles on x; false when neither
// orientation fits the 65535 limit of grid y and z
static inline bool tile_grid(int64_t M, int64_t N, int batch, int tm, int tn, dim3* grid, int* m_on_x) {
  const int64_t tmn = (M + tm - 1) / tm, tnn = (N + tn - 1) / tn;
  *m_on_x = tmn >= tnn ? 1 : 0;
  const int64_t gx = *m_on_x ? tmn : tnn, gy = *m_on_x ? tnn : tmn;
  if (gy > 65535 || batch > 65535 || gx > 0x7fffffff) return false;
  *grid = dim3((unsigned)gx, (unsigned)gy, (unsigned)batch);
  return true;
}

// ---------------------------------------------------------------------------
// operator application: Y[r][lead][t] = sign[r][t] * X[lead][src[r][t]]
// ---------------------------------------------------------------------------
__global__ void k_gather_apply(const double* __restrict__ X, int64_t nlead, int64_t dim_from,
                               const int32_t* __restrict__ src, const double* __restrict__ sign,
                               int na, int64_t dim_to, double* __restrict__ Y) {
  const int64_t total = (int64_t)na * nlead * dim_to;
  for (int64_t g = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; g < total;
       g += (int64_t)gridDim.x * blockDim.x) {
    const int64_t t = g % dim_to;
    const int64_t rl = g / dim_to;
    const int64_t lead = rl % nlead;
    const int64_t r = rl / nlead;
    const int32_t s = src[r * dim_to + t];
    Y[g] = s >= 0 ? sign[r * dim_to + t] * X[lead * dim_from + s] : 0.0;
  }
}

hipError_t launch_gather_apply(const double* X, int64_t nlead, int64_t dim_from,
                               const int32_t* src, const double* sign, int na, int64_t dim_to,
                               double* Y, hipStream_t s) {
  const int64_t total = (int64_t)na * nlead * dim_to;
  if (total == 0) return hipSuccess;
  unsigned grid = cdiv(total, 256);
  if (grid > 65536) grid = 65536;
  hipLaunchKernelGGL(k_gather_apply, dim3(grid), dim3(256), 0, s, X, nlead, dim_from, src, sign,
                     na, dim_to, Y);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// FP64 GEMM on MFMA (v_mfma_f64_16x16x4f64)
//   block tile 64x64, 4 waves of 32x32, K step 16 through LDS.
//   Operand layout of the 16x16x4 instruction (per lane l):
//     A[i][k]: i = l % 16, k = l / 16;  B[k][j]: j = l % 16, k = l / 16;
//     D[i][j]: j = l % 16, i = l / 16 + 4 * v, v = 0..3 (checked on gfx950).
// ---------------------------------------------------------------------------
constexpr int BM = 64, BN = 64, BK = BK_RESIDUAL;

// MT: 16-row MFMA blocks per wave along M; the workgroup tile is (32 MT) x
// 64 (MT = 2: 64 x 64, MT = 4: 128 x 64 -- more flops per byte staged, at
// twice the accumulator registers).  KB: K tile (16 or 32; a longer tile
// gives the register prefetch of the next tile more time to arrive).
// SPLIT: blockIdx.z selects a K range of kchunk (a multiple of KB); the raw
// partial products go to C as [split][M][N] (dual: the X S and X F products
// as [split][2][M][N]) for a separate epilogue.
template <bool B_NK, bool DUAL, bool SPLIT = false, int MT = 2, int KB = BK, int WPE = 1>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(WPE))) void k_gemm_f64(int64_t M, int64_t N, int64_t K, double alpha,
                                                  const double* __restrict__ A, int64_t lda,
                                                  int64_t sA, const double* __restrict__ B,
                                                  int64_t ldb, int64_t sB,
                                                  const double* __restrict__ B2, double beta,
                                                  double* __restrict__ C, int64_t ldc, int64_t sC,
                                                  const double* __restrict__ dvec, double dshift,
                                                  const double* __restrict__ V, int64_t ldv,
                                                  int order, int64_t kchunk) {
  constexpr int TM = 32 * MT;          // tile rows
  constexpr int TPR = 256 / TM;        // threads per A row of a K tile
  constexpr int UA = KB / TPR;         // consecutive k per thread in the A tile
  constexpr int LDP = KB + 1;          // LDS row pitch (odd: no bank conflicts on k)
  // B as [K][N]: KT threads per k row, UB consecutive n each; B as [N][K]:
  // four threads per n row, UN consecutive k each
  constexpr int KT = 256 / KB, UB = BN * KB / 256, UN = KB / 4;
  static_assert(TPR * TM == 256 && UA * TPR == KB, "A tile shares");
  static_assert(BN == 64 && KT * KB == 256 && UB * 256 == BN * KB, "B tile shares");
  // two LDS buffers where they fit in 64 KB: the next K tile is stored into
  // the other buffer while this one feeds the MFMAs, one barrier per tile
  constexpr bool DBUF = 2 * (TM + BN * (DUAL ? 2 : 1)) * LDP * 8 <= 64 * 1024;
  constexpr int NBUF = DBUF ? 2 : 1;
  __shared__ double As[NBUF][TM][LDP];
  __shared__ double Bs[NBUF][BN][LDP];
  __shared__ double B2s[NBUF][DUAL ? BN : 1][LDP];
  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = tid >> 6;
  const int wm = wave >> 1, wn = wave & 1;
  // tile of this workgroup.  order 0/1: n or m tile index on grid x (the
  // longer tile dimension runs on x; y and z are limited to 65535).  order 2:
  // XCD-grouped -- workgroups are dispatched round-robin over the 8 XCDs, so
  // linear id g runs on XCD g % 8; each XCD takes a contiguous range of the
  // tiles (n fastest), and the tiles of one row band that share their A rows
  // run on one XCD at about the same time (one L2)
  // order 3: the same with m fastest (the m tiles that share one B tile run
  // back to back on one XCD: for batched products with few m tiles)
  int64_t bz, tmi, tni;
  if (order >= 2) {
    const int64_t gx = gridDim.x, gy = gridDim.y;
    const int64_t nwg = gx * gy * (int64_t)gridDim.z;
    const int64_t g = ((int64_t)blockIdx.z * gy + blockIdx.y) * gx + blockIdx.x;
    const int64_t x = g & 7, j = g >> 3, per = nwg >> 3, rem = nwg & 7;
    const int64_t t = x * per + (x < rem ? x : rem) + j;
    const int64_t tnn = (N + BN - 1) / BN, tmn = (M + TM - 1) / TM;
    bz = t / (tmn * tnn);
    const int64_t r = t - bz * tmn * tnn;
    if (order == 2) {
      tmi = r / tnn;
      tni = r - tmi * tnn;
    } else {
      tni = r / tmn;
      tmi = r - tni * tmn;
    }
  } else {
    bz = blockIdx.z;
    tmi = order ? blockIdx.x : blockIdx.y;
    tni = order ? blockIdx.y : blockIdx.x;
  }
  int64_t kb = 0, ke = K;
  if (SPLIT) {
    kb = bz * kchunk;
    ke = kb + kchunk < K ? kb + kchunk : K;
  } else {
    A += bz * sA;
    B += bz * sB;
    C += bz * sC;
  }
  const int64_t m0 = tmi * TM;
  const int64_t n0 = tni * BN;
  d4 acc[MT][2], acc2[MT][2];
  for (int i = 0; i < MT; ++i)
    for (int j = 0; j < 2; ++j) {
      acc[i][j] = d4{0, 0, 0, 0};
      acc2[i][j] = d4{0, 0, 0, 0};
    }
  // global -> registers -> LDS; the next K tile's loads are issued before
  // the MFMAs of the current one (register prefetch), so their latency hides
  // behind the matrix work.  Each thread's load coordinates are fixed over
  // K: row validity and base pointers are resolved once, and the K bound is
  // checked only on a partial last tile.
  double ra[UA], rb[UN > UB ? UN : UB], rb2[UB];
  const int rA = tid / TPR, cA = (tid % TPR) * UA;
  const bool a_ok = m0 + rA < M;
  const double* pA = A + (a_ok ? m0 + rA : 0) * lda + cA;
  const int rB = tid >> 2, cB = (tid & 3) * UN;            // B as [N][K]
  const bool bn_ok = n0 + rB < N;
  const double* pBn = B + (bn_ok ? n0 + rB : 0) * ldb + cB;
  const int kB = tid / KT, cN = (tid % KT) * UB;           // B as [K][N]
  const int64_t nB0 = n0 + cN;
  auto load_tile = [&](int64_t k0) {
    const bool kfull = k0 + KB <= ke;
#pragma unroll
    for (int u = 0; u < UA; ++u) ra[u] = (a_ok && (kfull || k0 + cA + u < ke)) ? pA[k0 + u] : 0.0;
    if (B_NK) {
#pragma unroll
      for (int u = 0; u < UN; ++u) rb[u] = (bn_ok && (kfull || k0 + cB + u < ke)) ? pBn[k0 + u] : 0.0;
    } else {
      const bool krow = kfull || k0 + kB < ke;
      const int64_t off = (k0 + kB) * ldb + nB0;
#pragma unroll
      for (int u = 0; u < UB; ++u) {
        const bool in = krow && nB0 + u < N;
        rb[u] = in ? B[off + u] : 0.0;
        if (DUAL) rb2[u] = in ? B2[off + u] : 0.0;
      }
    }
  };
  auto store_tile = [&](int bf) {
#pragma unroll
    for (int u = 0; u < UA; ++u) As[bf][rA][cA + u] = ra[u];
    if (B_NK) {
#pragma unroll
      for (int u = 0; u < UN; ++u) Bs[bf][rB][cB + u] = rb[u];
    } else {
#pragma unroll
      for (int u = 0; u < UB; ++u) {
        Bs[bf][cN + u][kB] = rb[u];
        if (DUAL) B2s[bf][cN + u][kB] = rb2[u];
      }
    }
  };
  int buf = 0;
  if (kb < ke) load_tile(kb);
  if (DBUF) {
    if (kb < ke) store_tile(0);
    __syncthreads();
  }
  for (int64_t k0 = kb; k0 < ke; k0 += KB) {
    if (!DBUF) {
      store_tile(0);
      __syncthreads();
    }
    const bool more = k0 + KB < ke;
    if (more) load_tile(k0 + KB);
#pragma unroll
    for (int kk = 0; kk < KB; kk += 4) {
      double a[MT], b[2], b2[2];
      for (int i = 0; i < MT; ++i) a[i] = As[buf][wm * (16 * MT) + i * 16 + (lane & 15)][kk + (lane >> 4)];
      for (int j = 0; j < 2; ++j) {
        b[j] = Bs[buf][wn * 32 + j * 16 + (lane & 15)][kk + (lane >> 4)];
        if (DUAL) b2[j] = B2s[buf][wn * 32 + j * 16 + (lane & 15)][kk + (lane >> 4)];
      }
      for (int i = 0; i < MT; ++i)
        for (int j = 0; j < 2; ++j) {
          acc[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[i], b[j], acc[i][j], 0, 0, 0);
          if (DUAL) acc2[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[i], b2[j], acc2[i][j], 0, 0, 0);
        }
    }
    if (DBUF) {
      // the other buffer was last read before the previous barrier
      if (more) store_tile(buf ^ 1);
      __syncthreads();
      buf ^= 1;
    } else {
      __syncthreads();
    }
  }
  for (int i = 0; i < MT; ++i)
    for (int j = 0; j < 2; ++j)
      for (int v = 0; v < 4; ++v) {
        const int64_t gm = m0 + wm * (16 * MT) + i * 16 + (lane >> 4) + 4 * v;
        const int64_t gn = n0 + wn * 32 + j * 16 + (lane & 15);
        if (gm < M && gn < N) {
          if (SPLIT) {
            double* P = C + bz * (DUAL ? 2 : 1) * M * N;
            P[gm * N + gn] = acc[i][j][v];
            if (DUAL) P[M * N + gm * N + gn] = acc2[i][j][v];
          } else if (DUAL) {
            double r = dvec[gm] + dshift;
            double val = r * acc[i][j][v] + acc2[i][j][v];
            if (V) val += V[gm * ldv + gn];
            C[gm * ldc + gn] = val;
          } else {
            double val = alpha * acc[i][j][v];
            if (beta != 0.0) val += beta * C[gm * ldc + gn];
            C[gm * ldc + gn] = val;
          }
        }
      }
}

hipError_t gemm_f64(bool b_is_nk, int64_t M, int64_t N, int64_t K, double alpha, const double* A,
                    int64_t lda, int64_t sA, const double* B, int64_t ldb, int64_t sB, double beta,
                    double* C, int64_t ldc, int64_t sC, int batch, hipStream_t s) {
  if (M <= 0 || N <= 0 || batch <= 0) return hipSuccess;
  dim3 grid;
  int mx;
  if (!tile_grid(M, N, batch, BM, BN, &grid, &mx)) return hipErrorInvalidValue;
  // three waves per SIMD asked of the compiler (accumulators in VGPRs, a
  // third wave for the MFMA pipe while the others wait on LDS or loads) and
  // the XCD-grouped tile order (the tiles sharing an A row band run on one
  // XCD at about the same time); the grid only fixes the workgroup count
  // Products with fewer than two 64 x 64 tiles per CU take 32 x 64 tiles
  // (twice the workgroups; each output element sums its K terms in the same
  // order either way).
  (void)mx;
  const bool narrow = (int64_t)grid.x * grid.y * grid.z < 512 && tile_grid(M, N, batch, BM / 2, BN, &grid, &mx);
#define GEMM_F64_LAUNCH(NK, MT_)                                                                               \
  hipLaunchKernelGGL((k_gemm_f64<NK, false, false, MT_, BK, 3>), grid, dim3(256), 0, s, M, N, K, alpha, A, lda, \
                     sA, B, ldb, sB, (const double*)nullptr, beta, C, ldc, sC, (const double*)nullptr, 0.0,     \
                     (const double*)nullptr, (int64_t)0, 2, (int64_t)0)
  if (b_is_nk) {
    if (narrow) GEMM_F64_LAUNCH(true, 1);
    else GEMM_F64_LAUNCH(true, 2);
  } else {
    if (narrow) GEMM_F64_LAUNCH(false, 1);
    else GEMM_F64_LAUNCH(false, 2);
  }
#undef GEMM_F64_LAUNCH
  return hipGetLastError();
}

// C = alpha sum_s P[s] + beta C over ns partial products P [ns][M][N]
// (summed in split order, so the result does not depend on the launch)
__global__ void k_splitk_sum(int64_t M, int64_t N, int ns, const double* __restrict__ P, double alpha, double beta,
                             double* __restrict__ C, int64_t ldc) {
  const int64_t mn = M * N;
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < mn; e += (int64_t)gridDim.x * blockDim.x) {
    double acc = 0.0;
    for (int k = 0; k < ns; ++k) acc += P[k * mn + e];
    const int64_t m = e / N, n = e % N;
    double v = alpha * acc;
    if (beta != 0.0) v += beta * C[m * ldc + n];
    C[m * ldc + n] = v;
  }
}

hipError_t gemm_f64_ws(bool b_is_nk, int64_t M, int64_t N, int64_t K, double alpha, const double* A, int64_t lda,
                       const double* B, int64_t ldb, double beta, double* C, int64_t ldc, double* ws, int64_t ws_n,
                       hipStream_t s) {
  if (M <= 0 || N <= 0) return hipSuccess;
  const int64_t tiles = ((M + BM - 1) / BM) * ((N + BN - 1) / BN);
  int64_t ns = 1;
  if (tiles < 512 && K >= 8 * BK) {
    ns = std::min<int64_t>((1024 + tiles - 1) / tiles, K / (4 * BK));
    ns = std::min<int64_t>(ns, 16);
    while (ns > 1 && ns * M * N > ws_n) --ns;
  }
  if (ns < 2 || !ws) return gemm_f64(b_is_nk, M, N, K, alpha, A, lda, 0, B, ldb, 0, beta, C, ldc, 0, 1, s);
  int64_t kchunk = (K + ns - 1) / ns;
  kchunk = (kchunk + BK - 1) / BK * BK;
  ns = (K + kchunk - 1) / kchunk;
  dim3 grid;
  int mx;
  if (!tile_grid(M, N, (int)ns, BM, BN, &grid, &mx)) return hipErrorInvalidValue;
  if (b_is_nk)
    hipLaunchKernelGGL((k_gemm_f64<true, false, true, 2, BK, 3>), grid, dim3(256), 0, s, M, N, K, 1.0, A, lda,
                       (int64_t)0, B, ldb, (int64_t)0, (const double*)nullptr, 0.0, ws, N, (int64_t)0,
                       (const double*)nullptr, 0.0, (const double*)nullptr, (int64_t)0, mx, kchunk);
  else
    hipLaunchKernelGGL((k_gemm_f64<false, false, true, 2, BK, 3>), grid, dim3(256), 0, s, M, N, K, 1.0, A, lda,
                       (int64_t)0, B, ldb, (int64_t)0, (const double*)nullptr, 0.0, ws, N, (int64_t)0,
                       (const double*)nullptr, 0.0, (const double*)nullptr, (int64_t)0, mx, kchunk);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  const unsigned g2 = cdiv(M * N, 256) > 65536 ? 65536 : cdiv(M * N, 256);
  hipLaunchKernelGGL(k_splitk_sum, dim3(g2), dim3(256), 0, s, M, N, (int)ns, (const double*)ws, alpha, beta, C, ldc);
  return hipGetLastError();
}

// batched C_p = A B_p (B_p [K][N], A shared or strided): 64 x 64 tiles with
// the accumulators in VGPRs (3 waves per SIMD asked of the compiler) and the
// XCD-grouped tile order with m fastest, so that the few m tiles reading one
// B tile run back to back on one XCD and B comes from HBM about once
hipError_t gemm_f64_batched(int64_t M, int64_t N, int64_t K, const double* A, int64_t lda, int64_t sA,
                            const double* B, int64_t ldb, int64_t sB, double* C, int64_t ldc, int64_t sC,
                            int batch, hipStream_t s) {
  if (M <= 0 || N <= 0 || batch <= 0) return hipSuccess;
  const int64_t tmn = (M + BM - 1) / BM, tnn = (N + BN - 1) / BN;
  if (tmn > 65535 || batch > 65535 || tnn > 0x7fffffff) return hipErrorInvalidValue;
  hipLaunchKernelGGL((k_gemm_f64<false, false, false, 2, 16, 3>), dim3((unsigned)tnn, (unsigned)tmn, (unsigned)batch),
                     dim3(256), 0, s, M, N, K, 1.0, A, lda, sA, B, ldb, sB, (const double*)nullptr, 0.0, C, ldc, sC,
                     (const double*)nullptr, 0.0, (const double*)nullptr, (int64_t)0, 3, (int64_t)0);
  return hipGetLastError();
}

int residual_splitk(int64_t M, int64_t N, int64_t K) {
  if (M <= 0 || N <= 0 || K < 8 * BK) return 1;
  const int64_t tiles = ((M + BM - 1) / BM) * ((N + BN - 1) / BN);
  if (tiles >= 512) return 1;
  int64_t ns = 1024 / tiles;             // about 1024 workgroups in all
  const int64_t maxs = K / (4 * BK);      // at least four K tiles per split
  if (ns > maxs) ns = maxs;
  if (ns > 64) ns = 64;
  return ns < 2 ? 1 : (int)ns;
}

// C[m][n] = V[m][n] + (d[m] + dshift) sum_z P[z][0][m][n] + sum_z P[z][1][m][n]
__global__ void k_splitk_epilogue(int64_t M, int64_t N, int ns, const double* __restrict__ P,
                                  const double* __restrict__ d, double dshift,
                                  const double* __restrict__ V, int64_t ldv, double* __restrict__ C,
                                  int64_t ldc) {
  const int64_t total = M * N;
  for (int64_t g = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; g < total;
       g += (int64_t)gridDim.x * blockDim.x) {
    const int64_t m = g / N, n = g % N;
    double xs = 0.0, xf = 0.0;
    for (int z = 0; z < ns; ++z) {
      xs += P[(int64_t)z * 2 * total + g];
      xf += P[(int64_t)z * 2 * total + total + g];
    }
    double val = (d[m] + dshift) * xs + xf;
    if (V) val += V[m * ldv + n];
    C[m * ldc + n] = val;
  }
}

hipError_t residual_gemm_f64(int64_t M, int64_t N, int64_t K, const double* X, int64_t ldx,
                             const double* S, const double* F, const double* d, double dshift,
                             const double* V, int64_t ldv, double* C, int64_t ldc, hipStream_t s,
                             double* ws, int64_t ws_len, LaunchTune tune) {
  if (M <= 0 || N <= 0) return hipSuccess;
  if (tune.tile != 0 && tune.tile != 64 && tune.tile != 128) return hipErrorInvalidValue;
  if (tune.kb != 0 && tune.kb != 16 && tune.kb != 32) return hipErrorInvalidValue;
  if (tune.occ < 0 || tune.occ > 3) return hipErrorInvalidValue;
  int ns = tune.splitk >= 1 ? tune.splitk : residual_splitk(M, N, K);
  if (!(ns > 1 && ws && ws_len >= (int64_t)ns * 2 * M * N)) ns = 1;
  const int tm = (ns == 1 && tune.tile == 128) ? 128 : 64;   // 128-row tiles without K splits only
  dim3 grid;
  int mx;
  if (!tile_grid(M, N, 1, tm, BN, &grid, &mx)) return hipErrorInvalidValue;
  if (tune.order >= 0) {
    // 0: n tiles on grid x, 1: m tiles on grid x, 2: XCD-grouped (the
    // kernel linearises the grid, any shape with the right count works)
    if (tune.order > 2) return hipErrorInvalidValue;
    if (tune.order != mx && tune.order != 2) {
      const unsigned gx = grid.x, gy = grid.y;
      if (gx > 65535) return hipErrorInvalidValue;
      grid.x = gy;
      grid.y = gx;
    }
    mx = tune.order;
  }
  if (ns > 1) {
    // few output tiles: split K over ns workgroups per tile, then one epilogue
    const int64_t kchunk = ((K + ns - 1) / ns + BK - 1) / BK * BK;
    const int nsplit = (int)((K + kchunk - 1) / kchunk);
    grid.z = nsplit;
    hipLaunchKernelGGL((k_gemm_f64<false, true, true>), grid, dim3(256), 0, s, M, N, K, 1.0, X, ldx,
                       (int64_t)0, S, N, (int64_t)0, F, 0.0, ws, N, (int64_t)0, d, dshift, V, ldv, mx,
                       kchunk);
    unsigned eg = (unsigned)((M * N + 255) / 256);
    if (eg > 4096) eg = 4096;
    hipLaunchKernelGGL(k_splitk_epilogue, dim3(eg), dim3(256), 0, s, M, N, nsplit, (const double*)ws, d,
                       dshift, V, ldv, C, ldc);
    return hipGetLastError();
  }
#define CASPT2_DUAL(MT_, KB_, WPE_)                                                                      \
  hipLaunchKernelGGL((k_gemm_f64<false, true, false, MT_, KB_, WPE_>), grid, dim3(256), 0, s, M, N, K, 1.0, X, \
                     ldx, (int64_t)0, S, N, (int64_t)0, F, 0.0, C, ldc, (int64_t)0, d, dshift, V, ldv, mx, (int64_t)0)
  // waves per SIMD asked of the compiler (it then keeps the accumulators in
  // VGPRs); by rule the most that compiles without spills: 3 for 64-row
  // tiles, 2 for 128-row tiles with K tile 16, 1 for 128 x 32
  const bool k32 = tune.kb == 32;
  if (tm == 128) {
    if (k32) {
      if (tune.occ > 1) return hipErrorInvalidValue;
      CASPT2_DUAL(4, 32, 1);
    } else if (tune.occ == 1) {
      CASPT2_DUAL(4, 16, 1);
    } else {
      if (tune.occ > 2) return hipErrorInvalidValue;
      CASPT2_DUAL(4, 16, 2);
    }
  } else {
    if (tune.occ == 2) return hipErrorInvalidValue;
    if (k32) {
      if (tune.occ == 1)
        CASPT2_DUAL(2, 32, 1);
      else
        CASPT2_DUAL(2, 32, 3);
    } else {
      if (tune.occ == 1)
        CASPT2_DUAL(2, 16, 1);
      else
        CASPT2_DUAL(2, 16, 3);
    }
  }
#undef CASPT2_DUAL
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// streaming residual for small alpha dimension (K = N <= 64):
//   C[m][n] = V[m][n] + (d[m] + dshift) * sum_k X[m][k] S[k][n] + sum_k X[m][k] F[k][n]
// ---------------------------------------------------------------------------
template <typename T>
__global__ __launch_bounds__(256) void k_residual_small(int64_t M, int N, const T* __restrict__ X,
                                                        const T* __restrict__ S,
                                                        const T* __restrict__ F,
                                                        const T* __restrict__ d, T dshift,
                                                        const T* __restrict__ V,
                                                        T* __restrict__ C) {
  __shared__ T Ss[64 * 64];
  __shared__ T Fs[64 * 64];
  for (int i = threadIdx.x; i < N * N; i += blockDim.x) {
    Ss[i] = S[i];
    Fs[i] = F[i];
  }
  __syncthreads();
  const int64_t total = M * N;
  for (int64_t g = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; g < total;
       g += (int64_t)gridDim.x * blockDim.x) {
    const int64_t m = g / N;
    const int n = (int)(g % N);
    const T* x = X + m * N;
    T as = 0, af = 0;
    for (int k = 0; k < N; ++k) {
      const T xv = x[k];
      as += xv * Ss[k * N + n];
      af += xv * Fs[k * N + n];
    }
    T val = (d[m] + dshift) * as + af;
    if (V) val += V[g];
    C[g] = val;
  }
}

// Streaming residual on MFMA for 16 < K = N <= 64: S and F (zero padded to
// K16 = ceil16(K)) live in LDS for the whole launch; each wave stages 16 rows
// of X in LDS with coalesced loads and accumulates X S and X F with
// v_mfma_f64_16x16x4f64; epilogue (d[m] + dshift) XS + XF + V.
// PIPE: the wave's next 16-row tile of X is loaded into registers while the
// current one is multiplied, and the current tile's V and row energies are
// requested before the MFMAs, so HBM latency overlaps the matrix work (the
// plain form waits for its loads at every tile).  BREG: each lane keeps its
// MFMA B operands of S and F (the same for every tile) in registers instead
// of reading them from LDS per tile (fewer LDS reads, more registers).
template <int K16, bool PIPE, bool BREG = false>
__global__ __launch_bounds__(256) void k_residual_mfma(int64_t M, int K, const double* __restrict__ X,
                                                       const double* __restrict__ S,
                                                       const double* __restrict__ F,
                                                       const double* __restrict__ d, double dshift,
                                                       const double* __restrict__ V,
                                                       double* __restrict__ C) {
  constexpr int XPL = 16 * K16 / 64;   // staged X values per lane
  constexpr int NCT = K16 / 16;        // 16-column output tiles
  __shared__ double Ss[K16][K16 + 1];
  __shared__ double Fs[K16][K16 + 1];
  __shared__ double Xs[4][16][K16 + 1];
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  for (int i = tid; i < K16 * K16; i += 256) {
    const int r = i / K16, c = i % K16;
    const bool in = r < K && c < K;
    Ss[r][c] = in ? S[r * K + c] : 0.0;
    Fs[r][c] = in ? F[r * K + c] : 0.0;
  }
  __syncthreads();
  const int64_t ntiles = (M + 15) / 16;
  const int64_t stride = (int64_t)gridDim.x * 4;
  const int64_t limit = M * (int64_t)K;
  constexpr int NKS = K16 / 4;
  double bsr[BREG ? NCT : 1][BREG ? NKS : 1], bfr[BREG ? NCT : 1][BREG ? NKS : 1];
  if (BREG) {
#pragma unroll
    for (int ct = 0; ct < NCT; ++ct)
#pragma unroll
      for (int ks = 0; ks < NKS; ++ks) {
        bsr[ct][ks] = Ss[ks * 4 + (lane >> 4)][ct * 16 + (lane & 15)];
        bfr[ct][ks] = Fs[ks * 4 + (lane >> 4)][ct * 16 + (lane & 15)];
      }
  }
  double xr[XPL];
  auto load_x = [&](int64_t tile) {   // 16 rows (contiguous 16*K doubles) of X
    const int64_t base = tile * 16 * K;
#pragma unroll
    for (int j = 0; j < XPL; ++j) {
      const int i = lane + 64 * j;
      const int r = i / K16, c = i % K16;
      const int64_t gi = base + (int64_t)r * K + c;
      xr[j] = (c < K && gi < limit) ? X[gi] : 0.0;
    }
  };
  int64_t tile = (int64_t)blockIdx.x * 4 + w;
  if (PIPE && tile < ntiles) load_x(tile);
  for (; tile < ntiles; tile += stride) {
    const int64_t m0 = tile * 16;
    if (!PIPE) load_x(tile);
#pragma unroll
    for (int j = 0; j < XPL; ++j) {
      const int i = lane + 64 * j;
      Xs[w][i / K16][i % K16] = xr[j];
    }
    // the staged tile is read by other lanes of this wave: wait for the LDS
    // writes only (lgkmcnt 0; vmcnt and expcnt left at their maxima)
    __builtin_amdgcn_s_waitcnt(0xC07F);
    __builtin_amdgcn_wave_barrier();
    // this tile's row energies and V, then the next tile's X, all in flight
    // during the MFMAs (loads complete in order: V before the prefetch)
    double rr[4], vr[NCT][4];
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int64_t row = m0 + (lane >> 4) + 4 * v;
      rr[v] = row < M ? d[row] + dshift : 0.0;
#pragma unroll
      for (int ct = 0; ct < NCT; ++ct) {
        const int col = ct * 16 + (lane & 15);
        vr[ct][v] = (V && row < M && col < K) ? V[row * K + col] : 0.0;
      }
    }
    if (PIPE && tile + stride < ntiles) load_x(tile + stride);
#pragma unroll
    for (int ct = 0; ct < NCT; ++ct) {
      d4 as = {0, 0, 0, 0}, af = {0, 0, 0, 0};
#pragma unroll
      for (int k0 = 0; k0 < K16; k0 += 4) {
        const double a = Xs[w][lane & 15][k0 + (lane >> 4)];
        const double bs = BREG ? bsr[BREG ? ct : 0][BREG ? k0 / 4 : 0] : Ss[k0 + (lane >> 4)][ct * 16 + (lane & 15)];
        const double bf = BREG ? bfr[BREG ? ct : 0][BREG ? k0 / 4 : 0] : Fs[k0 + (lane >> 4)][ct * 16 + (lane & 15)];
        as = __builtin_amdgcn_mfma_f64_16x16x4f64(a, bs, as, 0, 0, 0);
        af = __builtin_amdgcn_mfma_f64_16x16x4f64(a, bf, af, 0, 0, 0);
      }
      const int col = ct * 16 + (lane & 15);
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int64_t row = m0 + (lane >> 4) + 4 * v;
        if (row < M && col < K) C[row * K + col] = rr[v] * as[v] + af[v] + vr[ct][v];
      }
    }
    __builtin_amdgcn_wave_barrier();
  }
}

hipError_t residual_small_f64(int64_t M, int64_t N, const double* X, const double* S,
                              const double* F, const double* d, double dshift, const double* V,
                              double* C, hipStream_t s, LaunchTune tune) {
  if (M <= 0 || N <= 0) return hipSuccess;
  if (N > 64) return hipErrorInvalidValue;
  const unsigned cap = tune.grid ? tune.grid : 0;
  if (N > 16) {
    const int64_t ntiles = (M + 15) / 16;
    unsigned grid = cdiv(ntiles, 4);
    if (grid > (cap ? cap : 16384u)) grid = cap ? cap : 16384u;
#define CASPT2_RMFMA(K16_)                                                                              \
  do {                                                                                                  \
    if (tune.plain)                                                                                     \
      hipLaunchKernelGGL((k_residual_mfma<K16_, false>), dim3(grid), dim3(256), 0, s, M, (int)N, X, S, F, d, \
                         dshift, V, C);                                                                 \
    else                                                                                                \
      hipLaunchKernelGGL((k_residual_mfma<K16_, true>), dim3(grid), dim3(256), 0, s, M, (int)N, X, S, F, d, \
                         dshift, V, C);                                                                 \
  } while (0)
    if (N <= 32 && tune.breg)   // B operands in registers (K16 = 32 only: 32 doubles per lane)
      hipLaunchKernelGGL((k_residual_mfma<32, true, true>), dim3(grid), dim3(256), 0, s, M, (int)N, X, S, F, d,
                         dshift, V, C);
    else if (N <= 32)
      CASPT2_RMFMA(32);
    else if (N <= 48)
      CASPT2_RMFMA(48);
    else
      CASPT2_RMFMA(64);
#undef CASPT2_RMFMA
    return hipGetLastError();
  }
  unsigned grid = cdiv(M * N, 256);
  if (grid > (cap ? cap : 65536u)) grid = cap ? cap : 65536u;
  hipLaunchKernelGGL(k_residual_small<double>, dim3(grid), dim3(256), 0, s, M, (int)N, X, S, F, d,
                     dshift, V, C);
  return hipGetLastError();
}

hipError_t residual_small_f32(int64_t M, int64_t N, const float* X, const float* S, const float* F,
                              const float* d, float dshift, const float* V, float* C,
                              hipStream_t s) {
  if (M <= 0 || N <= 0) return hipSuccess;
  if (N > 64) return hipErrorInvalidValue;
  unsigned grid = cdiv(M * N, 256);
  if (grid > 65536) grid = 65536;
  hipLaunchKernelGGL(k_residual_small<float>, dim3(grid), dim3(256), 0, s, M, (int)N, X, S, F, d,
                     dshift, V, C);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// ccvv streaming residual: rows of NST doubles, two consecutive entries (the
// '+' and '-' characters) in one launch.  Row m of entry c:
//   C[m][n] = V[m][n] + (d_c(m) + dshift) sum_k X[m][k] S_c[k][n] + sum_k X[m][k] F_c[k][n]
// S_c, F_c are NST x NST (kept in registers); one thread per row.  The row
// energy is separable in the packed row index, d_c(m) = A_c[m / nB_c] +
// B_c[m % nB_c] (first orbital unit / the rest; small tables that stay in
// cache), so no per-row energy stream is read.
// ---------------------------------------------------------------------------
template <typename T, int NST>
__global__ __launch_bounds__(256) void k_residual_rows(int64_t M0, int64_t M1,
                                                       const T* __restrict__ X,
                                                       const T* __restrict__ S0,
                                                       const T* __restrict__ F0,
                                                       const T* __restrict__ S1,
                                                       const T* __restrict__ F1,
                                                       RowEnergy<T> d0, RowEnergy<T> d1, T dshift,
                                                       const T* __restrict__ V,
                                                       T* __restrict__ C) {
  T s0[NST * NST], f0[NST * NST], s1[NST * NST], f1[NST * NST];
#pragma unroll
  for (int i = 0; i < NST * NST; ++i) {
    s0[i] = S0[i];
    f0[i] = F0[i];
    s1[i] = S1 ? S1[i] : T(0);
    f1[i] = F1 ? F1[i] : T(0);
  }
  const int64_t total = M0 + M1;
  for (int64_t m = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; m < total;
       m += (int64_t)gridDim.x * blockDim.x) {
    const bool second = m >= M0;
    const uint32_t mr = (uint32_t)(second ? m - M0 : m);
    const RowEnergy<T>& de = second ? d1 : d0;
    const uint32_t qa = mr / de.nB;
    const T r = de.A[qa] + de.B[mr - qa * de.nB] + dshift;
    T x[NST], out[NST];
#pragma unroll
    for (int k = 0; k < NST; ++k) x[k] = X[m * NST + k];
#pragma unroll
    for (int n = 0; n < NST; ++n) {
      T as = 0, af = 0;
#pragma unroll
      for (int k = 0; k < NST; ++k) {
        as += x[k] * (second ? s1[k * NST + n] : s0[k * NST + n]);
        af += x[k] * (second ? f1[k * NST + n] : f0[k * NST + n]);
      }
      out[n] = r * as + af;
    }
    if (V) {
#pragma unroll
      for (int n = 0; n < NST; ++n) out[n] += V[m * NST + n];
    }
#pragma unroll
    for (int n = 0; n < NST; ++n) C[m * NST + n] = out[n];
  }
}

template <typename T>
hipError_t residual_rows(int nst, int64_t M0, int64_t M1, const T* X, const T* S0, const T* F0,
                         const T* S1, const T* F1, RowEnergy<T> d0, RowEnergy<T> d1, T dshift,
                         const T* V, T* C, hipStream_t s, LaunchTune tune) {
  const int64_t total = M0 + M1;
  if (total <= 0) return hipSuccess;
  if (M0 >= ((int64_t)1 << 31) || M1 >= ((int64_t)1 << 31) || d0.nB == 0 || (M1 > 0 && d1.nB == 0))
    return hipErrorInvalidValue;
  const unsigned cap = tune.grid ? tune.grid : 65536u;
  unsigned grid = cdiv(total, 256);
  if (grid > cap) grid = cap;
  switch (nst) {
#define CASPT2_ROWS(NS)                                                                        \
  case NS:                                                                                     \
    hipLaunchKernelGGL((k_residual_rows<T, NS>), dim3(grid), dim3(256), 0, s, M0, M1, X, S0, F0, S1, \
                       F1, d0, d1, dshift, V, C);                                              \
    break;
    CASPT2_ROWS(1)
    CASPT2_ROWS(2)
    CASPT2_ROWS(3)
    CASPT2_ROWS(4)
#undef CASPT2_ROWS
    default:
      return hipErrorInvalidValue;
  }
  return hipGetLastError();
}
template hipError_t residual_rows<double>(int, int64_t, int64_t, const double*, const double*,
                                          const double*, const double*, const double*,
                                          RowEnergy<double>, RowEnergy<double>, double, const double*,
                                          double*, hipStream_t, LaunchTune);
template hipError_t residual_rows<float>(int, int64_t, int64_t, const float*, const float*,
                                         const float*, const float*, const float*, RowEnergy<float>,
                                         RowEnergy<float>, float, const float*, float*, hipStream_t,
                                         LaunchTune);

// separable row energies from the full table: A[a] = eps[a nB], B[b] =
// eps[b] - eps[0] (eps(a nB + b) = A[a] + B[b] when eps is a sum of a
// function of the first unit and a function of the rest)
__global__ void k_split_energies(int64_t nA, int64_t nB, const double* __restrict__ eps,
                                 double* __restrict__ A, double* __restrict__ B) {
  const int64_t n = nA > nB ? nA : nB;
  for (int64_t g = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; g < n;
       g += (int64_t)gridDim.x * blockDim.x) {
    if (g < nA) A[g] = eps[g * nB];
    if (g < nB) B[g] = eps[g] - eps[0];
  }
}

hipError_t split_energies(int64_t nA, int64_t nB, const double* eps, double* A, double* B,
                          hipStream_t s) {
  const int64_t n = nA > nB ? nA : nB;
  if (n <= 0) return hipSuccess;
  unsigned grid = cdiv(n, 256);
  if (grid > 4096) grid = 4096;
  hipLaunchKernelGGL(k_split_energies, dim3(grid), dim3(256), 0, s, nA, nB, eps, A, B);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// row transform for narrow rows (nin, nout <= 8), one thread per row:
//   out[m][j] = sum_i in[m][i] W[i * ws_in + j * ws_out]
// (the basis transforms of the entries with few active columns, streaming)
// ---------------------------------------------------------------------------
template <typename T>
__global__ __launch_bounds__(256) void k_transform_rows(int64_t M, int nin, int nout,
                                                        const T* __restrict__ in,
                                                        const T* __restrict__ W, int ws_in,
                                                        int ws_out, T* __restrict__ out) {
  T w[8][8];
#pragma unroll
  for (int i = 0; i < 8; ++i)
#pragma unroll
    for (int j = 0; j < 8; ++j) w[i][j] = (i < nin && j < nout) ? W[i * ws_in + j * ws_out] : T(0);
  for (int64_t m = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; m < M;
       m += (int64_t)gridDim.x * blockDim.x) {
    T x[8];
#pragma unroll
    for (int i = 0; i < 8; ++i) x[i] = i < nin ? in[m * nin + i] : T(0);
#pragma unroll
    for (int j = 0; j < 8; ++j) {
      if (j >= nout) break;
      T acc = 0;
#pragma unroll
      for (int i = 0; i < 8; ++i) acc += x[i] * w[i][j];
      out[m * nout + j] = acc;
    }
  }
}

template <typename T>
hipError_t transform_rows(int64_t M, int nin, int nout, const T* in, const T* W, int ws_in,
                          int ws_out, T* out, hipStream_t s) {
  if (M <= 0 || nout <= 0) return hipSuccess;
  if (nin < 0 || nin > 8 || nout > 8) return hipErrorInvalidValue;
  unsigned grid = cdiv(M, 256);
  if (grid > 65536) grid = 65536;
  hipLaunchKernelGGL(k_transform_rows<T>, dim3(grid), dim3(256), 0, s, M, nin, nout, in, W, ws_in,
                     ws_out, out);
  return hipGetLastError();
}
template hipError_t transform_rows<double>(int64_t, int, int, const double*, const double*, int,
                                           int, double*, hipStream_t);
template hipError_t transform_rows<float>(int64_t, int, int, const float*, const float*, int, int,
                                          float*, hipStream_t);

struct PermArgs {
  int nd;
  int64_t dims[10];
  int64_t dstride[10];
};

__global__ void k_permute_axpy(PermArgs p, int64_t total, double c, const double* __restrict__ src,
                               double* __restrict__ dst) {
  for (int64_t g = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; g < total;
       g += (int64_t)gridDim.x * blockDim.x) {
    int64_t rem = g, off = 0;
    for (int k = p.nd - 1; k >= 0; --k) {
      const int64_t ik = rem % p.dims[k];
      rem /= p.dims[k];
      off += ik * p.dstride[k];
    }
    dst[off] += c * src[g];
  }
}

hipError_t permute_axpy(int nd, const int64_t* dims, const int64_t* dstride, double c,
                        const double* src, double* dst, hipStream_t s) {
  PermArgs p;
  p.nd = nd;
  int64_t total = 1;
  for (int k = 0; k < nd; ++k) {
    p.dims[k] = dims[k];
    p.dstride[k] = dstride[k];
    total *= dims[k];
  }
  if (total == 0) return hipSuccess;
  unsigned grid = cdiv(total, 256);
  if (grid > 65536) grid = 65536;
  hipLaunchKernelGGL(k_permute_axpy, dim3(grid), dim3(256), 0, s, p, total, c, src, dst);
  return hipGetLastError();
}

// dst[sum_k i_k dstride[k]] = src[g] for the element g = (i_0, .., i_{nd-1})
// of src (row-major dims): a permutation of all elements, so dst needs no
// clearing
template <typename T, typename I>
__global__ void k_permute_copy(PermArgs p, int64_t total, const T* __restrict__ src, T* __restrict__ dst) {
  // I: 32-bit index arithmetic when every element index fits (the
  // division chain is the kernel's ALU cost)
  for (int64_t g = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; g < total;
       g += (int64_t)gridDim.x * blockDim.x) {
    I rem = (I)g;
    int64_t off = 0;
    for (int k = p.nd - 1; k >= 0; --k) {
      const I dk = (I)p.dims[k];
      const I q = rem / dk;
      off += (int64_t)(rem - q * dk) * p.dstride[k];
      rem = q;
    }
    dst[off] = src[g];
  }
}

template <typename T>
hipError_t permute_copy(int nd, const int64_t* dims, const int64_t* dstride, const T* src, T* dst, hipStream_t s) {
  if (nd < 1 || nd > 10) return hipErrorInvalidValue;
  PermArgs p;
  p.nd = nd;
  int64_t total = 1;
  for (int k = 0; k < nd; ++k) {
    p.dims[k] = dims[k];
    p.dstride[k] = dstride[k];
    total *= dims[k];
  }
  if (total == 0) return hipSuccess;
  unsigned grid = cdiv(total, 256);
  if (grid > 65536) grid = 65536;
  if (total <= (int64_t)0xffffffffu)
    hipLaunchKernelGGL((k_permute_copy<T, uint32_t>), dim3(grid), dim3(256), 0, s, p, total, src, dst);
  else
    hipLaunchKernelGGL((k_permute_copy<T, int64_t>), dim3(grid), dim3(256), 0, s, p, total, src, dst);
  return hipGetLastError();
}
template hipError_t permute_copy<double>(int, const int64_t*, const int64_t*, const double*, double*, hipStream_t);
template hipError_t permute_copy<float>(int, const int64_t*, const int64_t*, const float*, float*, hipStream_t);

__global__ void k_contract_lead(int64_t ni, int64_t nj, const double* __restrict__ c,
                                const double* __restrict__ G, double* __restrict__ y) {
  for (int64_t j = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; j < nj;
       j += (int64_t)gridDim.x * blockDim.x) {
    double acc = 0.0;
    for (int64_t i = 0; i < ni; ++i) acc += c[i] * G[i * nj + j];
    y[j] += acc;
  }
}

hipError_t contract_lead(int64_t ni, int64_t nj, const double* c, const double* G, double* y,
                         hipStream_t s) {
  if (nj == 0) return hipSuccess;
  unsigned grid = cdiv(nj, 256);
  if (grid > 65536) grid = 65536;
  hipLaunchKernelGGL(k_contract_lead, dim3(grid), dim3(256), 0, s, ni, nj, c, G, y);
  return hipGetLastError();
}

__global__ void k_df_pack(const double* __restrict__ B, int naux, int nmo, int p0, int np, int q0,
                          int nq, double* __restrict__ Bt) {
  const int64_t total = (int64_t)np * nq * naux;
  for (int64_t g = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; g < total;
       g += (int64_t)gridDim.x * blockDim.x) {
    const int64_t Q = g % naux;
    const int64_t pq = g / naux;
    const int64_t p = pq / nq, q = pq % nq;
    Bt[g] = B[(Q * nmo + p0 + p) * nmo + q0 + q];
  }
}

hipError_t df_pack(const double* B, int naux, int nmo, int p0, int np, int q0, int nq, double* Bt,
                   hipStream_t s) {
  const int64_t total = (int64_t)np * nq * naux;
  if (total == 0) return hipSuccess;
  unsigned grid = cdiv(total, 256);
  if (grid > 65536) grid = 65536;
  hipLaunchKernelGGL(k_df_pack, dim3(grid), dim3(256), 0, s, B, naux, nmo, p0, np, q0, nq, Bt);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// packed term contraction
//   out[row][alpha] += scale * sum_{images e of the orbit} w chi(pi_e)
//                      * sum_{y} C[idx(e, y)] * G[(y * nalpha + alpha) * gcols + gcol]
// ---------------------------------------------------------------------------

__global__ void k_term_source(TermDesc d, const double* __restrict__ C, const double* __restrict__ G,
                              double* __restrict__ out) {
  const int64_t total = d.nrow * d.nalpha;
  for (int64_t g = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; g < total;
       g += (int64_t)gridDim.x * blockDim.x) {
    const int64_t row = g / d.nalpha;
    const int64_t al = g % d.nalpha;
    int e0[4] = {0, 0, 0, 0};
    decode_orbit(d, row, e0);
    int ndistinct = 0;
    for (int s = 0; s < d.nswap; ++s)
      if (e0[d.swap_k[s]] != e0[d.swap_l[s]]) ++ndistinct;
    const double w = d.mode_avg ? 1.0 : 1.0 / sqrt((double)(1 << ndistinct));
    double acc = 0.0;
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
      // C offset: the slot part, and the stride of each summed active label
      int64_t base = 0, ls[3] = {0, 0, 0};
      for (int a = 0; a < d.ncax; ++a) {
        const int src = d.c_slot[a];
        if (src >= 0) base += (int64_t)e[src] * d.c_stride[a];
        else ls[-1 - src] += d.c_stride[a];
      }
      // y = (y0 na + y1) na + y2 (labels past nopact fixed at 0) in
      // ascending order, the offsets advanced by additions
      const int n0 = d.nopact >= 1 ? d.na : 1, n1 = d.nopact >= 2 ? d.na : 1, n2 = d.nopact >= 3 ? d.na : 1;
      const int64_t gstep = d.galpha * d.gcols;
      const double* gp = G + (d.goff + al) * d.gcols + d.gcol;
      double val = 0.0;
      int64_t o0 = base;
      for (int y0 = 0; y0 < n0; ++y0, o0 += ls[0]) {
        int64_t o1 = o0;
        for (int y1 = 0; y1 < n1; ++y1, o1 += ls[1]) {
          int64_t o2 = o1;
          for (int y2 = 0; y2 < n2; ++y2, o2 += ls[2]) {
            val += C[o2] * *gp;
            gp += gstep;
          }
        }
      }
      acc += sg * val;
    }
    out[row * d.ldo + al] += d.scale * w * acc;
  }
}

hipError_t term_source(const TermDesc& d, const double* C, const double* G, double* out,
                       hipStream_t s) {
  const int64_t total = d.nrow * d.nalpha;
  if (total == 0) return hipSuccess;
  unsigned grid = cdiv(total, 256);
  if (grid > 65536) grid = 65536;
  hipLaunchKernelGGL(k_term_source, dim3(grid), dim3(256), 0, s, d, C, G, out);
  return hipGetLastError();
}

__global__ void k_select_scale_cols(int64_t n, int64_t ncq, const double* __restrict__ Q,
                                    const int32_t* __restrict__ idx, const double* __restrict__ sc,
                                    int64_t nk, double* __restrict__ X0) {
  const int64_t total = n * nk;
  for (int64_t g = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; g < total;
       g += (int64_t)gridDim.x * blockDim.x) {
    const int64_t i = g / nk, k = g % nk;
    X0[g] = Q[i * ncq + idx[k]] * sc[k];
  }
}

hipError_t select_scale_cols(int64_t n, int64_t ncq, const double* Q, const int32_t* idx,
                             const double* scale, int64_t nk, double* X0, hipStream_t s) {
  const int64_t total = n * nk;
  if (total == 0) return hipSuccess;
  unsigned grid = cdiv(total, 256);
  if (grid > 65536) grid = 65536;
  hipLaunchKernelGGL(k_select_scale_cols, dim3(grid), dim3(256), 0, s, n, ncq, Q, idx, scale, nk, X0);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Jacobi eigensolver: parallel cyclic (round-robin) two-sided rotations
// ---------------------------------------------------------------------------
__device__ inline int rr_player(int pos, int step, int m) {
  if (pos == 0) return 0;
  return 1 + ((pos - 1 + step) % (m - 1));
}

__global__ void k_jac_params(int n, int m, int step, const double* __restrict__ A,
                             double* __restrict__ cs, int* __restrict__ pq) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= m / 2) return;
  int p = rr_player(k, step, m), q = rr_player(m - 1 - k, step, m);
  if (p > q) {
    const int t = p;
    p = q;
    q = t;
  }
  double c = 1.0, s = 0.0;
  if (q < n) {
    const double apq = A[(int64_t)p * n + q];
    if (apq != 0.0) {
      const double app = A[(int64_t)p * n + p], aqq = A[(int64_t)q * n + q];
      const double tau = (aqq - app) / (2.0 * apq);
      const double t = (tau >= 0.0 ? 1.0 : -1.0) / (fabs(tau) + sqrt(1.0 + tau * tau));
      c = 1.0 / sqrt(1.0 + t * t);
      s = t * c;
    }
  }
  cs[2 * k] = c;
  cs[2 * k + 1] = s;
  pq[2 * k] = p;
  pq[2 * k + 1] = q;
}

// one thread per (pair a, pair b): rotate the 2x2 block; extra threads rotate V
__global__ void k_jac_apply(int n, int m, double* __restrict__ A, double* __restrict__ V,
                            const double* __restrict__ cs, const int* __restrict__ pq) {
  const int64_t h = m / 2;
  const int64_t g = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (g < h * h) {
    const int a = (int)(g / h), b = (int)(g % h);
    const int pa = pq[2 * a], qa = pq[2 * a + 1], pb = pq[2 * b], qb = pq[2 * b + 1];
    const double ca = cs[2 * a], sa = cs[2 * a + 1], cb = cs[2 * b], sb = cs[2 * b + 1];
    const bool ipa = pa < n, iqa = qa < n, ipb = pb < n, iqb = qb < n;
    const double m00 = (ipa && ipb) ? A[(int64_t)pa * n + pb] : 0.0;
    const double m01 = (ipa && iqb) ? A[(int64_t)pa * n + qb] : 0.0;
    const double m10 = (iqa && ipb) ? A[(int64_t)qa * n + pb] : 0.0;
    const double m11 = (iqa && iqb) ? A[(int64_t)qa * n + qb] : 0.0;
    // rows: J_a^T
    const double r00 = ca * m00 - sa * m10, r01 = ca * m01 - sa * m11;
    const double r10 = sa * m00 + ca * m10, r11 = sa * m01 + ca * m11;
    // cols: J_b
    const double o00 = cb * r00 - sb * r01, o01 = sb * r00 + cb * r01;
    const double o10 = cb * r10 - sb * r11, o11 = sb * r10 + cb * r11;
    if (ipa && ipb) A[(int64_t)pa * n + pb] = o00;
    if (ipa && iqb) A[(int64_t)pa * n + qb] = o01;
    if (iqa && ipb) A[(int64_t)qa * n + pb] = o10;
    if (iqa && iqb) A[(int64_t)qa * n + qb] = o11;
  } else if (g < h * h + (int64_t)n * h) {
    const int64_t gg = g - h * h;
    const int i = (int)(gg / h), a = (int)(gg % h);
    const int pa = pq[2 * a], qa = pq[2 * a + 1];
    if (qa >= n) return;
    const double ca = cs[2 * a], sa = cs[2 * a + 1];
    const double vp = V[(int64_t)i * n + pa], vq = V[(int64_t)i * n + qa];
    V[(int64_t)i * n + pa] = ca * vp - sa * vq;
    V[(int64_t)i * n + qa] = sa * vp + ca * vq;
  }
}

// rotation (c, s) that annihilates A[p][q] (p < q) of the current matrix
__device__ inline void jac_rotation(int n, const double* __restrict__ A, int p, int q, double& c, double& s) {
  c = 1.0;
  s = 0.0;
  if (q >= n) return;
  const double apq = A[(int64_t)p * n + q];
  if (apq == 0.0) return;
  const double app = A[(int64_t)p * n + p], aqq = A[(int64_t)q * n + q];
  const double tau = (aqq - app) / (2.0 * apq);
  const double t = (tau >= 0.0 ? 1.0 : -1.0) / (fabs(tau) + sqrt(1.0 + tau * tau));
  c = 1.0 / sqrt(1.0 + t * t);
  s = t * c;
}

__device__ inline void jac_pair(int k, int step, int m, int& p, int& q) {
  p = rr_player(k, step, m);
  q = rr_player(m - 1 - k, step, m);
  if (p > q) {
    const int t = p;
    p = q;
    q = t;
  }
}

// One rotation step in one launch: every thread derives the rotations it
// needs from the matrix of the previous step (Aold, read only), so no
// separate parameter launch and no race on the diagonal blocks; the rotated
// matrix goes to Anew (the two buffers alternate).  Threads [0, h^2) rotate
// the 2 x 2 blocks, the rest the rows of V (in place: each V element has one
// owner).
__global__ void k_jac_step(int n, int m, int step, const double* __restrict__ Aold, double* __restrict__ Anew,
                           double* __restrict__ V) {
  const int64_t h = m / 2;
  const int64_t g = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (g < h * h) {
    const int a = (int)(g / h), b = (int)(g % h);
    int pa, qa, pb, qb;
    jac_pair(a, step, m, pa, qa);
    jac_pair(b, step, m, pb, qb);
    double ca, sa, cb, sb;
    jac_rotation(n, Aold, pa, qa, ca, sa);
    jac_rotation(n, Aold, pb, qb, cb, sb);
    const bool ipa = pa < n, iqa = qa < n, ipb = pb < n, iqb = qb < n;
    const double m00 = (ipa && ipb) ? Aold[(int64_t)pa * n + pb] : 0.0;
    const double m01 = (ipa && iqb) ? Aold[(int64_t)pa * n + qb] : 0.0;
    const double m10 = (iqa && ipb) ? Aold[(int64_t)qa * n + pb] : 0.0;
    const double m11 = (iqa && iqb) ? Aold[(int64_t)qa * n + qb] : 0.0;
    const double r00 = ca * m00 - sa * m10, r01 = ca * m01 - sa * m11;
    const double r10 = sa * m00 + ca * m10, r11 = sa * m01 + ca * m11;
    if (ipa && ipb) Anew[(int64_t)pa * n + pb] = cb * r00 - sb * r01;
    if (ipa && iqb) Anew[(int64_t)pa * n + qb] = sb * r00 + cb * r01;
    if (iqa && ipb) Anew[(int64_t)qa * n + pb] = cb * r10 - sb * r11;
    if (iqa && iqb) Anew[(int64_t)qa * n + qb] = sb * r10 + cb * r11;
  } else if (g < h * h + (int64_t)n * h) {
    const int64_t gg = g - h * h;
    const int i = (int)(gg / h), a = (int)(gg % h);
    int pa, qa;
    jac_pair(a, step, m, pa, qa);
    if (qa >= n) return;
    double ca, sa;
    jac_rotation(n, Aold, pa, qa, ca, sa);
    const double vp = V[(int64_t)i * n + pa], vq = V[(int64_t)i * n + qa];
    V[(int64_t)i * n + pa] = ca * vp - sa * vq;
    V[(int64_t)i * n + qa] = sa * vp + ca * vq;
  }
}

__global__ void k_eye(int n, double* V) {
  const int64_t g = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (g < (int64_t)n * n) V[g] = (g / n == g % n) ? 1.0 : 0.0;
}

// off-diagonal and total squared norms: per-workgroup partial sums over a
// grid-stride range (part[2 b], part[2 b + 1]), then one workgroup adds the
// partials in a fixed order (out[0] = off-diagonal, out[1] = total)
constexpr int JAC_NORM_WG = 256;   // workgroups of the partial pass (<= 256)
__global__ void k_jac_norms_part(int n, const double* __restrict__ A, double* __restrict__ part) {
  __shared__ double so[256], st[256];
  double off = 0.0, tot = 0.0;
  const int64_t nn = (int64_t)n * n;
  for (int64_t g = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; g < nn; g += (int64_t)gridDim.x * blockDim.x) {
    const double v = A[g];
    tot += v * v;
    if (g / n != g % n) off += v * v;
  }
  so[threadIdx.x] = off;
  st[threadIdx.x] = tot;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (threadIdx.x < w) {
      so[threadIdx.x] += so[threadIdx.x + w];
      st[threadIdx.x] += st[threadIdx.x + w];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    part[2 * blockIdx.x] = so[0];
    part[2 * blockIdx.x + 1] = st[0];
  }
}

__global__ void k_jac_norms_fin(int nb, const double* __restrict__ part, double* __restrict__ out) {
  __shared__ double so[256], st[256];
  const int t = threadIdx.x;
  so[t] = t < nb ? part[2 * t] : 0.0;
  st[t] = t < nb ? part[2 * t + 1] : 0.0;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (t < w) {
      so[t] += so[t + w];
      st[t] += st[t + w];
    }
    __syncthreads();
  }
  if (t == 0) {
    out[0] = so[0];
    out[1] = st[0];
  }
}

// Whole cyclic-Jacobi solve in one workgroup (n <= JACOBI_WG_MAX): the same
// round-robin rotations as the multi-launch path, with barriers instead of
// launches; stops when the off-diagonal norm falls below tol * |A|_F, stops
// decreasing, or after max_sweeps.  LDS = true (n <= JACOBI_LDS_MAX): A and
// V live in LDS for the whole solve (dynamic shared memory of 2 n^2
// doubles) and are written back at the end.
constexpr int JACOBI_WG_MAX = 512, JACOBI_LDS_MAX = 64;
template <bool LDS>
__global__ __launch_bounds__(1024) void k_jacobi_small(int n, double* __restrict__ Ag,
                                                       double* __restrict__ Vg, double tol,
                                                       int max_sweeps, int* __restrict__ sweeps) {
  __shared__ double cs[JACOBI_WG_MAX];
  __shared__ int pq[JACOBI_WG_MAX];
  __shared__ double red[2][1024];
  __shared__ int stop;
  extern __shared__ double dyn[];
  const int t = threadIdx.x, nt = blockDim.x;
  const int m = n + (n & 1);
  const int h = m / 2;
  double* A = LDS ? dyn : Ag;
  double* V = LDS ? dyn + (int64_t)n * n : Vg;
  if (LDS)
    for (int64_t g = t; g < (int64_t)n * n; g += nt) A[g] = Ag[g];
  for (int64_t g = t; g < (int64_t)n * n; g += nt) V[g] = (g / n == g % n) ? 1.0 : 0.0;
  double prev_off = INFINITY;
  int sw = 0;
  __syncthreads();
  for (; sw < max_sweeps; ++sw) {
    double off = 0.0, tot = 0.0;
    for (int64_t g = t; g < (int64_t)n * n; g += nt) {
      const double v = A[g];
      tot += v * v;
      if (g / n != g % n) off += v * v;
    }
    red[0][t] = off;
    red[1][t] = tot;
    __syncthreads();
    for (int w = nt / 2; w > 0; w >>= 1) {
      if (t < w) {
        red[0][t] += red[0][t + w];
        red[1][t] += red[1][t + w];
      }
      __syncthreads();
    }
    if (t == 0) {
      const double o = red[0][0], tt = red[1][0];
      // converged, or no longer decreasing (round-off floor)
      stop = (o <= tol * tol * tt || tt == 0.0 || m < 2 || (sw > 2 && !(o < prev_off))) ? 1 : 0;
    }
    prev_off = red[0][0];
    __syncthreads();
    if (stop) break;
    for (int step = 0; step < m - 1; ++step) {
      for (int k = t; k < h; k += nt) {
        int p = rr_player(k, step, m), q = rr_player(m - 1 - k, step, m);
        if (p > q) {
          const int tmp = p;
          p = q;
          q = tmp;
        }
        double c = 1.0, s = 0.0;
        if (q < n) {
          const double apq = A[(int64_t)p * n + q];
          if (apq != 0.0) {
            const double app = A[(int64_t)p * n + p], aqq = A[(int64_t)q * n + q];
            const double tau = (aqq - app) / (2.0 * apq);
            const double tt2 = (tau >= 0.0 ? 1.0 : -1.0) / (fabs(tau) + sqrt(1.0 + tau * tau));
            c = 1.0 / sqrt(1.0 + tt2 * tt2);
            s = tt2 * c;
          }
        }
        cs[2 * k] = c;
        cs[2 * k + 1] = s;
        pq[2 * k] = p;
        pq[2 * k + 1] = q;
      }
      __syncthreads();
      const int64_t work = (int64_t)h * h + (int64_t)n * h;
      for (int64_t g = t; g < work; g += nt) {
        if (g < (int64_t)h * h) {
          const int a = (int)(g / h), b = (int)(g % h);
          const int pa = pq[2 * a], qa = pq[2 * a + 1], pb = pq[2 * b], qb = pq[2 * b + 1];
          const double ca = cs[2 * a], sa = cs[2 * a + 1], cb = cs[2 * b], sb = cs[2 * b + 1];
          const bool ipa = pa < n, iqa = qa < n, ipb = pb < n, iqb = qb < n;
          const double m00 = (ipa && ipb) ? A[(int64_t)pa * n + pb] : 0.0;
          const double m01 = (ipa && iqb) ? A[(int64_t)pa * n + qb] : 0.0;
          const double m10 = (iqa && ipb) ? A[(int64_t)qa * n + pb] : 0.0;
          const double m11 = (iqa && iqb) ? A[(int64_t)qa * n + qb] : 0.0;
          const double r00 = ca * m00 - sa * m10, r01 = ca * m01 - sa * m11;
          const double r10 = sa * m00 + ca * m10, r11 = sa * m01 + ca * m11;
          if (ipa && ipb) A[(int64_t)pa * n + pb] = cb * r00 - sb * r01;
          if (ipa && iqb) A[(int64_t)pa * n + qb] = sb * r00 + cb * r01;
          if (iqa && ipb) A[(int64_t)qa * n + pb] = cb * r10 - sb * r11;
          if (iqa && iqb) A[(int64_t)qa * n + qb] = sb * r10 + cb * r11;
        } else {
          const int64_t gg = g - (int64_t)h * h;
          const int i = (int)(gg / h), a = (int)(gg % h);
          const int pa = pq[2 * a], qa = pq[2 * a + 1];
          if (qa < n) {
            const double ca = cs[2 * a], sa = cs[2 * a + 1];
            const double vp = V[(int64_t)i * n + pa], vq = V[(int64_t)i * n + qa];
            V[(int64_t)i * n + pa] = ca * vp - sa * vq;
            V[(int64_t)i * n + qa] = sa * vp + ca * vq;
          }
        }
      }
      __syncthreads();
    }
  }
  if (LDS) {
    __syncthreads();
    for (int64_t g = t; g < (int64_t)n * n; g += nt) {
      Ag[g] = A[g];
      Vg[g] = V[g];
    }
  }
  if (t == 0 && sweeps) *sweeps = sw;
}

// Block Jacobi (large n): the indices are cut into blocks of BJ_B, and the
// blocks play the round-robin tournament the scalar form plays with single
// indices.  At each step every pair of blocks (I, J) diagonalises its own
// 2 BJ_B x 2 BJ_B submatrix (k_bjac_solve: BJ_INNER cyclic sweeps in LDS,
// the accumulated rotation then permuted so that the pair's diagonal is in
// ascending order, smallest values into block I, as a full eigensolver of the
// submatrix would order them), and one launch applies every pair's rotation
// R to the whole matrix, A <- P^T A P and V <- V P with P the block-diagonal
// (after the pairing permutation) of the R (k_bjac_apply).  A sweep is
// mb - 1 steps instead of n - 1, each reading A and V once.  The ordering
// matters for convergence: without it the couplings inside a cluster of
// equal eigenvalues (the null space of a rank-deficient metric) decay
// slowly, with it the clusters gather into blocks and the sweep count is
// that of an exact inner solve.
constexpr int BJ_B = 16, BJ_P = 2 * BJ_B, BJ_INNER = 2;

// local index l (0 .. BJ_P - 1) of the pair (I, J) -> global index
__device__ inline int bj_index(int l, int I, int J) { return l < BJ_B ? I * BJ_B + l : J * BJ_B + (l - BJ_B); }

// 1/x for a normal x: the hardware estimate and two Newton steps
__device__ inline double bj_rcp(double x) {
  double y = __builtin_amdgcn_rcp(x);
  double e = fma(-x, y, 1.0);
  y = fma(y, e, y);
  e = fma(-x, y, 1.0);
  return fma(y, e, y);
}

// 1/sqrt(x) for x in [1, 2]: the hardware estimate and two Newton steps
__device__ inline double bj_rsq(double x) {
  const double h = 0.5 * x;
  double y = __builtin_amdgcn_rsq(x);
  y = y * fma(-h * y, y, 1.5);
  return y * fma(-h * y, y, 1.5);
}

// Jacobi rotation (c, s) that annihilates apq, t = tan(theta) the root of
// t^2 + 2 tau t - 1 = 0 of smaller magnitude, tau = (aqq - app) / (2 apq),
// written in |aqq - app| and 2 |apq| scaled by their maximum so that every
// intermediate stays in [1, 2.5] (no overflow for a tiny apq, no IEEE
// divide or square root: hardware estimates refined by Newton steps); an
// |apq| below 1e-290 (or NaN) gives no rotation.  Straight-line code, so that
// the two rotations a thread needs are computed side by side.
__device__ inline void bj_rotation(double app, double aqq, double apq, double& c, double& s) {
  const double d = aqq - app, b = 2.0 * apq;
  const bool skip = !(fabs(b) >= 1e-290);
  const double bs = skip ? 1.0 : b;
  const double rm = bj_rcp(fmax(fabs(d), fabs(bs)));
  const double d1 = fabs(d) * rm, b1 = fabs(bs) * rm;   // the larger is 1
  const double q = fma(d1, d1, b1 * b1);                // [1, 2]
  const double tt = b1 * bj_rcp(d1 + q * bj_rsq(q));   // |t| <= 1
  const double t = ((d < 0.0) != (bs < 0.0) && d != 0.0) ? -tt : tt;   // sign of tau, + for tau = 0
  const double cc = bj_rsq(fma(t, t, 1.0));
  c = skip ? 1.0 : cc;
  s = skip ? 0.0 : t * cc;
}

// one workgroup per pair of blocks: R[k] (BJ_P x BJ_P, row-major) rotates the
// pair's local indices; indices >= n are left alone (zero rows and columns,
// identity in R).  Thread (a, b) owns the 2 x 2 block of S at the index pairs
// a and b of the inner step and the entries (b, a), (b + BJ_B, a) of Q's
// column pairs; it computes the two rotations itself (the 16 threads that
// need a rotation compute the same one) from the previous S, and writes the
// next S to the other buffer: one barrier per inner step.
constexpr int BJ_SOLVE_THREADS = BJ_B * BJ_B;
__global__ __launch_bounds__(BJ_SOLVE_THREADS) void k_bjac_solve(int n, int mb, int step,
                                                                 const double* __restrict__ A,
                                                                 double* __restrict__ R) {
  __shared__ double S[2][BJ_P][BJ_P + 1], Q[BJ_P][BJ_P + 1];
  __shared__ int perm[BJ_P];
  __shared__ double dg[BJ_P];
  const int t = threadIdx.x, k = blockIdx.x;
  const int a = t / BJ_B, b = t % BJ_B;
  int I, J;
  jac_pair(k, step, mb, I, J);
  for (int e = t; e < BJ_P * BJ_P; e += blockDim.x) {
    const int r = e / BJ_P, c = e % BJ_P;
    const int gr = bj_index(r, I, J), gc = bj_index(c, I, J);
    S[0][r][c] = (gr < n && gc < n) ? A[(int64_t)gr * n + gc] : 0.0;
    Q[r][c] = r == c ? 1.0 : 0.0;
  }
  if (t < BJ_P) perm[t] = t;
  __syncthreads();
  int cur = 0;
  for (int sw = 0; sw < BJ_INNER; ++sw) {
    for (int st = 0; st < BJ_P - 1; ++st) {
      int pa, qa, pb, qb;
      jac_pair(a, st, BJ_P, pa, qa);
      jac_pair(b, st, BJ_P, pb, qb);
      const double(*Sc)[BJ_P + 1] = S[cur];
      double(*Sn)[BJ_P + 1] = S[cur ^ 1];
      double ca, sa, cb, sb;
      bj_rotation(Sc[pa][pa], Sc[qa][qa], Sc[pa][qa], ca, sa);
      bj_rotation(Sc[pb][pb], Sc[qb][qb], Sc[pb][qb], cb, sb);
      const double m00 = Sc[pa][pb], m01 = Sc[pa][qb], m10 = Sc[qa][pb], m11 = Sc[qa][qb];
      const double r00 = ca * m00 - sa * m10, r01 = ca * m01 - sa * m11;
      const double r10 = sa * m00 + ca * m10, r11 = sa * m01 + ca * m11;
      Sn[pa][pb] = cb * r00 - sb * r01;
      Sn[pa][qb] = sb * r00 + cb * r01;
      Sn[qa][pb] = cb * r10 - sb * r11;
      Sn[qa][qb] = sb * r10 + cb * r11;
#pragma unroll
      for (int i = b; i < BJ_P; i += BJ_B) {
        const double vp = Q[i][pa], vq = Q[i][qa];
        Q[i][pa] = ca * vp - sa * vq;
        Q[i][qa] = sa * vp + ca * vq;
      }
      cur ^= 1;
      __syncthreads();
    }
  }
  const double(*Sf)[BJ_P + 1] = S[cur];
  double(*Sw)[BJ_P + 1] = S[cur ^ 1];   // free: the Q^T Q product below
  // one Newton-Schulz step towards the nearest orthogonal matrix, Q <- Q (3 -
  // Q^T Q) / 2: the accumulated rotations are orthogonal only to a few ulps,
  // with a bias of one sign on the diagonal of Q^T Q, and A and V take one
  // such Q per step (hundreds per solve), which would otherwise add up to
  // a drift of the eigenvalues well above the stopping bound
  if (t < BJ_P) dg[t] = Sf[t][t];
  {
    constexpr int RS = BJ_SOLVE_THREADS / BJ_P, OPT = BJ_P / RS;   // row stride, outputs per thread
    const int j = t % BJ_P, i0 = t / BJ_P;
    double acc[OPT];
#pragma unroll
    for (int m = 0; m < OPT; ++m) {
      const int i = i0 + RS * m;
      double g = 0.0;
      for (int r = 0; r < BJ_P; ++r) g += Q[r][i] * Q[r][j];
      acc[m] = g;
    }
#pragma unroll
    for (int m = 0; m < OPT; ++m) Sw[i0 + RS * m][j] = acc[m];
    __syncthreads();
#pragma unroll
    for (int m = 0; m < OPT; ++m) {
      const int i = i0 + RS * m;
      double g = 0.0;
      for (int c = 0; c < BJ_P; ++c) g += Q[i][c] * Sw[c][j];
      acc[m] = 1.5 * Q[i][j] - 0.5 * g;
    }
    __syncthreads();
#pragma unroll
    for (int m = 0; m < OPT; ++m) Q[i0 + RS * m][j] = acc[m];
    __syncthreads();
  }
  // ascending diagonal over the pair's valid positions ([0, vI) of block I,
  // then [BJ_B, BJ_B + vJ) of block J); ties keep the local order
  if (t < BJ_P && bj_index(t, I, J) < n) {
    const int vI = min(max(n - I * BJ_B, 0), BJ_B);
    const double d = dg[t];
    int rank = 0;
    for (int m = 0; m < BJ_P; ++m)
      if (bj_index(m, I, J) < n && (dg[m] < d || (dg[m] == d && m < t))) ++rank;
    perm[rank < vI ? rank : BJ_B + rank - vI] = t;
  }
  __syncthreads();
  for (int e = t; e < BJ_P * BJ_P; e += blockDim.x) {
    const int r = e / BJ_P, c = e % BJ_P;
    R[(int64_t)k * BJ_P * BJ_P + e] = Q[r][perm[c]];
  }
}

// A <- P^T A P and V <- V P for the rotations R of step `step`.  Workgroups
// [0, nA): the tile of rows of pair k1 and columns of pair k2 (k1 <= k2),
// R[k1]^T A R[k2], written to both mirrored positions (A stays exactly
// symmetric; the mirror goes through LDS so that both writes are row
// segments); the rest: 32 rows of V by the columns of one pair.  The tiles
// of one step partition A and V, so every element has one owner.  The
// 32 x 32 products run on FP64 MFMA, one 16 x 16 output tile per wave.
__global__ __launch_bounds__(256) void k_bjac_apply(int n, int mb, int step, double* __restrict__ A,
                                                    double* __restrict__ V, const double* __restrict__ R) {
  __shared__ double X[BJ_P][BJ_P + 1], T[BJ_P][BJ_P + 1], R1[BJ_P][BJ_P + 1], R2[BJ_P][BJ_P + 1];
  const int t = threadIdx.x, lane = t & 63, wv = t >> 6, nh = mb / 2;
  const int ti = (wv >> 1) * 16, tj = (wv & 1) * 16;   // this wave's output tile
  const int li = lane & 15, lk = lane >> 4;
  const int64_t nA = (int64_t)nh * (nh + 1) / 2;
  const int64_t g = blockIdx.x;
  if (g < nA) {
    int k1 = 0;
    int64_t rem = g;
    while (rem >= nh - k1) {
      rem -= nh - k1;
      ++k1;
    }
    const int k2 = k1 + (int)rem;
    int I1, J1, I2, J2;
    jac_pair(k1, step, mb, I1, J1);
    jac_pair(k2, step, mb, I2, J2);
    for (int e = t; e < BJ_P * BJ_P; e += blockDim.x) {
      const int r = e / BJ_P, c = e % BJ_P;
      const int gr = bj_index(r, I1, J1), gc = bj_index(c, I2, J2);
      X[r][c] = (gr < n && gc < n) ? A[(int64_t)gr * n + gc] : 0.0;
      R1[r][c] = R[(int64_t)k1 * BJ_P * BJ_P + e];
      R2[r][c] = R[(int64_t)k2 * BJ_P * BJ_P + e];
    }
    __syncthreads();
    d4 acc = {0.0, 0.0, 0.0, 0.0};
    for (int k0 = 0; k0 < BJ_P; k0 += 4)   // T = R1^T X
      acc = __builtin_amdgcn_mfma_f64_16x16x4f64(R1[k0 + lk][ti + li], X[k0 + lk][tj + li], acc, 0, 0, 0);
#pragma unroll
    for (int v = 0; v < 4; ++v) T[ti + lk + 4 * v][tj + li] = acc[v];
    __syncthreads();
    acc = d4{0.0, 0.0, 0.0, 0.0};
    for (int k0 = 0; k0 < BJ_P; k0 += 4)   // Y = T R2
      acc = __builtin_amdgcn_mfma_f64_16x16x4f64(T[ti + li][k0 + lk], R2[k0 + lk][tj + li], acc, 0, 0, 0);
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int i = ti + lk + 4 * v, j = tj + li;
      X[i][j] = acc[v];   // X is free after the first product
      const int gr = bj_index(i, I1, J1), gc = bj_index(j, I2, J2);
      if (gr < n && gc < n) A[(int64_t)gr * n + gc] = acc[v];
    }
    if (k1 == k2) return;
    __syncthreads();
    // mirror: A[gc][gr] = Y[i][j], consecutive threads along i
    for (int e = t; e < BJ_P * BJ_P; e += blockDim.x) {
      const int i = e % BJ_P, j = e / BJ_P;
      const int gr = bj_index(i, I1, J1), gc = bj_index(j, I2, J2);
      if (gr < n && gc < n) A[(int64_t)gc * n + gr] = X[i][j];
    }
  } else {
    const int64_t gv = g - nA;
    const int rt = (int)(gv / nh), k = (int)(gv % nh);
    int I, J;
    jac_pair(k, step, mb, I, J);
    for (int e = t; e < BJ_P * BJ_P; e += blockDim.x) {
      const int r = e / BJ_P, c = e % BJ_P;
      const int gr = rt * BJ_P + r, gc = bj_index(c, I, J);
      X[r][c] = (gr < n && gc < n) ? V[(int64_t)gr * n + gc] : 0.0;
      R1[r][c] = R[(int64_t)k * BJ_P * BJ_P + e];
    }
    __syncthreads();
    d4 acc = {0.0, 0.0, 0.0, 0.0};
    for (int k0 = 0; k0 < BJ_P; k0 += 4)   // V X R
      acc = __builtin_amdgcn_mfma_f64_16x16x4f64(X[ti + li][k0 + lk], R1[k0 + lk][tj + li], acc, 0, 0, 0);
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int gr = rt * BJ_P + ti + lk + 4 * v, gc = bj_index(tj + li, I, J);
      if (gr < n && gc < n) V[(int64_t)gr * n + gc] = acc[v];
    }
  }
}

// F^ref_MN = sum_rs f_rs (G[M][N][r][s] + G[N][M][r][s]) / 2: the Fock
// operator in the reference space (Eq. 3) from the transition one-particle
// densities, symmetrised; one thread per (M, N)
__global__ void k_xms_fref(int na, int nst, const double* __restrict__ f, const double* __restrict__ G,
                           double* __restrict__ F) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= nst * nst) return;
  const int M = t / nst, N = t % nst;
  const int64_t nf = (int64_t)na * na;
  const double* gmn = G + ((int64_t)M * nst + N) * nf;
  const double* gnm = G + ((int64_t)N * nst + M) * nf;
  double acc = 0.0;
  for (int64_t k = 0; k < nf; ++k) acc += f[k] * (gmn[k] + gnm[k]);
  F[t] = 0.5 * acc;
}

hipError_t xms_fref(int na, int nst, const double* f, const double* G, double* F, hipStream_t s) {
  if (nst <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_xms_fref, dim3(cdiv((int64_t)nst * nst, 64)), dim3(64), 0, s, na, nst, f, G, F);
  return hipGetLastError();
}

hipError_t jacobi_eigh(int n, double* A, double* V, double* ws, int max_sweeps, double tol,
                       hipStream_t s, int* sweeps_done, int method, double* A2, double* hpin,
                       double abs_tol) {
  if (n <= 0) return hipSuccess;
  if (!hpin) return hipErrorInvalidValue;
  // the attainable off-diagonal norm grows with n (round-off of the rotations)
  tol = fmax(tol, 4e-16 * (double)n);
  if (method == 0 || method == 1) {
    // the LDS form needs 2 n^2 doubles of dynamic LDS beside its static arrays
    int dev = 0, lds_max = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e == hipSuccess) e = hipDeviceGetAttribute(&lds_max, hipDeviceAttributeMaxSharedMemoryPerBlock, dev);
    if (e != hipSuccess) return e;
    const size_t need = 2 * (size_t)n * n * sizeof(double) + 24 * 1024;
    const bool lds_ok = n <= JACOBI_LDS_MAX && need <= (size_t)lds_max;
    if (method == 1 && !lds_ok) return hipErrorInvalidValue;
    if (method == 0) method = lds_ok ? 1 : n <= JACOBI_WG_AUTO ? 2 : n >= JACOBI_BLOCK_MIN ? 5 : 3;
  }
  if (method == 2 && n > JACOBI_WG_MAX) return hipErrorInvalidValue;
  if (method < 0 || method > 5) return hipErrorInvalidValue;
  if (method == 1 || method == 2) {
    int* dsw = reinterpret_cast<int*>(ws + 2 * n + 8);
    if (method == 1)
      hipLaunchKernelGGL(k_jacobi_small<true>, dim3(1), dim3(1024), 2 * (size_t)n * n * sizeof(double), s, n,
                         A, V, tol, max_sweeps, dsw);
    else
      hipLaunchKernelGGL(k_jacobi_small<false>, dim3(1), dim3(1024), 0, s, n, A, V, tol, max_sweeps, dsw);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    if (sweeps_done) {
      e = hipMemcpyAsync(hpin, dsw, sizeof(int), hipMemcpyDeviceToHost, s);
      if (e != hipSuccess) return e;
      e = hipStreamSynchronize(s);
      if (e != hipSuccess) return e;
      std::memcpy(sweeps_done, hpin, sizeof(int));
    }
    return hipSuccess;
  }
  const int m = n + (n & 1);
  // workspace (doubles): cs [2m] | norms [2] + pad [2] | pq [m ints] | partials [2 JAC_NORM_WG]
  double* cs = ws;
  double* norms = ws + 2 * m;
  int* pq = reinterpret_cast<int*>(ws + 2 * m + 4);
  double* npart = ws + 2 * m + 4 + (m + 1) / 2 + 1;
  double* Rb = npart + 2 * JAC_NORM_WG;   // block form: bjac_pairs(n) rotations of BJ_P x BJ_P
  const int nbn = (int)std::min<int64_t>(JAC_NORM_WG, std::max<int64_t>(1, cdiv((int64_t)n * n, 256 * 16)));
  hipLaunchKernelGGL(k_eye, dim3(cdiv((int64_t)n * n, 256)), dim3(256), 0, s, n, V);
  int sw = 0;
  double prev = INFINITY;
  for (; sw < max_sweeps; ++sw) {
    hipLaunchKernelGGL(k_jac_norms_part, dim3(nbn), dim3(256), 0, s, n, (const double*)A, npart);
    hipLaunchKernelGGL(k_jac_norms_fin, dim3(1), dim3(256), 0, s, nbn, (const double*)npart, norms);
    hipError_t e = hipMemcpyAsync(hpin, norms, 2 * sizeof(double), hipMemcpyDeviceToHost, s);
    if (e != hipSuccess) return e;
    e = hipStreamSynchronize(s);
    if (e != hipSuccess) return e;
    const double off = hpin[0], tot = hpin[1];
    // converged, or at the round-off floor (the off-diagonal norm no longer
    // decreases); a sweep that decreases it only a little is not the floor:
    // a large cluster of zero eigenvalues (rank-deficient metrics) keeps the
    // couplings of the cluster to the rest converging slowly
    const bool small = off <= tol * tol * tot && (abs_tol <= 0.0 || off <= abs_tol * abs_tol);
    if (small || tot == 0.0 || m < 2 || (sw > 2 && !(off < prev))) break;
    prev = off;
    if (method == 5) {
      const int nb = (n + BJ_B - 1) / BJ_B, mb = nb + (nb & 1), nh = mb / 2;
      const int64_t nwg = (int64_t)nh * (nh + 1) / 2 + (int64_t)cdiv(n, BJ_P) * nh;
      for (int step = 0; step < mb - 1; ++step) {
        hipLaunchKernelGGL(k_bjac_solve, dim3(nh), dim3(BJ_SOLVE_THREADS), 0, s, n, mb, step, (const double*)A, Rb);
        hipLaunchKernelGGL(k_bjac_apply, dim3((unsigned)nwg), dim3(256), 0, s, n, mb, step, A, V, (const double*)Rb);
      }
      continue;
    }
    const int64_t work = (int64_t)(m / 2) * (m / 2) + (int64_t)n * (m / 2);
    if (A2) {
      // one launch per step, alternating buffers; an odd step count leaves
      // the sweep's result in A2, copied back below
      double* cur = A;
      double* nxt = A2;
      for (int step = 0; step < m - 1; ++step) {
        hipLaunchKernelGGL(k_jac_step, dim3(cdiv(work, 256)), dim3(256), 0, s, n, m, step, (const double*)cur,
                           nxt, V);
        double* t = cur;
        cur = nxt;
        nxt = t;
      }
      if (cur != A) {
        e = hipMemcpyAsync(A, cur, (size_t)n * n * sizeof(double), hipMemcpyDeviceToDevice, s);
        if (e != hipSuccess) return e;
      }
    } else {
      for (int step = 0; step < m - 1; ++step) {
        hipLaunchKernelGGL(k_jac_params, dim3(cdiv(m / 2, 128)), dim3(128), 0, s, n, m, step, A, cs,
                           pq);
        hipLaunchKernelGGL(k_jac_apply, dim3(cdiv(work, 256)), dim3(256), 0, s, n, m, A, V, cs, pq);
      }
    }
  }
  if (sweeps_done) *sweeps_done = sw;
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// vectors
// ---------------------------------------------------------------------------
template <typename T>
__global__ void k_dot_partial(int64_t n, const T* __restrict__ x, const T* __restrict__ y,
                              double* __restrict__ partial) {
  __shared__ double sh[256];
  double acc = 0.0;
  for (int64_t g = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; g < n;
       g += (int64_t)gridDim.x * blockDim.x)
    acc += (double)x[g] * (double)y[g];
  sh[threadIdx.x] = acc;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (threadIdx.x < w) sh[threadIdx.x] += sh[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) partial[blockIdx.x] = sh[0];
}

__global__ void k_sum_final(int np, const double* __restrict__ partial, double* __restrict__ out) {
  __shared__ double sh[256];
  double acc = 0.0;
  for (int i = threadIdx.x; i < np; i += blockDim.x) acc += partial[i];
  sh[threadIdx.x] = acc;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (threadIdx.x < w) sh[threadIdx.x] += sh[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) out[0] = sh[0];
}

// FP64 accumulation for either element type; fixed grid so the summation
// order is the same on every call
template <typename T>
hipError_t vec_dot(int64_t n, const T* x, const T* y, double* partial, double* out, hipStream_t s) {
  const int nb = 1024;
  hipLaunchKernelGGL(k_dot_partial<T>, dim3(nb), dim3(256), 0, s, n, x, y, partial);
  hipLaunchKernelGGL(k_sum_final, dim3(1), dim3(256), 0, s, nb, partial, out);
  return hipGetLastError();
}
template hipError_t vec_dot<double>(int64_t, const double*, const double*, double*, double*,
                                    hipStream_t);
template hipError_t vec_dot<float>(int64_t, const float*, const float*, double*, double*,
                                   hipStream_t);

__global__ void k_min_partial(int64_t n, const double* __restrict__ x, double* __restrict__ partial) {
  __shared__ double sh[256];
  double acc = INFINITY;
  for (int64_t g = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; g < n;
       g += (int64_t)gridDim.x * blockDim.x)
    acc = fmin(acc, x[g]);
  sh[threadIdx.x] = acc;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (threadIdx.x < w) sh[threadIdx.x] = fmin(sh[threadIdx.x], sh[threadIdx.x + w]);
    __syncthreads();
  }
  if (threadIdx.x == 0) partial[blockIdx.x] = sh[0];
}

__global__ void k_min_final(int np, const double* __restrict__ partial, double* __restrict__ out) {
  __shared__ double sh[256];
  double acc = INFINITY;
  for (int i = threadIdx.x; i < np; i += blockDim.x) acc = fmin(acc, partial[i]);
  sh[threadIdx.x] = acc;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (threadIdx.x < w) sh[threadIdx.x] = fmin(sh[threadIdx.x], sh[threadIdx.x + w]);
    __syncthreads();
  }
  if (threadIdx.x == 0) out[0] = sh[0];
}

hipError_t vec_min(int64_t n, const double* x, double* partial, double* out, hipStream_t s) {
  const int nb = 1024;
  hipLaunchKernelGGL(k_min_partial, dim3(nb), dim3(256), 0, s, n, x, partial);
  hipLaunchKernelGGL(k_min_final, dim3(1), dim3(256), 0, s, nb, partial, out);
  return hipGetLastError();
}

// element-wise kernels; X is the input element type, Y the output one
#define CASPT2_ELEMENTWISE(NAME, EXPR)                                                        \
  template <typename X, typename Y>                                                          \
  __global__ void k_##NAME(int64_t n, double a, const X* __restrict__ x,                     \
                           const Y* __restrict__ d, Y* __restrict__ y) {                     \
    for (int64_t g = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; g < n;                 \
         g += (int64_t)gridDim.x * blockDim.x) {                                             \
      EXPR;                                                                                  \
    }                                                                                        \
  }

CASPT2_ELEMENTWISE(axpy, y[g] += (Y)(a * x[g]))
CASPT2_ELEMENTWISE(xpay, y[g] = x[g] + (Y)a * y[g])
CASPT2_ELEMENTWISE(div, y[g] = x[g] / d[g])
CASPT2_ELEMENTWISE(scale_copy, y[g] = (Y)(a * x[g]))
CASPT2_ELEMENTWISE(fill, y[g] = (Y)a)
CASPT2_ELEMENTWISE(negsum, y[g] = -(x[g] + y[g]))

static inline unsigned egrid(int64_t n) {
  unsigned g = cdiv(n, 256);
  return g > 65536 ? 65536 : (g == 0 ? 1 : g);
}

template <typename X, typename Y>
hipError_t vec_axpy(int64_t n, double a, const X* x, Y* y, hipStream_t s) {
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL((k_axpy<X, Y>), dim3(egrid(n)), dim3(256), 0, s, n, a, x, (const Y*)nullptr, y);
  return hipGetLastError();
}
template <typename T>
hipError_t vec_xpay(int64_t n, const T* x, double a, T* y, hipStream_t s) {
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL((k_xpay<T, T>), dim3(egrid(n)), dim3(256), 0, s, n, a, x, (const T*)nullptr, y);
  return hipGetLastError();
}
hipError_t vec_negsum(int64_t n, const double* x, double* y, hipStream_t s) {
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL((k_negsum<double, double>), dim3(egrid(n)), dim3(256), 0, s, n, 0.0, x,
                     (const double*)nullptr, y);
  return hipGetLastError();
}
template <typename T>
hipError_t vec_div(int64_t n, const T* x, const T* d, T* y, hipStream_t s) {
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL((k_div<T, T>), dim3(egrid(n)), dim3(256), 0, s, n, 0.0, x, d, y);
  return hipGetLastError();
}
template <typename X, typename Y>
hipError_t vec_scale_copy(int64_t n, double a, const X* x, Y* y, hipStream_t s) {
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL((k_scale_copy<X, Y>), dim3(egrid(n)), dim3(256), 0, s, n, a, x, (const Y*)nullptr,
                     y);
  return hipGetLastError();
}
template <typename T>
hipError_t vec_fill(int64_t n, double v, T* y, hipStream_t s) {
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL((k_fill<T, T>), dim3(egrid(n)), dim3(256), 0, s, n, v, (const T*)nullptr,
                     (const T*)nullptr, y);
  return hipGetLastError();
}
template hipError_t vec_axpy<double, double>(int64_t, double, const double*, double*, hipStream_t);
template hipError_t vec_axpy<float, float>(int64_t, double, const float*, float*, hipStream_t);
template hipError_t vec_axpy<float, double>(int64_t, double, const float*, double*, hipStream_t);
template hipError_t vec_xpay<double>(int64_t, const double*, double, double*, hipStream_t);
template hipError_t vec_xpay<float>(int64_t, const float*, double, float*, hipStream_t);
template hipError_t vec_div<double>(int64_t, const double*, const double*, double*, hipStream_t);
template hipError_t vec_div<float>(int64_t, const float*, const float*, float*, hipStream_t);
template hipError_t vec_scale_copy<double, double>(int64_t, double, const double*, double*,
                                                   hipStream_t);
template hipError_t vec_scale_copy<double, float>(int64_t, double, const double*, float*,
                                                  hipStream_t);
template hipError_t vec_scale_copy<float, float>(int64_t, double, const float*, float*, hipStream_t);
template hipError_t vec_fill<double>(int64_t, double, double*, hipStream_t);
template hipError_t vec_fill<float>(int64_t, double, float*, hipStream_t);

// ---------------------------------------------------------------------------
// small symmetric eigenproblem (n <= 16) on a single thread: cyclic Jacobi,
// ascending values, eigenvector columns with largest-magnitude entry positive
// ---------------------------------------------------------------------------
__global__ void k_small_eigh(int n, const double* __restrict__ Ain, double* __restrict__ w,
                             double* __restrict__ R) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  double A[16][16], Vm[16][16];
  for (int i = 0; i < n; ++i)
    for (int j = 0; j < n; ++j) {
      A[i][j] = 0.5 * (Ain[i * n + j] + Ain[j * n + i]);
      Vm[i][j] = i == j ? 1.0 : 0.0;
    }
  for (int sweep = 0; sweep < 60; ++sweep) {
    double off = 0.0, tot = 0.0;
    for (int i = 0; i < n; ++i)
      for (int j = 0; j < n; ++j) {
        tot += A[i][j] * A[i][j];
        if (i != j) off += A[i][j] * A[i][j];
      }
    if (off <= 1e-34 * tot || off == 0.0) break;
    for (int p = 0; p < n - 1; ++p)
      for (int q = p + 1; q < n; ++q) {
        const double apq = A[p][q];
        if (apq == 0.0) continue;
        const double tau = (A[q][q] - A[p][p]) / (2.0 * apq);
        const double t = (tau >= 0.0 ? 1.0 : -1.0) / (fabs(tau) + sqrt(1.0 + tau * tau));
        const double c = 1.0 / sqrt(1.0 + t * t), s = t * c;
        for (int k = 0; k < n; ++k) {
          const double akp = A[k][p], akq = A[k][q];
          A[k][p] = c * akp - s * akq;
          A[k][q] = s * akp + c * akq;
        }
        for (int k = 0; k < n; ++k) {
          const double apk = A[p][k], aqk = A[q][k];
          A[p][k] = c * apk - s * aqk;
          A[q][k] = s * apk + c * aqk;
        }
        for (int k = 0; k < n; ++k) {
          const double vkp = Vm[k][p], vkq = Vm[k][q];
          Vm[k][p] = c * vkp - s * vkq;
          Vm[k][q] = s * vkp + c * vkq;
        }
      }
  }
  int order[16];
  for (int i = 0; i < n; ++i) order[i] = i;
  for (int i = 0; i < n; ++i)
    for (int j = i + 1; j < n; ++j)
      if (A[order[j]][order[j]] < A[order[i]][order[i]]) {
        const int t = order[i];
        order[i] = order[j];
        order[j] = t;
      }
  for (int c = 0; c < n; ++c) {
    const int k = order[c];
    w[c] = A[k][k];
    int imax = 0;
    for (int i = 1; i < n; ++i)
      if (fabs(Vm[i][k]) > fabs(Vm[imax][k])) imax = i;
    const double sg = Vm[imax][k] < 0.0 ? -1.0 : 1.0;
    for (int i = 0; i < n; ++i) R[i * n + c] = sg * Vm[i][k];
  }
}

hipError_t small_eigh(int n, const double* A, double* w, double* R, hipStream_t s) {
  if (n <= 0 || n > 16) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_small_eigh, dim3(1), dim3(64), 0, s, n, A, w, R);
  return hipGetLastError();
}

}  // namespace caspt2
