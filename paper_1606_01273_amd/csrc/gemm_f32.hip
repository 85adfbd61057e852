// FP32 GEMMs for the inner solver of the mixed-precision mode: the basis
// transforms and the GEMMs of the Fock couplings (SIMT), and the dense
// residual of the blocks with a wide active index (MFMA, below).  The SIMT
// kernel works on 64 x 64 output tiles, K staged
// through LDS in steps of 16; each of the 256 threads owns a 4 x 4 sub-tile
// strided by 16 in both directions, so LDS reads are broadcasts or
// conflict-free.
#include "kernels.hpp"

namespace caspt2 {

namespace {

constexpr int TM = 64, TN = 64, TK = 16, PAD = 4;

inline unsigned cdiv(int64_t a, int64_t b) { return (unsigned)((a + b - 1) / b); }

// grid of tiles: the dimension with more tiles on x; false when neither
// orientation fits the 65535 limit of grid y and z
inline bool tile_grid(int64_t M, int64_t N, int batch, int tm, int tn, dim3* grid, int* m_on_x) {
  const int64_t tmn = (M + tm - 1) / tm, tnn = (N + tn - 1) / tn;
  *m_on_x = tmn >= tnn ? 1 : 0;
  const int64_t gx = *m_on_x ? tmn : tnn, gy = *m_on_x ? tnn : tmn;
  if (gy > 65535 || batch > 65535 || gx > 0x7fffffff) return false;
  *grid = dim3((unsigned)gx, (unsigned)gy, (unsigned)batch);
  return true;
}

template <bool B_NK, bool DUAL>
__global__ __launch_bounds__(256) void k_gemm_f32(int64_t M, int64_t N, int64_t K, float alpha,
                                                  const float* __restrict__ A, int64_t lda,
                                                  int64_t sA, const float* __restrict__ B,
                                                  int64_t ldb, int64_t sB,
                                                  const float* __restrict__ B2, float beta,
                                                  float* __restrict__ C, int64_t ldc, int64_t sC,
                                                  const float* __restrict__ dvec, float dshift,
                                                  const float* __restrict__ V, int64_t ldv,
                                                  int m_on_x) {
  __shared__ float As[TK][TM + PAD];
  __shared__ float Bs[TK][TN + PAD];
  __shared__ float B2s[DUAL ? TK : 1][TN + PAD];
  const int tid = threadIdx.x;
  const int tx = tid & 15, ty = tid >> 4;
  const int64_t bz = blockIdx.z;
  A += bz * sA;
  B += bz * sB;
  C += bz * sC;
  // the longer tile dimension runs on grid x (y and z are limited to 65535)
  const int64_t m0 = (int64_t)(m_on_x ? blockIdx.x : blockIdx.y) * TM;
  const int64_t n0 = (int64_t)(m_on_x ? blockIdx.y : blockIdx.x) * TN;
  float acc[4][4], acc2[4][4];
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      acc[i][j] = 0.f;
      acc2[i][j] = 0.f;
    }
  for (int64_t k0 = 0; k0 < K; k0 += TK) {
    {  // A tile: row r = tid / 4, k = 4 (tid % 4) + u
      const int r = tid >> 2, c = (tid & 3) * 4;
      const int64_t gm = m0 + r;
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const int64_t gk = k0 + c + u;
        As[c + u][r] = (gm < M && gk < K) ? A[gm * lda + gk] : 0.f;
      }
    }
    if (B_NK) {  // B is [N][K]
      const int r = tid >> 2, c = (tid & 3) * 4;
      const int64_t gn = n0 + r;
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const int64_t gk = k0 + c + u;
        Bs[c + u][r] = (gn < N && gk < K) ? B[gn * ldb + gk] : 0.f;
      }
    } else {  // B is [K][N]: k = tid / 16, n = 4 (tid % 16) + u
      const int kk = tid >> 4, c = (tid & 15) * 4;
      const int64_t gk = k0 + kk;
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const int64_t gn = n0 + c + u;
        const bool in = gn < N && gk < K;
        Bs[kk][c + u] = in ? B[gk * ldb + gn] : 0.f;
        if (DUAL) B2s[kk][c + u] = in ? B2[gk * ldb + gn] : 0.f;
      }
    }
    __syncthreads();
#pragma unroll
    for (int kk = 0; kk < TK; ++kk) {
      float a[4], b[4], b2[4];
#pragma unroll
      for (int i = 0; i < 4; ++i) a[i] = As[kk][ty + 16 * i];
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        b[j] = Bs[kk][tx + 16 * j];
        if (DUAL) b2[j] = B2s[kk][tx + 16 * j];
      }
#pragma unroll
      for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) {
          acc[i][j] = fmaf(a[i], b[j], acc[i][j]);
          if (DUAL) acc2[i][j] = fmaf(a[i], b2[j], acc2[i][j]);
        }
    }
    __syncthreads();
  }
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    const int64_t gm = m0 + ty + 16 * i;
    if (gm >= M) continue;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int64_t gn = n0 + tx + 16 * j;
      if (gn >= N) continue;
      if (DUAL) {
        float val = (dvec[gm] + dshift) * acc[i][j] + acc2[i][j];
        if (V) val += V[gm * ldv + gn];
        C[gm * ldc + gn] = val;
      } else {
        float val = alpha * acc[i][j];
        if (beta != 0.f) val += beta * C[gm * ldc + gn];
        C[gm * ldc + gn] = val;
      }
    }
  }
}

}  // namespace

hipError_t gemm_f32(bool b_is_nk, int64_t M, int64_t N, int64_t K, float alpha, const float* A,
                    int64_t lda, int64_t sA, const float* B, int64_t ldb, int64_t sB, float beta,
                    float* C, int64_t ldc, int64_t sC, int batch, hipStream_t s) {
  if (M <= 0 || N <= 0 || batch <= 0) return hipSuccess;
  dim3 grid;
  int mx;
  if (!tile_grid(M, N, batch, TM, TN, &grid, &mx)) return hipErrorInvalidValue;
  if (b_is_nk)
    hipLaunchKernelGGL((k_gemm_f32<true, false>), grid, dim3(256), 0, s, M, N, K, alpha, A, lda, sA,
                       B, ldb, sB, (const float*)nullptr, beta, C, ldc, sC, (const float*)nullptr,
                       0.f, (const float*)nullptr, (int64_t)0, mx);
  else
    hipLaunchKernelGGL((k_gemm_f32<false, false>), grid, dim3(256), 0, s, M, N, K, alpha, A, lda,
                       sA, B, ldb, sB, (const float*)nullptr, beta, C, ldc, sC,
                       (const float*)nullptr, 0.f, (const float*)nullptr, (int64_t)0, mx);
  return hipGetLastError();
}

// Dense residual of one entry in FP32 on MFMA (v_mfma_f32_16x16x4f32, FP32
// accumulation): C = V + (d + dshift) X S + X F with X [M][K], S, F [K][N].
// 64 x 64 output tiles, four waves of 32 x 32 (2 x 2 blocks of 16 x 16), K
// in steps of 16 through LDS with the next step's loads in registers while
// the current one is multiplied.  Operand layout of the instruction (lane l):
// A[i][k]: i = l % 16, k = l / 16; B[k][j]: j = l % 16, k = l / 16; the four
// results of a lane: D[4 (l / 16) + v][l % 16].
namespace {
typedef float f4 __attribute__((ext_vector_type(4)));
constexpr int MK = 16, MLD = MK + 1;
__global__ __launch_bounds__(256) void k_residual_mfma_f32(int64_t M, int64_t N, int64_t K,
                                                           const float* __restrict__ X, int64_t ldx,
                                                           const float* __restrict__ S,
                                                           const float* __restrict__ F,
                                                           const float* __restrict__ d, float dshift,
                                                           const float* __restrict__ V, int64_t ldv,
                                                           float* __restrict__ C, int64_t ldc, int m_on_x) {
  __shared__ float As[64][MLD];
  __shared__ float Bs[64][MLD];
  __shared__ float B2s[64][MLD];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm = wave >> 1, wn = wave & 1;
  const int64_t m0 = (int64_t)(m_on_x ? blockIdx.x : blockIdx.y) * 64;
  const int64_t n0 = (int64_t)(m_on_x ? blockIdx.y : blockIdx.x) * 64;
  f4 acc[2][2], acc2[2][2];
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j) {
      acc[i][j] = f4{0.f, 0.f, 0.f, 0.f};
      acc2[i][j] = f4{0.f, 0.f, 0.f, 0.f};
    }
  // per thread: A row r = tid / 4, k = 4 (tid % 4) .. + 3; B row k = tid / 16,
  // n = 4 (tid % 16) .. + 3
  const int ra = tid >> 2, ca = (tid & 3) * 4;
  const int kb = tid >> 4, cb = (tid & 15) * 4;
  const bool a_ok = m0 + ra < M;
  const float* pA = X + (a_ok ? m0 + ra : 0) * ldx + ca;
  float xa[4], xs[4], xf[4];
  auto load = [&](int64_t k0) {
    const bool full = k0 + MK <= K;
#pragma unroll
    for (int u = 0; u < 4; ++u) xa[u] = (a_ok && (full || k0 + ca + u < K)) ? pA[k0 + u] : 0.f;
    const bool krow = full || k0 + kb < K;
    const int64_t off = (k0 + kb) * N + n0 + cb;
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const bool in = krow && n0 + cb + u < N;
      xs[u] = in ? S[off + u] : 0.f;
      xf[u] = in ? F[off + u] : 0.f;
    }
  };
  if (K > 0) load(0);
  for (int64_t k0 = 0; k0 < K; k0 += MK) {
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      As[ra][ca + u] = xa[u];
      Bs[cb + u][kb] = xs[u];
      B2s[cb + u][kb] = xf[u];
    }
    __syncthreads();
    if (k0 + MK < K) load(k0 + MK);
#pragma unroll
    for (int kk = 0; kk < MK; kk += 4) {
      float a[2], b[2], b2[2];
#pragma unroll
      for (int i = 0; i < 2; ++i) a[i] = As[wm * 32 + i * 16 + (lane & 15)][kk + (lane >> 4)];
#pragma unroll
      for (int j = 0; j < 2; ++j) {
        b[j] = Bs[wn * 32 + j * 16 + (lane & 15)][kk + (lane >> 4)];
        b2[j] = B2s[wn * 32 + j * 16 + (lane & 15)][kk + (lane >> 4)];
      }
#pragma unroll
      for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j) {
          acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x4f32(a[i], b[j], acc[i][j], 0, 0, 0);
          acc2[i][j] = __builtin_amdgcn_mfma_f32_16x16x4f32(a[i], b2[j], acc2[i][j], 0, 0, 0);
        }
    }
    __syncthreads();
  }
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int64_t gm = m0 + wm * 32 + i * 16 + 4 * (lane >> 4) + v;
        const int64_t gn = n0 + wn * 32 + j * 16 + (lane & 15);
        if (gm < M && gn < N) {
          float val = (d[gm] + dshift) * acc[i][j][v] + acc2[i][j][v];
          if (V) val += V[gm * ldv + gn];
          C[gm * ldc + gn] = val;
        }
      }
}
}  // namespace

hipError_t residual_gemm_f32(int64_t M, int64_t N, int64_t K, const float* X, int64_t ldx,
                             const float* S, const float* F, const float* d, float dshift,
                             const float* V, int64_t ldv, float* C, int64_t ldc, hipStream_t s) {
  if (M <= 0 || N <= 0) return hipSuccess;
  dim3 grid;
  int mx;
  if (!tile_grid(M, N, 1, TM, TN, &grid, &mx)) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_residual_mfma_f32, grid, dim3(256), 0, s, M, N, K, X, ldx, S, F, d, dshift, V, ldv, C,
                     ldc, mx);
  return hipGetLastError();
}

}  // namespace caspt2
