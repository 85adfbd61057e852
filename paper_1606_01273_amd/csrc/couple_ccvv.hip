// The up coupling terms into ccvv (Fock couplings of Eq. 10 with the f of
// Eq. 11: ccvv <- cavv through f(active, closed), ccvv <- caav through
// f(virtual, closed), ccvv <- ccav through f(virtual, active)), added
// straight into the packed ccvv rows (+: i >= j, a >= b; -: i > j, a > b)
// instead of through the all-orderings sigma of ccvv.
//
// With sigma(i,j,a,b) the all-orderings contribution (columns c < ncol):
//   cavv:  sum_y f(y, j) [ W1(i,a,b) + W2(i,b,a) ](y, c),  W = X_cavv G^T
//   caav:  f(b, j) W5(i,a)(c) + f(a, j) W6(i,b)(c)
//   ccav:  sum_y f(b, y) W3(i,j,a)(y, c) + sum_y f(a, y) W4(i,j,b)(y, c)
// and the packed entries formed from the four images (i,j,a,b), (j,i,a,b),
// (i,j,b,a), (j,i,b,a) with the weights of the ccvv packing.  The cavv and
// caav terms fix the virtual pair and run over every closed pair (pass A, a
// workgroup per virtual pair group); the ccav terms fix the closed pair and
// run over virtual pairs (pass B, a workgroup per closed pair and 16 x 16
// tile of virtual pairs).  Each pass reads its inputs once per tile and
// adds into the packed rows once.
#include <cmath>

#include "device_common.hpp"
#include "kernels.hpp"

namespace caspt2 {

namespace {

constexpr int CUA_NB = 4;        // virtual pairs (a, b0 .. b0 + 3) per pass-A workgroup
constexpr int CUA_THREADS = 512;
constexpr int CUB_T = 16;        // pass-B virtual tile edge

__device__ inline void closed_pair(int q, int& i, int& j) {
  int ii = (int)((sqrt(8.0 * q + 1.0) - 1.0) * 0.5);
  while ((ii + 1) * (ii + 2) / 2 <= q) ++ii;
  while (ii * (ii + 1) / 2 > q) --ii;
  i = ii;
  j = q - ii * (ii + 1) / 2;
}

// the packed + and - entries of one ccvv element from its four images
template <typename T>
__device__ inline void pack_add(int i, int j, int a, int b, int64_t npv, int64_t nmv, int ncol, const double (&r1)[4],
                                const double (&r2)[4], const double (&r3)[4], const double (&r4)[4],
                                T* __restrict__ plus, T* __restrict__ minus) {
  const bool dij = i != j, dab = a != b;
  const double w = (dij && dab) ? 0.5 : ((dij || dab) ? 0.70710678118654752440 : 1.0);
  const int64_t rp = ((int64_t)i * (i + 1) / 2 + j) * npv + (int64_t)a * (a + 1) / 2 + b;
#pragma unroll
  for (int c = 0; c < 4; ++c) {
    if (c >= ncol) break;
    const double sp = r1[c] + (dij ? r2[c] : 0.0) + (dab ? r3[c] : 0.0) + ((dij && dab) ? r4[c] : 0.0);
    plus[rp * ncol + c] += (T)(w * sp);
  }
  if (dij && dab && minus) {
    const int64_t rm = ((int64_t)i * (i - 1) / 2 + j) * nmv + (int64_t)a * (a - 1) / 2 + b;
#pragma unroll
    for (int c = 0; c < 4; ++c)
      if (c < ncol) minus[rm * ncol + c] += (T)(0.5 * (r1[c] - r2[c] - r3[c] + r4[c]));
  }
}

}  // namespace

// Pass A.  Workgroup g: virtual index a and b_u = b0 + u (u < nb, b_u <= a)
// from groups[g] = a << 16 | b0.  Shared memory (doubles):
//   XU  [nb][2][nc][ldu]   cavv rows (i,a,b_u) (side 0) and (i,b_u,a) (side
//                          1), then overwritten with U = G1 X(side) + G2 X(other side);
//                          ldu = nak | 1 (odd: rows start on different banks)
//   Gt  [2][nak][nout]     G1^T, G2^T (nout = ny * ncol = nak)
//   fA  [ny][nc]           f(y, j)
//   fC  [1 + nb][nc]       f(v, j) for v = a, b_0 ..
//   W5s, W6s [1 + nb][nc][ncol]  W5(i, v), W6(i, v)
template <typename T>
__global__ __launch_bounds__(CUA_THREADS) void k_ccvv_up_vpair(CcvvUpArgs<T> p, const uint32_t* __restrict__ groups) {
  extern __shared__ double sm[];
  const int nc = p.nc, nv = p.nv, ncol = p.ncol, ny = p.ny, nak = p.nak, ldu = nak | 1;
  const uint32_t gv = groups[blockIdx.x];
  const int a = (int)(gv >> 16), b0 = (int)(gv & 0xffffu);
  const int nb = min(CUA_NB, a + 1 - b0);
  const int t = threadIdx.x;
  const bool havex = p.X != nullptr;
  double* XU = sm;
  double* Gt = XU + (havex ? (int64_t)CUA_NB * 2 * nc * ldu : 0);
  double* fA = Gt + (havex ? 2 * nak * nak : 0);
  double* fC = fA + (havex ? ny * nc : 0);
  double* W5s = fC + (p.fC ? (1 + CUA_NB) * nc : 0);
  double* W6s = W5s + (p.W5 ? (1 + CUA_NB) * nc * ncol : 0);
  auto vidx = [&](int v) { return v == 0 ? a : b0 + v - 1; };
  if (havex) {
    const int nrow = nb * 2 * nc;
    for (int e = t; e < nrow * nak; e += blockDim.x) {
      const int r = e / nak, k = e % nak;
      const int i = r % nc, side = (r / nc) & 1, u = r / (2 * nc);
      const int b = b0 + u;
      const int64_t row = side == 0 ? ((int64_t)i * nv + a) * nv + b : ((int64_t)i * nv + b) * nv + a;
      XU[r * ldu + k] = (double)p.X[row * nak + k];
    }
    for (int e = t; e < nak * nak; e += blockDim.x) {
      const int o = e / nak, k = e % nak;
      Gt[k * nak + o] = p.G1 ? (double)p.G1[e] : 0.0;
      Gt[nak * nak + k * nak + o] = p.G2 ? (double)p.G2[e] : 0.0;
    }
    for (int e = t; e < ny * nc; e += blockDim.x) fA[e] = p.fA[(e / nc) * p.fA_stride + e % nc];
  }
  if (p.fC)
    for (int e = t; e < (1 + nb) * nc; e += blockDim.x) fC[e] = p.fC[(int64_t)vidx(e / nc) * p.fC_stride + e % nc];
  if (p.W5 || p.W6)
    for (int e = t; e < (1 + nb) * nc * ncol; e += blockDim.x) {
      const int c = e % ncol, i = (e / ncol) % nc, v = e / (ncol * nc);
      const int64_t row = (int64_t)i * nv + vidx(v);
      if (p.W5) W5s[e] = (double)p.W5[row * ncol + c];
      if (p.W6) W6s[e] = (double)p.W6[row * ncol + c];
    }
  __syncthreads();
  if (havex) {
    // U in registers, then over X
    constexpr int MAXO = 16;   // outputs per thread: nb * 2 * nc * nak <= MAXO * blockDim (checked on the host)
    double acc[MAXO];
    const int nout = nb * 2 * nc * nak;
#pragma unroll
    for (int m = 0; m < MAXO; ++m) {
      acc[m] = 0.0;
      const int e = t + m * (int)blockDim.x;
      if (e < nout) {
        const int r = e / nak, o = e % nak;
        const int side = (r / nc) & 1;
        const double* xs = XU + (int64_t)r * ldu;                              // this side
        const double* xo = XU + (int64_t)(r + (side == 0 ? nc : -nc)) * ldu;   // the other side
        double s = 0.0;
        for (int k = 0; k < nak; ++k) s += Gt[k * nak + o] * xs[k] + Gt[nak * nak + k * nak + o] * xo[k];
        acc[m] = s;
      }
    }
    __syncthreads();
#pragma unroll
    for (int m = 0; m < MAXO; ++m) {
      const int e = t + m * (int)blockDim.x;
      if (e < nout) XU[(e / nak) * ldu + e % nak] = acc[m];
    }
    __syncthreads();
  }
  const int npc = nc * (nc + 1) / 2;
  const int64_t npv = (int64_t)nv * (nv + 1) / 2, nmv = (int64_t)nv * (nv - 1) / 2;
  for (int it = t; it < npc * nb; it += blockDim.x) {
    const int u = it % nb, q = it / nb;
    int i, j;
    closed_pair(q, i, j);
    const int b = b0 + u;
    double r1[4] = {0, 0, 0, 0}, r2[4] = {0, 0, 0, 0}, r3[4] = {0, 0, 0, 0}, r4[4] = {0, 0, 0, 0};
    if (havex) {
      // U rows: (u, side, i)
      const double* Uab_i = XU + ((int64_t)(u * 2 + 0) * nc + i) * ldu;
      const double* Uab_j = XU + ((int64_t)(u * 2 + 0) * nc + j) * ldu;
      const double* Uba_i = XU + ((int64_t)(u * 2 + 1) * nc + i) * ldu;
      const double* Uba_j = XU + ((int64_t)(u * 2 + 1) * nc + j) * ldu;
      for (int y = 0; y < ny; ++y) {
        const double fyj = fA[y * nc + j], fyi = fA[y * nc + i];
#pragma unroll
        for (int c = 0; c < 4; ++c) {
          if (c >= ncol) break;
          r1[c] += fyj * Uab_i[y * ncol + c];   // sigma(i,j,a,b)
          r2[c] += fyi * Uab_j[y * ncol + c];   // sigma(j,i,a,b)
          r3[c] += fyj * Uba_i[y * ncol + c];   // sigma(i,j,b,a)
          r4[c] += fyi * Uba_j[y * ncol + c];   // sigma(j,i,b,a)
        }
      }
    }
    if (p.fC) {
      // v = 0: a, v = 1 + u: b
      const double fbj = fC[(1 + u) * nc + j], fbi = fC[(1 + u) * nc + i];
      const double faj = fC[j], fai = fC[i];
#pragma unroll
      for (int c = 0; c < 4; ++c) {
        if (c >= ncol) break;
        const double w5ia = p.W5 ? W5s[(0 * nc + i) * ncol + c] : 0.0, w5ja = p.W5 ? W5s[(0 * nc + j) * ncol + c] : 0.0;
        const double w5ib = p.W5 ? W5s[((1 + u) * nc + i) * ncol + c] : 0.0;
        const double w5jb = p.W5 ? W5s[((1 + u) * nc + j) * ncol + c] : 0.0;
        const double w6ia = p.W6 ? W6s[(0 * nc + i) * ncol + c] : 0.0, w6ja = p.W6 ? W6s[(0 * nc + j) * ncol + c] : 0.0;
        const double w6ib = p.W6 ? W6s[((1 + u) * nc + i) * ncol + c] : 0.0;
        const double w6jb = p.W6 ? W6s[((1 + u) * nc + j) * ncol + c] : 0.0;
        r1[c] += fbj * w5ia + faj * w6ib;   // sigma(i,j,a,b)
        r2[c] += fbi * w5ja + fai * w6jb;   // sigma(j,i,a,b)
        r3[c] += faj * w5ib + fbj * w6ia;   // sigma(i,j,b,a)
        r4[c] += fai * w5jb + fbi * w6ja;   // sigma(j,i,b,a)
      }
    }
    pack_add<T>(i, j, a, b, npv, nmv, ncol, r1, r2, r3, r4, p.plus, p.minus);
  }
}

// Pass B.  blockIdx.x: virtual tile pair (A >= B), blockIdx.y: closed pair
// (i >= j).  Shared: W rows of both ccav terms for (i,j,v) and (j,i,v), v in
// tile A and tile B ([term][orientation][tile][16][nout + 1], padded), and
// f(v, y) for both tiles.
template <typename T>
__global__ __launch_bounds__(CUB_T * CUB_T) void k_ccvv_up_cpair(CcvvUpArgs<T> p) {
  extern __shared__ double sm[];
  const int nc = p.nc, nv = p.nv, ncol = p.ncol, ny = p.ny;
  const int nout = ny * ncol, ld = nout | 1;
  const int t = threadIdx.x;
  int A = 0, rem = blockIdx.x;
  while (rem > A) {   // blockIdx.x = A (A + 1) / 2 + B
    rem -= A + 1;
    ++A;
  }
  const int B = rem;
  int i, j;
  closed_pair((int)blockIdx.y, i, j);
  const int a0 = A * CUB_T, b0 = B * CUB_T;
  double* Ws = sm;                         // [2][2][2][CUB_T][ld]
  double* fV = Ws + 8 * CUB_T * ld;        // [2][CUB_T][ny]
  for (int e = t; e < 8 * CUB_T * nout; e += blockDim.x) {
    const int k = e % nout, r = (e / nout) % CUB_T, s = e / (nout * CUB_T);
    const int tile = s & 1, orient = (s >> 1) & 1, term = s >> 2;
    const int v = (tile == 0 ? a0 : b0) + r;
    const T* W = term == 0 ? p.W3 : p.W4;
    double val = 0.0;
    if (W && v < nv) {
      const int64_t row = ((int64_t)(orient == 0 ? i : j) * nc + (orient == 0 ? j : i)) * nv + v;
      val = (double)W[row * nout + k];
    }
    Ws[(s * CUB_T + r) * ld + k] = val;
  }
  for (int e = t; e < 2 * CUB_T * ny; e += blockDim.x) {
    const int y = e % ny, r = (e / ny) % CUB_T, tile = e / (ny * CUB_T);
    const int v = (tile == 0 ? a0 : b0) + r;
    fV[e] = v < nv ? p.fV[(int64_t)v * p.fV_stride + y] : 0.0;
  }
  __syncthreads();
  const int tl = t / CUB_T, tf = t % CUB_T;
  const int a = a0 + tl, b = b0 + tf;
  if (a >= nv || b >= nv || a < b) return;
  auto Wrow = [&](int term, int orient, int tile, int r) { return Ws + (((term * 2 + orient) * 2 + tile) * CUB_T + r) * ld; };
  const double* fa = fV + (0 * CUB_T + tl) * ny;
  const double* fb = fV + (1 * CUB_T + tf) * ny;
  double r1[4] = {0, 0, 0, 0}, r2[4] = {0, 0, 0, 0}, r3[4] = {0, 0, 0, 0}, r4[4] = {0, 0, 0, 0};
  // rows: term 0 (W3), term 1 (W4); orientation 0 (i,j), 1 (j,i); tile 0 (a), 1 (b)
  const double* w3ij_a = Wrow(0, 0, 0, tl);
  const double* w3ji_a = Wrow(0, 1, 0, tl);
  const double* w3ij_b = Wrow(0, 0, 1, tf);
  const double* w3ji_b = Wrow(0, 1, 1, tf);
  const double* w4ij_a = Wrow(1, 0, 0, tl);
  const double* w4ji_a = Wrow(1, 1, 0, tl);
  const double* w4ij_b = Wrow(1, 0, 1, tf);
  const double* w4ji_b = Wrow(1, 1, 1, tf);
  for (int y = 0; y < ny; ++y) {
    const double fay = fa[y], fby = fb[y];
#pragma unroll
    for (int c = 0; c < 4; ++c) {
      if (c >= ncol) break;
      const int k = y * ncol + c;
      r1[c] += fby * w3ij_a[k] + fay * w4ij_b[k];   // sigma(i,j,a,b)
      r2[c] += fby * w3ji_a[k] + fay * w4ji_b[k];   // sigma(j,i,a,b)
      r3[c] += fay * w3ij_b[k] + fby * w4ij_a[k];   // sigma(i,j,b,a)
      r4[c] += fay * w3ji_b[k] + fby * w4ji_a[k];   // sigma(j,i,b,a)
    }
  }
  pack_add<T>(i, j, a, b, (int64_t)nv * (nv + 1) / 2, (int64_t)nv * (nv - 1) / 2, ncol, r1, r2, r3, r4, p.plus,
              p.minus);
}

int64_t ccvv_up_vpair_shared(int nc, int nak, int ncol, int ny, bool havex, bool havec, bool havew) {
  int64_t n = 0;
  if (havex) n += (int64_t)CUA_NB * 2 * nc * (nak | 1) + 2 * (int64_t)nak * nak + (int64_t)ny * nc;
  if (havec) n += (int64_t)(1 + CUA_NB) * nc;
  if (havew) n += 2 * (int64_t)(1 + CUA_NB) * nc * ncol;
  return n * (int64_t)sizeof(double);
}

bool ccvv_up_supported(int nc, int nv, int ncol, int ny, int nak) {
  if (nc <= 0 || nv <= 0 || ncol < 1 || ncol > 4 || ny < 1 || ny > 8 || nv > 65535) return false;
  if (nak != ny * ncol) return false;
  if ((int64_t)CUA_NB * 2 * nc * nak > 16 * CUA_THREADS) return false;   // U outputs per thread
  if (ccvv_up_vpair_shared(nc, nak, ncol, ny, true, true, true) > 150 * 1024) return false;
  if ((int64_t)nc * (nc + 1) / 2 > 65535) return false;
  return true;
}

std::vector<uint32_t> ccvv_up_groups(int nv) {
  std::vector<uint32_t> g;
  for (int a = 0; a < nv; ++a)
    for (int b0 = 0; b0 <= a; b0 += CUA_NB) g.push_back((uint32_t)a << 16 | (uint32_t)b0);
  return g;
}

template <typename T>
hipError_t ccvv_up_apply(const CcvvUpArgs<T>& p, const uint32_t* groups, int64_t ngroups, hipStream_t s) {
  if (p.nc <= 0 || p.nv <= 0) return hipSuccess;
  if (!ccvv_up_supported(p.nc, p.nv, p.ncol, p.ny, p.nak)) return hipErrorInvalidValue;
  const bool havex = p.X && (p.G1 || p.G2) && p.fA;
  const bool havec = p.fC && (p.W5 || p.W6);
  if (havex || havec) {
    CcvvUpArgs<T> q = p;
    if (!havex) q.X = nullptr;
    if (!havec) q.fC = nullptr, q.W5 = q.W6 = nullptr;
    const int64_t shm = ccvv_up_vpair_shared(q.nc, q.nak, q.ncol, q.ny, havex, havec, havec);
    hipLaunchKernelGGL(k_ccvv_up_vpair<T>, dim3((unsigned)ngroups), dim3(CUA_THREADS), (size_t)shm, s, q, groups);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  if (p.fV && (p.W3 || p.W4)) {
    const int ntile = (p.nv + CUB_T - 1) / CUB_T;
    const int64_t ntp = (int64_t)ntile * (ntile + 1) / 2, npc = (int64_t)p.nc * (p.nc + 1) / 2;
    const int ld = (p.ny * p.ncol) | 1;
    const size_t shm = (size_t)(8 * CUB_T * ld + 2 * CUB_T * p.ny) * sizeof(double);
    hipLaunchKernelGGL(k_ccvv_up_cpair<T>, dim3((unsigned)ntp, (unsigned)npc), dim3(CUB_T * CUB_T), shm, s, p);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

template hipError_t ccvv_up_apply<double>(const CcvvUpArgs<double>&, const uint32_t*, int64_t, hipStream_t);
template hipError_t ccvv_up_apply<float>(const CcvvUpArgs<float>&, const uint32_t*, int64_t, hipStream_t);

}  // namespace caspt2
