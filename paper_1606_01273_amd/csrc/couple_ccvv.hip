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
#include <algorithm>
#include <cmath>

#include "device_common.hpp"
#include "kernels.hpp"

namespace caspt2 {

namespace {

constexpr int CUA_NB = VPAIR_GROUP;   // virtual pairs (a, b0 .. b0 + 2) per pass-A workgroup
constexpr int CUA_THREADS = 512;
constexpr int CUB_T = 16;        // pass-B virtual tile edge
constexpr int CUA_MAXT = 4;      // MFMA output tiles per wave and round of the pass-A contraction

typedef double d4 __attribute__((ext_vector_type(4)));

// row stride (doubles) of the staged rows of the virtual-pair up pass: even
// (16-byte aligned rows) and 2 mod 4 (consecutive rows start 8 banks apart)
__host__ __device__ constexpr int vpair_ld(int nak) {
  return ((nak + 1) & ~1) % 4 == 0 ? ((nak + 1) & ~1) + 2 : ((nak + 1) & ~1);
}

__device__ inline void closed_pair(int q, int& i, int& j) {
  int ii = (int)((sqrt(8.0 * q + 1.0) - 1.0) * 0.5);
  while ((ii + 1) * (ii + 2) / 2 <= q) ++ii;
  while (ii * (ii + 1) / 2 > q) --ii;
  i = ii;
  j = q - ii * (ii + 1) / 2;
}

// packed rows of ccvv element (i >= j, a >= b): + row, and - row (-1 when
// i == j or a == b, or there is no - entry)
__device__ inline void pack_rows(int i, int j, int a, int b, int64_t npv, int64_t nmv, bool haveminus, int64_t& rp,
                                 int64_t& rm) {
  rp = ((int64_t)i * (i + 1) / 2 + j) * npv + (int64_t)a * (a + 1) / 2 + b;
  rm = (haveminus && i != j && a != b) ? ((int64_t)i * (i - 1) / 2 + j) * nmv + (int64_t)a * (a - 1) / 2 + b : -1;
}

// the current values of the two packed rows (issued early: the loads are in
// flight while the workgroup stages and contracts its inputs)
// NC columns of a packed row as doubles (NC = 4: the row is 32 bytes of
// doubles or 16 bytes of floats, aligned: vector accesses; NC = 0: ncol
// element accesses)
template <typename T, int NC>
__device__ inline void row_load(const T* __restrict__ p, int ncol, double (&v)[4]) {
  if constexpr (NC == 4) {
    if constexpr (sizeof(T) == 8) {
      const double2 x = reinterpret_cast<const double2*>(p)[0], y = reinterpret_cast<const double2*>(p)[1];
      v[0] = x.x;
      v[1] = x.y;
      v[2] = y.x;
      v[3] = y.y;
    } else {
      const float4 x = *reinterpret_cast<const float4*>(p);
      v[0] = x.x;
      v[1] = x.y;
      v[2] = x.z;
      v[3] = x.w;
    }
  } else {
#pragma unroll
    for (int c = 0; c < 4; ++c) v[c] = c < ncol ? (double)p[c] : 0.0;
  }
}
template <typename T, int NC>
__device__ inline void row_store(T* __restrict__ p, int ncol, const double (&v)[4]) {
  if constexpr (NC == 4) {
    if constexpr (sizeof(T) == 8) {
      reinterpret_cast<double2*>(p)[0] = double2{v[0], v[1]};
      reinterpret_cast<double2*>(p)[1] = double2{v[2], v[3]};
    } else {
      *reinterpret_cast<float4*>(p) = float4{(float)v[0], (float)v[1], (float)v[2], (float)v[3]};
    }
  } else {
#pragma unroll
    for (int c = 0; c < 4; ++c)
      if (c < ncol) p[c] = (T)v[c];
  }
}

// the current values of the two packed rows (issued early: the loads are in
// flight while the workgroup stages and contracts its inputs)
template <typename T, int NC>
__device__ inline void pack_load(int64_t rp, int64_t rm, int ncol, const T* __restrict__ plus,
                                 const T* __restrict__ minus, double (&op)[4], double (&om)[4]) {
  row_load<T, NC>(plus + rp * ncol, ncol, op);
  if (rm >= 0) {
    row_load<T, NC>(minus + rm * ncol, ncol, om);
  } else {
#pragma unroll
    for (int c = 0; c < 4; ++c) om[c] = 0.0;
  }
}

}  // namespace

// Pass A.  Workgroup g: virtual index a and b_u = b0 + u (u < nb, b_u <= a)
// from groups[g] = a << 16 | b0.  With Q(u,i) = (G1 + G2)(X(i,a,b_u) +
// X(i,b_u,a)) and D(u,i) = (G1 - G2)(X(i,a,b_u) - X(i,b_u,a)) (rows of
// ny x ncol values), S = W5 + W6 and E = W5 - W6, the four images of
// (i,j,a,b) give
//   + entry: kappa w [f(.,j).Q(i) + f(.,i).Q(j) + f(b,j) S(i,a) + f(a,j) S(i,b)
//                     + f(b,i) S(j,a) + f(a,i) S(j,b)]
//   - entry: [f(.,j).D(i) - f(.,i).D(j) + f(b,j) E(i,a) - f(a,j) E(i,b)
//             - f(b,i) E(j,a) + f(a,i) E(j,b)] / 2
// (f(.,j).Q = sum_y f(y, j) Q(y, c); kappa as in pass B).  Shared memory
// (doubles):
//   XU  [nb][2][nc][ldu]   X(i,a,b_u) + X(i,b_u,a) and their difference,
//                          then Q and D in place; ldu = vpair_ld(nak) (rows
//                          16-byte aligned for vector reads, starting on
//                          different banks)
//   Gt  [2][nak][nak]      (G1 + G2)^T, (G1 - G2)^T
//   fA  [ny][nc]           f(y, j)
//   fC  [1 + nb][nc]       f(v, j) for v = a, b_0 ..
//   Ss, Es [1 + nb][nc][ncol]  S(i, v), E(i, v)
template <typename T, int NC>
// (two workgroups per CU: at most 80 KB of LDS and 128 VGPRs each)
__global__ __launch_bounds__(CUA_THREADS, 4) void k_ccvv_up_vpair(CcvvUpArgs<T> p, const uint32_t* __restrict__ groups) {
  extern __shared__ double sm[];
  const int nc = p.nc, nv = p.nv, ncol = p.ncol, ny = p.ny, nak = p.nak, ldu = vpair_ld(nak);
  const uint32_t gv = groups[blockIdx.x];
  const int a = (int)(gv >> 16), b0 = (int)(gv & 0xffffu);
  const int nb = min(CUA_NB, a + 1 - b0);
  const int t = threadIdx.x;
  const bool havex = p.X != nullptr, havec = p.fC != nullptr;
  double* XU = sm;
  double* Gt = XU + (havex ? (int64_t)CUA_NB * 2 * nc * ldu : 0);
  double* fA = Gt + (havex ? 2 * nak * nak : 0);
  double* fC = fA + (havex ? ny * nc : 0);
  double* Ss = fC + (havec ? (1 + CUA_NB) * nc : 0);
  double* Es = Ss + (havec ? (1 + CUA_NB) * nc * ncol : 0);
  auto vidx = [&](int v) { return v == 0 ? a : b0 + v - 1; };
  const int npc = nc * (nc + 1) / 2, nitem = npc * nb;
  const int64_t npv = (int64_t)nv * (nv + 1) / 2, nmv = (int64_t)nv * (nv - 1) / 2;
  // the packed rows of the first IPT items of this thread, loaded first so
  // that they are in flight during the staging and contraction below
  constexpr int IPT = 3;
  double op[IPT][4], om[IPT][4];
#pragma unroll
  for (int m = 0; m < IPT; ++m) {
    const int it = t + m * (int)blockDim.x;
#pragma unroll
    for (int c = 0; c < 4; ++c) op[m][c] = om[m][c] = 0.0;
    if (it < nitem) {
      int i, j;
      closed_pair(it / nb, i, j);
      int64_t rp, rm;
      pack_rows(i, j, a, b0 + it % nb, npv, nmv, p.minus != nullptr, rp, rm);
      pack_load<T, NC>(rp, rm, ncol, p.plus, p.minus, op[m], om[m]);
    }
  }
  if (havex) {
    for (int e = t; e < nb * nc * nak; e += blockDim.x) {
      const int k = e % nak, i = (e / nak) % nc, u = e / (nak * nc);
      const int b = b0 + u;
      const double x1 = (double)p.X[(((int64_t)i * nv + a) * nv + b) * nak + k];
      const double x2 = (double)p.X[(((int64_t)i * nv + b) * nv + a) * nak + k];
      XU[((u * 2 + 0) * nc + i) * ldu + k] = x1 + x2;
      XU[((u * 2 + 1) * nc + i) * ldu + k] = x1 - x2;
    }
    for (int e = t; e < nak * nak; e += blockDim.x) {
      const int o = e / nak, k = e % nak;
      const double g1 = p.G1 ? (double)p.G1[e] : 0.0, g2 = p.G2 ? (double)p.G2[e] : 0.0;
      Gt[k * nak + o] = g1 + g2;
      Gt[nak * nak + k * nak + o] = g1 - g2;
    }
    for (int e = t; e < ny * nc; e += blockDim.x) fA[e] = p.fA[(e / nc) * p.fA_stride + e % nc];
  }
  if (havec) {
    for (int e = t; e < (1 + nb) * nc; e += blockDim.x) fC[e] = p.fC[(int64_t)vidx(e / nc) * p.fC_stride + e % nc];
    for (int e = t; e < (1 + nb) * nc * ncol; e += blockDim.x) {
      const int c = e % ncol, i = (e / ncol) % nc, v = e / (ncol * nc);
      const int64_t row = (int64_t)i * nv + vidx(v);
      const double w5 = p.W5 ? (double)p.W5[row * ncol + c] : 0.0, w6 = p.W6 ? (double)p.W6[row * ncol + c] : 0.0;
      Ss[e] = w5 + w6;
      Es[e] = w5 - w6;
    }
  }
  __syncthreads();
  if (havex) {
    // Q and D on FP64 MFMA: for each (u, kind) block of nc staged rows,
    // out[r][o] = sum_k xsd[r][k] G_kind[o][k], in 16 x 16 tiles (rows past
    // nc and columns past nak are computed from clamped in-bounds operands
    // and never stored; k past nak contributes zero), written over the
    // staged rows.  Tiles run in rounds of MAXT per wave, column tiles
    // fastest: a round holds whole row tiles (its size is a multiple of the
    // column tile count, 1 or 2), so no round reads a row another round wrote.
    const int lane = t & 63, wv = t >> 6, nwv = (int)blockDim.x >> 6;
    const int ntr = (nc + 15) / 16, ntc = (nak + 15) / 16, ntile = nb * 2 * ntr * ntc;
    constexpr int MAXT = CUA_MAXT;
    for (int base = 0; base < ntile; base += MAXT * nwv) {
      d4 acc[MAXT];
#pragma unroll
      for (int m = 0; m < MAXT; ++m) {
        acc[m] = d4{0.0, 0.0, 0.0, 0.0};
        const int tile = base + wv * MAXT + m;   // uniform over the wave
        if (tile >= ntile) continue;
        const int blk = tile / (ntr * ntc), tr = (tile / ntc) % ntr, tc = tile % ntc;
        const double* xrow = XU + ((int64_t)blk * nc + min(tr * 16 + (lane & 15), nc - 1)) * ldu;
        const double* g = Gt + (blk & 1) * nak * nak + min(tc * 16 + (lane & 15), nak - 1);
        for (int k0 = 0; k0 < nak; k0 += 4) {
          const int k = k0 + (lane >> 4);
          const double av = k < nak ? xrow[k] : 0.0;
          const double bv = k < nak ? g[k * nak] : 0.0;
          acc[m] = __builtin_amdgcn_mfma_f64_16x16x4f64(av, bv, acc[m], 0, 0, 0);
        }
      }
      __syncthreads();
#pragma unroll
      for (int m = 0; m < MAXT; ++m) {
        const int tile = base + wv * MAXT + m;
        if (tile >= ntile) continue;
        const int blk = tile / (ntr * ntc), tr = (tile / ntc) % ntr, tc = tile % ntc;
        const int col = tc * 16 + (lane & 15);
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const int row = tr * 16 + (lane >> 4) + 4 * v;
          if (row < nc && col < nak) XU[((int64_t)blk * nc + row) * ldu + col] = acc[m][v];
        }
      }
      __syncthreads();
    }
  }
  // the + and - sums of item it (closed pair it / nb, virtual pair (a, b0 + it % nb))
  auto sums = [&](int it, int& i, int& j, int& b, double (&sp)[4], double (&sd)[4]) {
    const int u = it % nb;
    closed_pair(it / nb, i, j);
    b = b0 + u;
#pragma unroll
    for (int c = 0; c < 4; ++c) sp[c] = sd[c] = 0.0;
    if (havex) {
      const double* Qi = XU + ((int64_t)(u * 2 + 0) * nc + i) * ldu;
      const double* Qj = XU + ((int64_t)(u * 2 + 0) * nc + j) * ldu;
      const double* Di = XU + ((int64_t)(u * 2 + 1) * nc + i) * ldu;
      const double* Dj = XU + ((int64_t)(u * 2 + 1) * nc + j) * ldu;
      for (int y = 0; y < ny; ++y) {
        const double fyj = fA[y * nc + j], fyi = fA[y * nc + i];
#pragma unroll
        for (int c = 0; c < 4; ++c) {
          if (c >= ncol) break;
          sp[c] += fyj * Qi[y * ncol + c] + fyi * Qj[y * ncol + c];
          sd[c] += fyj * Di[y * ncol + c] - fyi * Dj[y * ncol + c];
        }
      }
    }
    if (havec) {
      // v = 0: a, v = 1 + u: b
      const double fbj = fC[(1 + u) * nc + j], fbi = fC[(1 + u) * nc + i];
      const double faj = fC[j], fai = fC[i];
      const double* Sa = Ss;
      const double* Sb = Ss + (1 + u) * nc * ncol;
      const double* Ea = Es;
      const double* Eb = Es + (1 + u) * nc * ncol;
#pragma unroll
      for (int c = 0; c < 4; ++c) {
        if (c >= ncol) break;
        sp[c] += fbj * Sa[i * ncol + c] + faj * Sb[i * ncol + c] + fbi * Sa[j * ncol + c] + fai * Sb[j * ncol + c];
        sd[c] += fbj * Ea[i * ncol + c] - faj * Eb[i * ncol + c] - fbi * Ea[j * ncol + c] + fai * Eb[j * ncol + c];
      }
    }
  };
  auto store = [&](int i, int j, int b, int64_t rp, int64_t rm, const double (&sp)[4], const double (&sd)[4],
                   const double (&o1)[4], const double (&o2)[4]) {
    const bool dij = i != j, dab = a != b;
    const double wk = (dij && dab) ? 0.5 : ((dij || dab) ? 0.5 * 0.70710678118654752440 : 0.25);
    double v[4];
#pragma unroll
    for (int c = 0; c < 4; ++c) v[c] = o1[c] + wk * sp[c];
    row_store<T, NC>(p.plus + rp * ncol, ncol, v);
    if (rm >= 0) {
#pragma unroll
      for (int c = 0; c < 4; ++c) v[c] = o2[c] + 0.5 * sd[c];
      row_store<T, NC>(p.minus + rm * ncol, ncol, v);
    }
  };
#pragma unroll
  for (int m = 0; m < IPT; ++m) {
    const int it = t + m * (int)blockDim.x;
    if (it >= nitem) continue;
    int i, j, b;
    double sp[4], sd[4];
    sums(it, i, j, b, sp, sd);
    int64_t rp, rm;
    pack_rows(i, j, a, b, npv, nmv, p.minus != nullptr, rp, rm);
    store(i, j, b, rp, rm, sp, sd, op[m], om[m]);
  }
  // items beyond the prefetched ones (more than IPT per thread)
  for (int it = t + IPT * (int)blockDim.x; it < nitem; it += blockDim.x) {
    int i, j, b;
    double sp[4], sd[4], o1[4], o2[4];
    sums(it, i, j, b, sp, sd);
    int64_t rp, rm;
    pack_rows(i, j, a, b, npv, nmv, p.minus != nullptr, rp, rm);
    pack_load<T, NC>(rp, rm, ncol, p.plus, p.minus, o1, o2);
    store(i, j, b, rp, rm, sp, sd, o1, o2);
  }
}

// Pass B.  blockIdx.x: virtual tile pair (A >= B), blockIdx.y: closed pair
// (i >= j).  With the W rows of both ccav terms summed over the four
// orientations, P(v) = W3(i,j,v) + W3(j,i,v) + W4(i,j,v) + W4(j,i,v) and
// M(v) = W3(i,j,v) - W3(j,i,v) - W4(i,j,v) + W4(j,i,v), the four images give
//   + entry: kappa w (f(b).P(a) + f(a).P(b)),  - entry: (f(b).M(a) - f(a).M(b)) / 2
// (f(v).P = sum_y f(v, y) P(y, c); kappa = 1, 1/2 or 1/4 as none, one or both
// of i = j, a = b hold, where P counts coinciding images twice).  Shared:
// P and M for tile A and tile B ([2][2][16][nout + 1], padded) and f(v, y).
template <typename T, int NC>
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
  const int tl = t / CUB_T, tf = t % CUB_T;
  const int a = a0 + tl, b = b0 + tf;
  const bool valid = a < nv && b < nv && a >= b;
  // this thread's packed rows, loaded before the staging below
  const int64_t npv = (int64_t)nv * (nv + 1) / 2, nmv = (int64_t)nv * (nv - 1) / 2;
  int64_t rp = 0, rm = -1;
  double op[4] = {0, 0, 0, 0}, om[4] = {0, 0, 0, 0};
  if (valid) {
    pack_rows(i, j, a, b, npv, nmv, p.minus != nullptr, rp, rm);
    pack_load<T, NC>(rp, rm, ncol, p.plus, p.minus, op, om);
  }
  double* PM = sm;                         // [P, M][tile A, B][CUB_T][ld]
  double* fV = PM + 4 * CUB_T * ld;        // [tile][CUB_T][ny]
  const int64_t rij = ((int64_t)i * nc + j) * nv, rji = ((int64_t)j * nc + i) * nv;
  for (int e = t; e < 2 * CUB_T * nout; e += blockDim.x) {
    const int k = e % nout, r = (e / nout) % CUB_T, tile = e / (nout * CUB_T);
    const int v = (tile == 0 ? a0 : b0) + r;
    double w3ij = 0.0, w3ji = 0.0, w4ij = 0.0, w4ji = 0.0;
    if (v < nv) {
      if (p.W3) {
        w3ij = (double)p.W3[(rij + v) * nout + k];
        w3ji = (double)p.W3[(rji + v) * nout + k];
      }
      if (p.W4) {
        w4ij = (double)p.W4[(rij + v) * nout + k];
        w4ji = (double)p.W4[(rji + v) * nout + k];
      }
    }
    PM[((0 * 2 + tile) * CUB_T + r) * ld + k] = w3ij + w3ji + w4ij + w4ji;
    PM[((1 * 2 + tile) * CUB_T + r) * ld + k] = w3ij - w3ji - w4ij + w4ji;
  }
  for (int e = t; e < 2 * CUB_T * ny; e += blockDim.x) {
    const int y = e % ny, r = (e / ny) % CUB_T, tile = e / (ny * CUB_T);
    const int v = (tile == 0 ? a0 : b0) + r;
    fV[e] = v < nv ? p.fV[(int64_t)v * p.fV_stride + y] : 0.0;
  }
  __syncthreads();
  if (!valid) return;
  const double* fa = fV + (0 * CUB_T + tl) * ny;
  const double* fb = fV + (1 * CUB_T + tf) * ny;
  const double* Pa = PM + ((0 * 2 + 0) * CUB_T + tl) * ld;
  const double* Pb = PM + ((0 * 2 + 1) * CUB_T + tf) * ld;
  const double* Ma = PM + ((1 * 2 + 0) * CUB_T + tl) * ld;
  const double* Mb = PM + ((1 * 2 + 1) * CUB_T + tf) * ld;
  double sp[4] = {0, 0, 0, 0}, sd[4] = {0, 0, 0, 0};
  for (int y = 0; y < ny; ++y) {
    const double fay = fa[y], fby = fb[y];
#pragma unroll
    for (int c = 0; c < 4; ++c) {
      if (c >= ncol) break;
      const int k = y * ncol + c;
      sp[c] += fby * Pa[k] + fay * Pb[k];
      sd[c] += fby * Ma[k] - fay * Mb[k];
    }
  }
  const bool dij = i != j, dab = a != b;
  const double wk = (dij && dab) ? 0.5 : ((dij || dab) ? 0.5 * 0.70710678118654752440 : 0.25);
  double v[4];
#pragma unroll
  for (int c = 0; c < 4; ++c) v[c] = op[c] + wk * sp[c];
  row_store<T, NC>(p.plus + rp * ncol, ncol, v);
  if (rm >= 0) {
#pragma unroll
    for (int c = 0; c < 4; ++c) v[c] = om[c] + 0.5 * sd[c];
    row_store<T, NC>(p.minus + rm * ncol, ncol, v);
  }
}

// Down terms out of ccvv into cavv (through f(closed, active)) and caav
// (through f(closed, virtual)), read straight from the packed ccvv rows.  A
// workgroup takes the virtual pairs (a, b_u = b0 + u), u < nb, of one group
// (the table of the up pass) and every closed pair.  With P, M the packed +
// and - values of closed pair (z, i) (either order) and Psym(z,i) = 2 w P,
// Msk(z,i) = s M (w the packing weight, s = +1 for z > i, -1 for z < i, 0
// for z = i), X(z,i,a,b) = (Psym + Msk) / 2 and X(z,i,b,a) = (Psym - Msk) / 2,
//   cavv:  Ys(i)(y,c) = sum_z f(z,y) Psym(z,i),  Yd(i) = sum_z f(z,y) Msk(z,i);
//          + entry (i,ab) += kv (G1 + G2) Ys(i),  - entry += (G1 - G2) Yd(i) / sqrt 2
//          (kv = 1/sqrt 2, or 1/2 for a = b), G1/G2 [cavv columns][ny x ncol]
//   caav:  T1(i,w,v) = sum_z f(z,w) X(z,i,w,v) and T2(i,v,w) = sum_z f(z,w)
//          X(z,i,v,w) for (w,v) in {(a,b), (b,a)}, stored as T[0][i][w][v] and
//          T[1][i][w][v] (T2 transposed), summed over w afterwards.
// A thread owns (u, i, c) and runs the z sum from its own loads; the
// contraction with G runs on FP64 MFMA (16 x 16 tiles of (i, column)).
constexpr int CDV_THREADS = 512;
constexpr int CDV_ZB = 8;   // closed indices whose packed values a thread loads at once
// (two workgroups per CU: at most 80 KB of LDS and 128 VGPRs each)
template <typename T>
__global__ __launch_bounds__(CDV_THREADS, 4) void k_ccvv_down_vpair(CcvvDownArgs<T> p,
                                                                    const uint32_t* __restrict__ groups) {
  extern __shared__ double sm[];
  const int nc = p.nc, nv = p.nv, ncol = p.ncol, ny = p.ny, nab = p.nab, nout = p.ny * p.ncol;
  const int t = threadIdx.x, lane = t & 63, wv = t >> 6, nwv = (int)blockDim.x >> 6;
  const uint32_t gv = groups[blockIdx.x];
  const int a = (int)(gv >> 16), b0 = (int)(gv & 0xffffu);
  const int nb = min(CUA_NB, a + 1 - b0);
  const int64_t npv = (int64_t)nv * (nv + 1) / 2, nmv = (int64_t)nv * (nv - 1) / 2;
  const bool havey = p.sp != nullptr, havet = p.Tw != nullptr;
  const int ldy = nout | 1;
  double* Gs = sm;                                    // [2][nab][nout]: G1 + G2, G1 - G2
  double* fca = Gs + (havey ? 2 * nab * nout : 0);    // [nc][ny]
  double* fcv = fca + (havey ? nc * ny : 0);          // [1 + nb][nc]: f(z, a), f(z, b_u)
  double* Ysd = fcv + (havet ? (1 + CUA_NB) * nc : 0);   // [nb][2][nc][ldy]
  // output tiles: (u, kind (+: Ys, -: Yd), row tile, column tile)
  const int ntr = (nc + 15) / 16, ntc = (nab + 15) / 16;
  const int ntile = havey ? nb * 2 * ntr * ntc : 0;
  auto tile_of = [&](int tile, int& u, int& kind, int& tr, int& tc) {
    u = tile / (2 * ntr * ntc);
    kind = (tile / (ntr * ntc)) & 1;
    tr = (tile / ntc) % ntr;
    tc = tile % ntc;
  };
  if (havey) {
    for (int e = t; e < nab * nout; e += blockDim.x) {
      const double g1 = p.G1 ? (double)p.G1[e] : 0.0, g2 = p.G2 ? (double)p.G2[e] : 0.0;
      Gs[e] = g1 + g2;
      Gs[nab * nout + e] = g1 - g2;
    }
    for (int e = t; e < nc * ny; e += blockDim.x) fca[e] = p.fA[(int64_t)(e / ny) * p.fA_stride + e % ny];
  }
  if (havet)
    for (int e = t; e < (1 + nb) * nc; e += blockDim.x) {
      const int v = e / nc, z = e % nc;
      fcv[e] = p.fC[(int64_t)z * p.fC_stride + (v == 0 ? a : b0 + v - 1)];
    }
  __syncthreads();
  // thread (u, i, c): the sums over the closed index z
  for (int it = t; it < nb * nc * ncol; it += blockDim.x) {
    const int c = it % ncol, i = (it / ncol) % nc, u = it / (ncol * nc);
    const int b = b0 + u;
    const bool dab = a != b;
    const int64_t pab = (int64_t)a * (a + 1) / 2 + b, mab = (int64_t)a * (a - 1) / 2 + b;
    double ys[8] = {0, 0, 0, 0, 0, 0, 0, 0}, yd[8] = {0, 0, 0, 0, 0, 0, 0, 0};
    double t1ab = 0.0, t1ba = 0.0, t2ab = 0.0, t2ba = 0.0;
    for (int z0 = 0; z0 < nc; z0 += CDV_ZB) {
      double psym[CDV_ZB], msk[CDV_ZB];
#pragma unroll
      for (int k = 0; k < CDV_ZB; ++k) {
        psym[k] = msk[k] = 0.0;
        const int z = z0 + k;
        if (z >= nc) continue;
        const int hi = max(z, i), lo = min(z, i);
        const bool dzi = z != i;
        const double w = (dzi && dab) ? 0.5 : ((dzi || dab) ? 0.70710678118654752440 : 1.0);
        psym[k] = 2.0 * w * (double)p.xp[(((int64_t)hi * (hi + 1) / 2 + lo) * npv + pab) * ncol + c];
        if (dzi && dab && p.xm) {
          const double m = (double)p.xm[(((int64_t)hi * (hi - 1) / 2 + lo) * nmv + mab) * ncol + c];
          msk[k] = z > i ? m : -m;
        }
      }
#pragma unroll
      for (int k = 0; k < CDV_ZB; ++k) {
        const int z = z0 + k;
        if (z >= nc) break;
        if (havey) {
#pragma unroll
          for (int y = 0; y < 8; ++y) {
            if (y >= ny) break;
            const double f = fca[z * ny + y];
            ys[y] += f * psym[k];
            yd[y] += f * msk[k];
          }
        }
        if (havet) {
          const double xab = 0.5 * (psym[k] + msk[k]), xba = 0.5 * (psym[k] - msk[k]);
          const double fa = fcv[z], fb = fcv[(1 + u) * nc + z];
          t1ab += fa * xab;
          t1ba += fb * xba;
          t2ab += fb * xab;
          t2ba += fa * xba;
        }
      }
    }
    if (havey) {
#pragma unroll
      for (int y = 0; y < 8; ++y) {
        if (y >= ny) break;
        Ysd[((u * 2 + 0) * nc + i) * ldy + y * ncol + c] = ys[y];
        Ysd[((u * 2 + 1) * nc + i) * ldy + y * ncol + c] = yd[y];
      }
    }
    if (havet) {
      const int64_t nv2 = (int64_t)nv * nv, nt = (int64_t)nc * nv2;
      const int64_t iab = (int64_t)i * nv2 + (int64_t)a * nv + b, iba = (int64_t)i * nv2 + (int64_t)b * nv + a;
      p.Tw[iab * ncol + c] = (T)t1ab;             // T1(i, a, b)
      p.Tw[iba * ncol + c] = (T)t1ba;             // T1(i, b, a)
      p.Tw[(nt + iba) * ncol + c] = (T)t2ab;      // T2(i, a, b) at [i][b][a]
      p.Tw[(nt + iab) * ncol + c] = (T)t2ba;      // T2(i, b, a) at [i][a][b]
    }
  }
  if (!havey) return;
  __syncthreads();
  for (int tile = wv; tile < ntile; tile += nwv) {   // uniform over the wave
    int u, kind, tr, tc;
    tile_of(tile, u, kind, tr, tc);
    const int b = b0 + u;
    if (kind == 1 && (a == b || !p.sm)) continue;
    const int col = tc * 16 + (lane & 15);
    // the rows this lane updates, loaded before the contraction
    const int64_t base = kind == 0 ? (int64_t)a * (a + 1) / 2 + b : (int64_t)a * (a - 1) / 2 + b;
    const int64_t rstride = kind == 0 ? npv : nmv;
    T* out = kind == 0 ? p.sp : p.sm;
    double ov[4];
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int i = tr * 16 + (lane >> 4) + 4 * v;
      ov[v] = (i < nc && col < nab) ? (double)out[((int64_t)i * rstride + base) * nab + col] : 0.0;
    }
    const double* yrow = Ysd + ((int64_t)(u * 2 + kind) * nc + min(tr * 16 + (lane & 15), nc - 1)) * ldy;
    const double* grow = Gs + (int64_t)kind * nab * nout + (int64_t)min(tc * 16 + (lane & 15), nab - 1) * nout;
    d4 acc = {0.0, 0.0, 0.0, 0.0};
    for (int k0 = 0; k0 < nout; k0 += 4) {
      const int k = k0 + (lane >> 4);
      const double av = k < nout ? yrow[k] : 0.0;
      const double bv = k < nout ? grow[k] : 0.0;
      acc = __builtin_amdgcn_mfma_f64_16x16x4f64(av, bv, acc, 0, 0, 0);
    }
    const double scale = kind == 0 ? (a != b ? 0.70710678118654752440 : 0.5) : 0.70710678118654752440;
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int i = tr * 16 + (lane >> 4) + 4 * v;
      if (i < nc && col < nab) out[((int64_t)i * rstride + base) * nab + col] = (T)(ov[v] + scale * acc[v]);
    }
  }
}

// Y[k][i][v][c] = sum_w T[k][i][w][v][c] (k = 0, 1)
template <typename T>
__global__ __launch_bounds__(256) void k_sum_middle(int64_t n_outer, int64_t n_mid, int64_t n_inner, const T* __restrict__ in,
                                                    T* __restrict__ out) {
  const int64_t total = n_outer * n_inner;
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < total; e += (int64_t)gridDim.x * blockDim.x) {
    const int64_t o = e / n_inner, r = e % n_inner;
    const T* src = in + o * n_mid * n_inner + r;
    double s = 0.0;
    for (int64_t w = 0; w < n_mid; ++w) s += (double)src[w * n_inner];
    out[e] = (T)s;
  }
}

// Down terms out of ccvv into ccav (through f(active, virtual)) read
// straight from the packed ccvv rows.  A workgroup takes one closed pair
// (i >= j) and CDB_A virtual indices a.  With P, M the packed + and -
// values at (i, j) and the virtual pair {w, a}, and f(y, w) the Fock block,
//   Ys(a)(y,c) = sum_w f(y,w) 2 wt P,  Yd(a)(y,c) = sum_w f(y,w) s M
// (wt the packing weight, s = +1 for w > a, -1 for w < a, 0 for w = a) are
// the sum and the difference of the (i,j) and (j,i) reductions of the first
// term (the second term's are Ys and -Yd), so
//   + entry (ij, a) += kc (G3 + G4) Ys(a),  - entry += (G3 - G4) Yd(a) / sqrt 2
// (kc = 1/sqrt 2, or 1/2 for i = j; G3/G4 [ccav columns][ny x ncol]).  A
// thread owns (a, c) and runs the w sum from its own loads, CDB_WB w at a
// time; the G contraction runs on MFMA.
constexpr int CDB_A = 64;
constexpr int CDB_WB = 8;    // virtual indices whose packed values a thread loads at once
template <typename T>
__global__ __launch_bounds__(256) void k_ccvv_down_cpair(CcvvDownArgs<T> p) {
  extern __shared__ double sm[];
  const int nc = p.nc, nv = p.nv, ncol = p.ncol, ny = p.ny, nab = p.nab3, nout = p.ny * p.ncol;
  const int t = threadIdx.x, lane = t & 63, wv = t >> 6, nwv = (int)blockDim.x >> 6;
  int i, j;
  closed_pair((int)blockIdx.y, i, j);
  const int a0 = (int)blockIdx.x * CDB_A;
  const int na = min(CDB_A, nv - a0);
  const int64_t npv = (int64_t)nv * (nv + 1) / 2, nmv = (int64_t)nv * (nv - 1) / 2;
  const int64_t pij = (int64_t)i * (i + 1) / 2 + j, mij = (int64_t)i * (i - 1) / 2 + j;
  const bool dij = i != j;
  const int ldy = nout | 1;
  double* Gs = sm;                               // [2][nab][nout]
  double* Ysd = Gs + 2 * nab * nout;             // [2][CDB_A][ldy]
  // the ccav rows this lane updates (MFMA output layout), loaded first
  const int ntr = CDB_A / 16, ntc = (nab + 15) / 16, ntile = 2 * ntr * ntc;
  constexpr int MAXT = 4;   // tiles per wave (checked on the host)
  double old[MAXT][4];
#pragma unroll
  for (int m = 0; m < MAXT; ++m) {
    const int tile = wv + m * nwv;
#pragma unroll
    for (int v = 0; v < 4; ++v) old[m][v] = 0.0;
    if (tile >= ntile) continue;
    const int kind = tile / (ntr * ntc), tr = (tile / ntc) % ntr, tc = tile % ntc;
    if (kind == 1 && (!dij || !p.cm)) continue;
    const int col = tc * 16 + (lane & 15);
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int al = tr * 16 + (lane >> 4) + 4 * v;
      if (al < na && col < nab)
        old[m][v] = kind == 0 ? (double)p.cp[(pij * nv + a0 + al) * nab + col]
                              : (double)p.cm[(mij * nv + a0 + al) * nab + col];
    }
  }
  for (int e = t; e < nab * nout; e += blockDim.x) {
    const double g3 = p.G3 ? (double)p.G3[e] : 0.0, g4 = p.G4 ? (double)p.G4[e] : 0.0;
    Gs[e] = g3 + g4;
    Gs[nab * nout + e] = g3 - g4;
  }
  // thread (a, c): the sums over w
  const int al = t / 4, c = t % 4;
  const bool act = al < na && c < ncol;
  const int a = a0 + min(al, na - 1);
  double ys[8] = {0, 0, 0, 0, 0, 0, 0, 0}, yd[8] = {0, 0, 0, 0, 0, 0, 0, 0};
  // f(y, w) is read at addresses uniform over the workgroup (w runs in step
  // on every thread): scalar loads, no LDS
  const double* __restrict__ fV = p.fV;
  const int64_t fs = p.fV_stride;
  if (act) {
    const int f0 = 0, nf = nv;
    for (int w0 = 0; w0 < nf; w0 += CDB_WB) {
      double pv[CDB_WB], mv[CDB_WB];
#pragma unroll
      for (int u = 0; u < CDB_WB; ++u) {
        pv[u] = mv[u] = 0.0;
        if (w0 + u >= nf) continue;
        const int w = f0 + w0 + u;
        const int hi = max(w, a), lo = min(w, a);
        const bool dwa = w != a;
        const double wt = (dij && dwa) ? 0.5 : ((dij || dwa) ? 0.70710678118654752440 : 1.0);
        pv[u] = 2.0 * wt * (double)p.xp[(pij * npv + (int64_t)hi * (hi + 1) / 2 + lo) * ncol + c];
        if (dij && dwa && p.xm) {
          const double m = (double)p.xm[(mij * nmv + (int64_t)hi * (hi - 1) / 2 + lo) * ncol + c];
          mv[u] = w > a ? m : -m;
        }
      }
#pragma unroll
      for (int u = 0; u < CDB_WB; ++u) {
        if (w0 + u >= nf) break;
#pragma unroll
        for (int y = 0; y < 8; ++y) {
          if (y >= ny) break;
          const double f = fV[(int64_t)y * fs + f0 + w0 + u];
          ys[y] += f * pv[u];
          yd[y] += f * mv[u];
        }
      }
    }
  }
  if (act) {
#pragma unroll
    for (int y = 0; y < 8; ++y) {
      if (y >= ny) break;
      Ysd[al * ldy + y * ncol + c] = ys[y];
      Ysd[(CDB_A + al) * ldy + y * ncol + c] = yd[y];
    }
  }
  __syncthreads();
#pragma unroll
  for (int m = 0; m < MAXT; ++m) {
    const int tile = wv + m * nwv;   // uniform over the wave
    if (tile >= ntile) continue;
    const int kind = tile / (ntr * ntc), tr = (tile / ntc) % ntr, tc = tile % ntc;
    if (kind == 1 && (!dij || !p.cm)) continue;
    const double* yrow = Ysd + ((int64_t)kind * CDB_A + min(tr * 16 + (lane & 15), na - 1)) * ldy;
    const double* grow = Gs + (int64_t)kind * nab * nout + (int64_t)min(tc * 16 + (lane & 15), nab - 1) * nout;
    d4 acc = {0.0, 0.0, 0.0, 0.0};
    for (int k0 = 0; k0 < nout; k0 += 4) {
      const int k = k0 + (lane >> 4);
      const double av = k < nout ? yrow[k] : 0.0;
      const double bv = k < nout ? grow[k] : 0.0;
      acc = __builtin_amdgcn_mfma_f64_16x16x4f64(av, bv, acc, 0, 0, 0);
    }
    const double scale = kind == 0 ? (dij ? 0.70710678118654752440 : 0.5) : 0.70710678118654752440;
    const int col = tc * 16 + (lane & 15);
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int ar = tr * 16 + (lane >> 4) + 4 * v;
      if (ar >= na || col >= nab) continue;
      const double val = old[m][v] + scale * acc[v];
      if (kind == 0) p.cp[(pij * nv + a0 + ar) * nab + col] = (T)val;
      else p.cm[(mij * nv + a0 + ar) * nab + col] = (T)val;
    }
  }
}

int64_t ccvv_down_shared(int nc, int ncol, int ny, int nab, bool havey, bool havet) {
  int64_t n = 0;
  if (havey)
    n += 2 * (int64_t)nab * ny * ncol + (int64_t)nc * ny + (int64_t)CUA_NB * 2 * nc * ((ny * ncol) | 1);
  if (havet) n += (int64_t)(1 + CUA_NB) * nc;
  return n * (int64_t)sizeof(double);
}

int64_t ccvv_down_cpair_shared(int ncol, int ny, int nab3) {
  return (int64_t)(2 * (int64_t)nab3 * ny * ncol + 2 * CDB_A * ((ny * ncol) | 1)) * (int64_t)sizeof(double);
}

bool ccvv_down_supported(int nc, int nv, int ncol, int ny, int nab) {
  if (nc <= 0 || nv <= 0 || ncol < 1 || ncol > 4 || ny < 1 || ny > 8 || nab != ny * ncol) return false;
  int dev = 0, lds_max = 0;
  if (hipGetDevice(&dev) != hipSuccess ||
      hipDeviceGetAttribute(&lds_max, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) != hipSuccess)
    return false;
  return ccvv_down_shared(nc, ncol, ny, nab, true, true) <= lds_max &&
         ccvv_down_cpair_shared(ncol, ny, nab) <= lds_max &&
         2 * (CDB_A / 16) * ((nab + 15) / 16) <= 4 * 4;   // closed-pair pass: MFMA tiles per wave
}

template <typename T>
hipError_t ccvv_down_apply(const CcvvDownArgs<T>& p, const uint32_t* groups, int64_t ngroups, hipStream_t s) {
  if (p.nc <= 0 || p.nv <= 0) return hipSuccess;
  if (!ccvv_down_supported(p.nc, p.nv, p.ncol, p.ny, p.nab)) return hipErrorInvalidValue;
  const bool havey = p.sp && (p.G1 || p.G2) && p.fA;
  const bool havet = p.Tw && p.fC;
  const bool havec = p.cp && (p.G3 || p.G4) && p.fV;
  if (havec) {
    if (p.nab3 != p.ny * p.ncol) return hipErrorInvalidValue;
    const size_t shm = (size_t)ccvv_down_cpair_shared(p.ncol, p.ny, p.nab3);
    const unsigned nblk = (unsigned)((p.nv + CDB_A - 1) / CDB_A), npc = (unsigned)(p.nc * (p.nc + 1) / 2);
    hipLaunchKernelGGL(k_ccvv_down_cpair<T>, dim3(nblk, npc), dim3(256), shm, s, p);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  if (!havey && !havet) return hipSuccess;
  CcvvDownArgs<T> q = p;
  if (!havey) q.sp = q.sm = nullptr;
  if (!havet) q.Tw = nullptr;
  const size_t shm = (size_t)ccvv_down_shared(q.nc, q.ncol, q.ny, q.nab, havey, havet);
  hipLaunchKernelGGL(k_ccvv_down_vpair<T>, dim3((unsigned)ngroups), dim3(CDV_THREADS), shm, s, q, groups);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess || !havet) return e;
  const int64_t inner = (int64_t)p.nv * p.ncol, outer = 2 * (int64_t)p.nc;
  const unsigned grid = (unsigned)std::min<int64_t>((outer * inner + 255) / 256, 65536);
  hipLaunchKernelGGL(k_sum_middle<T>, dim3(grid), dim3(256), 0, s, outer, (int64_t)p.nv, inner, p.Tw, p.Y);
  return hipGetLastError();
}

template hipError_t ccvv_down_apply<double>(const CcvvDownArgs<double>&, const uint32_t*, int64_t, hipStream_t);
template hipError_t ccvv_down_apply<float>(const CcvvDownArgs<float>&, const uint32_t*, int64_t, hipStream_t);

int64_t ccvv_up_vpair_shared(int nc, int nak, int ncol, int ny, bool havex, bool havec) {
  int64_t n = 0;
  if (havex) n += (int64_t)CUA_NB * 2 * nc * vpair_ld(nak) + 2 * (int64_t)nak * nak + (int64_t)ny * nc;
  if (havec) n += (int64_t)(1 + CUA_NB) * nc + 2 * (int64_t)(1 + CUA_NB) * nc * ncol;
  return n * (int64_t)sizeof(double);
}

bool ccvv_up_supported(int nc, int nv, int ncol, int ny, int nak) {
  if (nc <= 0 || nv <= 0 || ncol < 1 || ncol > 4 || ny < 1 || ny > 8 || nv > 65535) return false;
  if (nak != ny * ncol) return false;
  int dev = 0, lds_max = 0;
  if (hipGetDevice(&dev) != hipSuccess ||
      hipDeviceGetAttribute(&lds_max, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) != hipSuccess)
    return false;
  if (ccvv_up_vpair_shared(nc, nak, ncol, ny, true, true) > lds_max) return false;
  if ((int64_t)nc * (nc + 1) / 2 > 65535) return false;
  return true;
}

std::vector<uint32_t> ccvv_up_groups(int nv, bool b_major) {
  std::vector<uint32_t> g;
  if (!b_major) {
    for (int a = 0; a < nv; ++a)
      for (int b0 = 0; b0 <= a; b0 += CUA_NB) g.push_back((uint32_t)a << 16 | (uint32_t)b0);
    return g;
  }
  // b0 outermost, and workgroup g (dispatched to XCD g % 8) takes entry
  // start(g % 8) + g / 8 of that list: each XCD runs a contiguous run of
  // groups sharing b0, so rows indexed by the b of a pair stay in its L2
  std::vector<uint32_t> list;
  for (int b0 = 0; b0 < nv; b0 += CUA_NB)
    for (int a = b0; a < nv; ++a) list.push_back((uint32_t)a << 16 | (uint32_t)b0);
  const int64_t n = (int64_t)list.size(), q = n / 8, r = n % 8;
  g.resize(list.size());
  for (int64_t k = 0; k < n; ++k) {
    const int64_t x = k % 8;
    g[k] = list[x * q + std::min<int64_t>(x, r) + k / 8];
  }
  return g;
}

// the packed rows as whole vector accesses: four columns and both entries
// aligned to a row
template <typename T>
bool rows_vectorised(const CcvvUpArgs<T>& p) {
  const uintptr_t row = 4 * sizeof(T);
  return p.ncol == 4 && reinterpret_cast<uintptr_t>(p.plus) % row == 0 &&
         (!p.minus || reinterpret_cast<uintptr_t>(p.minus) % row == 0);
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
    const int64_t shm = ccvv_up_vpair_shared(q.nc, q.nak, q.ncol, q.ny, havex, havec);
    if (rows_vectorised(q))
      hipLaunchKernelGGL((k_ccvv_up_vpair<T, 4>), dim3((unsigned)ngroups), dim3(CUA_THREADS), (size_t)shm, s, q, groups);
    else
      hipLaunchKernelGGL((k_ccvv_up_vpair<T, 0>), dim3((unsigned)ngroups), dim3(CUA_THREADS), (size_t)shm, s, q, groups);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  if (p.fV && (p.W3 || p.W4)) {
    const int ntile = (p.nv + CUB_T - 1) / CUB_T;
    const int64_t ntp = (int64_t)ntile * (ntile + 1) / 2, npc = (int64_t)p.nc * (p.nc + 1) / 2;
    const int ld = (p.ny * p.ncol) | 1;
    const size_t shm = (size_t)(4 * CUB_T * ld + 2 * CUB_T * p.ny) * sizeof(double);
    if (rows_vectorised(p))
      hipLaunchKernelGGL((k_ccvv_up_cpair<T, 4>), dim3((unsigned)ntp, (unsigned)npc), dim3(CUB_T * CUB_T), shm, s, p);
    else
      hipLaunchKernelGGL((k_ccvv_up_cpair<T, 0>), dim3((unsigned)ntp, (unsigned)npc), dim3(CUB_T * CUB_T), shm, s, p);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

template hipError_t ccvv_up_apply<double>(const CcvvUpArgs<double>&, const uint32_t*, int64_t, hipStream_t);
template hipError_t ccvv_up_apply<float>(const CcvvUpArgs<float>&, const uint32_t*, int64_t, hipStream_t);

}  // namespace caspt2
