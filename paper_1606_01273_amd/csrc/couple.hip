// Coupling kernels (Fock couplings between excitation blocks) and the
// packed <-> all-orderings conversions, for FP64 and FP32 data.
#include <algorithm>

#include "device_common.hpp"
#include "kernels.hpp"

namespace caspt2 {

static inline unsigned cdiv(int64_t a, int64_t b) { return (unsigned)((a + b - 1) / b); }

// calls fn(e, chi) for every distinct image e of the orbit of e0 under the
// swaps of d (chi = product of the characters of the applied swaps) and
// returns the packing weight 1 / sqrt(number of images)
template <typename D, typename F>
__device__ inline double orbit_images(const D& d, const int e0[4], F&& fn) {
  int ndist = 0;
  bool eq[2] = {false, false};
#pragma unroll
  for (int sw = 0; sw < 2; ++sw) {
    if (sw >= d.nswap) continue;
    int u, v;
    pair_values(d, sw, e0, u, v);
    eq[sw] = u == v;
    ndist += u != v ? 1 : 0;
  }
#pragma unroll
  for (int bits = 0; bits < 4; ++bits) {
    if (bits >= (1 << d.nswap)) continue;
    if (((bits & 1) && eq[0]) || ((bits & 2) && eq[1])) continue;
    int e[4] = {e0[0], e0[1], e0[2], e0[3]};
    double sg = 1.0;
    if (bits & 1) {
      swap_pair(d, 0, e);
      sg *= d.chi[0];
    }
    if (bits & 2) {
      swap_pair(d, 1, e);
      sg *= d.chi[1];
    }
    fn(e, sg);
  }
  return ndist == 0 ? 1.0 : (ndist == 1 ? 0.70710678118654752440 : 0.5);
}

// NC consecutive values at p as doubles.  vec: the group is whole and p is
// aligned to the group (row length a multiple of NC), so the values move in
// 16-byte loads (two doubles or four floats per load) instead of one request
// per value -- a thread's row segment is contiguous, so element-wise loads
// would issue one memory request per lane per value.
template <typename T, int NC>
__device__ inline void load_group(const T* __restrict__ p, bool vec, double (&v)[NC]) {
  if (vec && NC >= 2) {
    if constexpr (sizeof(T) == 8) {
#pragma unroll
      for (int c = 0; c < NC; c += 2) {
        const double2 q = *reinterpret_cast<const double2*>(p + c);
        v[c] = q.x;
        v[c + 1] = q.y;
      }
    } else if constexpr (NC == 4) {
      const float4 q = *reinterpret_cast<const float4*>(p);
      v[0] = q.x;
      v[1] = q.y;
      v[2] = q.z;
      v[3] = q.w;
    } else {
      const float2 q = *reinterpret_cast<const float2*>(p);
      v[0] = q.x;
      v[1] = q.y;
    }
    return;
  }
#pragma unroll
  for (int c = 0; c < NC; ++c) v[c] = (double)p[c];
}
template <typename T, int NC>
__device__ inline void store_group(T* __restrict__ p, bool vec, const double (&v)[NC]) {
  if (vec && NC >= 2) {
    if constexpr (sizeof(T) == 8) {
#pragma unroll
      for (int c = 0; c < NC; c += 2) *reinterpret_cast<double2*>(p + c) = double2{v[c], v[c + 1]};
    } else if constexpr (NC == 4) {
      *reinterpret_cast<float4*>(p) = float4{(float)v[0], (float)v[1], (float)v[2], (float)v[3]};
    } else {
      *reinterpret_cast<float2*>(p) = float2{(float)v[0], (float)v[1]};
    }
    return;
  }
#pragma unroll
  for (int c = 0; c < NC; ++c) p[c] = (T)v[c];
}

// Column groups: a thread handles NC consecutive alpha columns of one row
// (NC = 4, 2 or 1 by the row length), so index work and Fock values are
// shared by the group and the row data moves in wide loads.
static inline int col_group(int64_t ncol) { return ncol >= 4 ? 4 : (ncol >= 2 ? 2 : 1); }

#define CASPT2_NC_DISPATCH(NCV, KERNEL, GRID, ...)                                             \
  switch (NCV) {                                                                               \
    case 4: hipLaunchKernelGGL((KERNEL<T, 4>), GRID, dim3(256), 0, s, __VA_ARGS__); break;     \
    case 2: hipLaunchKernelGGL((KERNEL<T, 2>), GRID, dim3(256), 0, s, __VA_ARGS__); break;     \
    default: hipLaunchKernelGGL((KERNEL<T, 1>), GRID, dim3(256), 0, s, __VA_ARGS__); break;    \
  }

template <typename T, int NC>
__global__ __launch_bounds__(256) void k_unpack_all(PackInfo p, AllDesc a, int64_t nrows,
                                                    const T* __restrict__ packed, T* __restrict__ out) {
  const int64_t ng = (p.rowlen + NC - 1) / NC;
  const int64_t total = nrows * ng;
  for (int64_t g = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; g < total;
       g += (int64_t)gridDim.x * blockDim.x) {
    const int64_t row = g / ng, c0 = (g - row * ng) * NC;
    int e[4];
    decode_all(a, row, e);
    int64_t off[2];
    double sg[2];
    gather_rows(p, e, off, sg);   // once per row and column group
    const bool full = c0 + NC <= p.rowlen;
    double v[NC];
#pragma unroll
    for (int c = 0; c < NC; ++c) v[c] = 0.0;
#pragma unroll
    for (int ent = 0; ent < 2; ++ent) {
      if (sg[ent] == 0.0) continue;
      const T* src = packed + off[ent] + c0;
      double q[NC];
      if (full && (reinterpret_cast<uintptr_t>(src) & 15) == 0) {
        load_group<T, NC>(src, true, q);
      } else {
#pragma unroll
        for (int c = 0; c < NC; ++c) q[c] = c0 + c < p.rowlen ? (double)src[c] : 0.0;
      }
#pragma unroll
      for (int c = 0; c < NC; ++c) v[c] += sg[ent] * q[c];
    }
    T* dst = out + row * p.rowlen + c0;
    if (full && (reinterpret_cast<uintptr_t>(dst) & 15) == 0) {
      store_group<T, NC>(dst, true, v);
    } else {
#pragma unroll
      for (int c = 0; c < NC; ++c)
        if (c0 + c < p.rowlen) dst[c] = (T)v[c];
    }
  }
}

template <typename T>
hipError_t unpack_all(const PackInfo& p, const AllDesc& a, const T* packed, T* out_all,
                      hipStream_t s) {
  int64_t nrows = 1;
  for (int k = 0; k < a.nslot; ++k) nrows *= a.slot_dim[k];
  if (nrows * p.rowlen == 0) return hipSuccess;
  if (nrows >= ((int64_t)1 << 31)) return hipErrorInvalidValue;
  const int nc = col_group(p.rowlen);
  unsigned grid = cdiv(nrows * ((p.rowlen + nc - 1) / nc), 256);
  if (grid > 65536) grid = 65536;
  CASPT2_NC_DISPATCH(nc, k_unpack_all, dim3(grid), p, a, nrows, packed, out_all)
  return hipGetLastError();
}

template <typename T, int NC>
__global__ __launch_bounds__(256) void k_pack_acc(TermDesc d, AllDesc a, const T* __restrict__ in,
                                                  T* __restrict__ out) {
  const int64_t ng = (d.nalpha + NC - 1) / NC;
  const int64_t total = d.nrow * ng;
  for (int64_t g = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; g < total;
       g += (int64_t)gridDim.x * blockDim.x) {
    const int64_t row = g / ng, c0 = (g - row * ng) * NC;
    int e0[4];
    decode_orbit(d, row, e0);
    const bool full = c0 + NC <= d.nalpha;
    double acc[NC];
#pragma unroll
    for (int c = 0; c < NC; ++c) acc[c] = 0.0;
    const double w = orbit_images(d, e0, [&](const int e[4], double sg) {
      const T* ip = in + encode_all(a, e) * d.nalpha + c0;
      double q[NC];
      if (full && (reinterpret_cast<uintptr_t>(ip) & 15) == 0) {
        load_group<T, NC>(ip, true, q);
      } else {
#pragma unroll
        for (int c = 0; c < NC; ++c) q[c] = c0 + c < d.nalpha ? (double)ip[c] : 0.0;
      }
#pragma unroll
      for (int c = 0; c < NC; ++c) acc[c] += sg * q[c];
    });
    T* op = out + row * d.ldo + c0;
    if (full && (reinterpret_cast<uintptr_t>(op) & 15) == 0) {
      double cur[NC];
      load_group<T, NC>(op, true, cur);
#pragma unroll
      for (int c = 0; c < NC; ++c) cur[c] = (double)(T)(cur[c] + (double)(T)(w * acc[c]));
      store_group<T, NC>(op, true, cur);
    } else {
#pragma unroll
      for (int c = 0; c < NC; ++c)
        if (c0 + c < d.nalpha) op[c] += (T)(w * acc[c]);
    }
  }
}

template <typename T>
hipError_t pack_acc(const TermDesc& d, const AllDesc& a, const T* in_all, T* packed,
                    hipStream_t s) {
  if (d.nrow * d.nalpha == 0) return hipSuccess;
  if (d.nrow >= ((int64_t)1 << 31)) return hipErrorInvalidValue;
  const int nc = col_group(d.nalpha);
  unsigned grid = cdiv(d.nrow * ((d.nalpha + nc - 1) / nc), 256);
  if (grid > 65536) grid = 65536;
  CASPT2_NC_DISPATCH(nc, k_pack_acc, dim3(grid), d, a, in_all, packed)
  return hipGetLastError();
}

// ccvv (slots i, j | a, b, swaps (i,j) and (a,b)) all-orderings sigma into
// its two packed entries: + (i >= j, a >= b) and - (i > j, a > b), added to
// packed + and - (rows of ncol <= 4 values).  A workgroup takes one closed
// pair (i >= j) and a 16 x 16 tile (A, B) of virtual pairs with A >= B: the
// four images (i,j,a,b), (j,i,a,b), (i,j,b,a), (j,i,b,a) of the tile are
// staged through LDS -- the two (a,b)-swapped ones loaded from the mirrored
// tile (B, A) row by row and read back transposed -- so every global access
// runs along contiguous rows instead of gathering 32-byte rows 400 apart.
constexpr int PCC_T = 16;
template <typename T>
__global__ __launch_bounds__(256) void k_pack_ccvv(int nc, int nv, int ncol, const T* __restrict__ in,
                                                   T* __restrict__ plus, T* __restrict__ minus, int ntile) {
  __shared__ double img[4][PCC_T * PCC_T][4];
  const int t = threadIdx.x;
  // tile pair (A >= B) from blockIdx.x, closed pair (i >= j) from blockIdx.y
  int A = 0, rem = blockIdx.x;
  while (rem > A) {   // blockIdx.x = A (A + 1) / 2 + B
    rem -= A + 1;
    ++A;
  }
  const int B = rem;
  int i = 0;
  {
    int r = blockIdx.y;
    while (r > i) {
      r -= i + 1;
      ++i;
    }
    rem = r;
  }
  const int j = rem;
  const int a0 = A * PCC_T, b0 = B * PCC_T;
  const int tl = t / PCC_T, tf = t % PCC_T;   // slow / fast index within the tile
  const int64_t nv2 = (int64_t)nv * nv;
  const int64_t pij = ((int64_t)i * nc + j) * nv2, pji = ((int64_t)j * nc + i) * nv2;
  // identity and (i,j)-swapped images: row (a0 + tl, b0 + tf); the
  // (a,b)-swapped ones: row (b0 + tl, a0 + tf) of the mirrored tile, stored
  // at the transposed position (tf, tl)
  {
    const int a = a0 + tl, b = b0 + tf;
    const bool ok = a < nv && b < nv;
    const int64_t r = (int64_t)a * nv + b;
    const int ba = b0 + tl, bb = a0 + tf;
    const bool ok2 = ba < nv && bb < nv;
    const int64_t r2 = (int64_t)ba * nv + bb;
    for (int c = 0; c < 4; ++c) {
      const bool in_c = c < ncol;
      img[0][t][c] = (ok && in_c) ? (double)in[(pij + r) * ncol + c] : 0.0;
      img[1][t][c] = (ok && in_c) ? (double)in[(pji + r) * ncol + c] : 0.0;
      img[2][tf * PCC_T + tl][c] = (ok2 && in_c) ? (double)in[(pij + r2) * ncol + c] : 0.0;
      img[3][tf * PCC_T + tl][c] = (ok2 && in_c) ? (double)in[(pji + r2) * ncol + c] : 0.0;
    }
  }
  __syncthreads();
  const int a = a0 + tl, b = b0 + tf;
  if (a >= nv || b >= nv || a < b) return;
  const bool dij = i != j, dab = a != b;
  const int64_t npv = (int64_t)nv * (nv + 1) / 2, nmv = (int64_t)nv * (nv - 1) / 2;
  const int64_t rp = ((int64_t)i * (i + 1) / 2 + j) * npv + (int64_t)a * (a + 1) / 2 + b;
  const double w = (dij && dab) ? 0.5 : ((dij || dab) ? 0.70710678118654752440 : 1.0);
  for (int c = 0; c < ncol; ++c) {
    const double r1 = img[0][t][c], r2 = img[1][t][c], r3 = img[2][t][c], r4 = img[3][t][c];
    // distinct images only: (i,j)-swap when i != j, (a,b)-swap when a != b
    const double sp = r1 + (dij ? r2 : 0.0) + (dab ? r3 : 0.0) + ((dij && dab) ? r4 : 0.0);
    plus[rp * ncol + c] += (T)(w * sp);
  }
  if (dij && dab && minus) {
    const int64_t rm = ((int64_t)i * (i - 1) / 2 + j) * nmv + (int64_t)a * (a - 1) / 2 + b;
    for (int c = 0; c < ncol; ++c) {
      const double r1 = img[0][t][c], r2 = img[1][t][c], r3 = img[2][t][c], r4 = img[3][t][c];
      minus[rm * ncol + c] += (T)(0.5 * (r1 - r2 - r3 + r4));
    }
  }
}

template <typename T>
hipError_t pack_ccvv(int nc, int nv, int ncol, const T* in_all, T* plus, T* minus, hipStream_t s) {
  if (nc <= 0 || nv <= 0 || ncol <= 0) return hipSuccess;
  if (ncol > 4) return hipErrorInvalidValue;
  const int ntile = (nv + PCC_T - 1) / PCC_T;
  const int64_t ntp = (int64_t)ntile * (ntile + 1) / 2, npc = (int64_t)nc * (nc + 1) / 2;
  if (ntp > 0x7fffffff || npc > 65535) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_pack_ccvv<T>, dim3((unsigned)ntp, (unsigned)npc), dim3(PCC_T * PCC_T), 0, s, nc, nv, ncol,
                     in_all, plus, minus, ntile);
  return hipGetLastError();
}

// The transpose of k_pack_ccvv: the packed ccvv entries + (i >= j, a >= b)
// and - (i > j, a > b) (rows of ncol <= 4 values) into the all-orderings
// tensor [i][j][a][b][ncol], every element written once (no clearing):
// x[e] = sum_chi chi(pi_e) t_chi[rep(e)] / sqrt(|orbit|).  A workgroup takes
// one closed pair (i >= j) and a 16 x 16 tile (A, B) of virtual pairs with
// A >= B; the images with (a, b) unswapped are written straight from the
// thread that read the packed rows (rows along b), the swapped ones through
// LDS from the transposed position, so every global access runs along
// contiguous rows.
template <typename T>
__global__ __launch_bounds__(256) void k_unpack_ccvv(int nc, int nv, int ncol, const T* __restrict__ plus,
                                                     const T* __restrict__ minus, T* __restrict__ out) {
  __shared__ double sw[2][PCC_T * PCC_T][4];   // (i,j,b,a) and (j,i,b,a) images of rep (a, b)
  const int t = threadIdx.x;
  int A = 0, rem = blockIdx.x;
  while (rem > A) {
    rem -= A + 1;
    ++A;
  }
  const int B = rem;
  int i = 0;
  {
    int r = blockIdx.y;
    while (r > i) {
      r -= i + 1;
      ++i;
    }
    rem = r;
  }
  const int j = rem;
  const int a0 = A * PCC_T, b0 = B * PCC_T;
  const int tl = t / PCC_T, tf = t % PCC_T;
  const int64_t nv2 = (int64_t)nv * nv;
  const int64_t pij = ((int64_t)i * nc + j) * nv2, pji = ((int64_t)j * nc + i) * nv2;
  const int64_t npv = (int64_t)nv * (nv + 1) / 2, nmv = (int64_t)nv * (nv - 1) / 2;
  const bool dij = i != j;
  {
    const int a = a0 + tl, b = b0 + tf;
    double v[4][4];
#pragma unroll
    for (int k = 0; k < 4; ++k)
#pragma unroll
      for (int c = 0; c < 4; ++c) v[k][c] = 0.0;
    const bool rep = a < nv && b < nv && a >= b;
    if (rep) {
      const bool dab = a != b;
      const double w = (dij && dab) ? 0.5 : ((dij || dab) ? 0.70710678118654752440 : 1.0);
      const int64_t rp = ((int64_t)i * (i + 1) / 2 + j) * npv + (int64_t)a * (a + 1) / 2 + b;
      const bool hasm = dij && dab && minus;
      const int64_t rm = hasm ? ((int64_t)i * (i - 1) / 2 + j) * nmv + (int64_t)a * (a - 1) / 2 + b : 0;
      for (int c = 0; c < ncol; ++c) {
        const double pv = w * (double)plus[rp * ncol + c];
        const double mv = hasm ? 0.5 * (double)minus[rm * ncol + c] : 0.0;
        v[0][c] = pv + mv;   // (i, j, a, b)
        v[1][c] = pv - mv;   // (j, i, a, b)
        v[2][c] = pv - mv;   // (i, j, b, a)
        v[3][c] = pv + mv;   // (j, i, b, a)
      }
      const int64_t r = (int64_t)a * nv + b;
      for (int c = 0; c < ncol; ++c) {
        out[(pij + r) * ncol + c] = (T)v[0][c];
        if (dij) out[(pji + r) * ncol + c] = (T)v[1][c];
      }
    }
#pragma unroll
    for (int c = 0; c < 4; ++c) {
      sw[0][t][c] = v[2][c];
      sw[1][t][c] = v[3][c];
    }
  }
  __syncthreads();
  // swapped images: all-orderings row (b0 + tl, a0 + tf), the image of rep
  // (a0 + tf, b0 + tl) held by thread tf * PCC_T + tl
  const int bb = b0 + tl, aa = a0 + tf;
  if (bb >= nv || aa >= nv || !(aa > bb)) return;
  const int src = tf * PCC_T + tl;
  const int64_t r = (int64_t)bb * nv + aa;
  for (int c = 0; c < ncol; ++c) {
    out[(pij + r) * ncol + c] = (T)sw[0][src][c];
    if (dij) out[(pji + r) * ncol + c] = (T)sw[1][src][c];
  }
}

template <typename T>
hipError_t unpack_ccvv(int nc, int nv, int ncol, const T* plus, const T* minus, T* out_all, hipStream_t s) {
  if (nc <= 0 || nv <= 0 || ncol <= 0) return hipSuccess;
  if (ncol > 4) return hipErrorInvalidValue;
  const int ntile = (nv + PCC_T - 1) / PCC_T;
  const int64_t ntp = (int64_t)ntile * (ntile + 1) / 2, npc = (int64_t)nc * (nc + 1) / 2;
  if (ntp > 0x7fffffff || npc > 65535) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_unpack_ccvv<T>, dim3((unsigned)ntp, (unsigned)npc), dim3(PCC_T * PCC_T), 0, s, nc, nv,
                     ncol, plus, minus, out_all);
  return hipGetLastError();
}

// Linear index maps of an expand term, folded on the host: the bra
// all-orderings row and the Fock offset as functions of the ket slot values,
// the free bra slots (not fed from the ket; at most two, looped) and y.
struct ExpandPlan {
  uint32_t kdim[4];          // ket all-orderings dims (1 beyond the ket's slots)
  int64_t ob_k[4], ob_f[2];  // bra row stride per ket slot / per free slot
  int64_t fk[4], ff[2], fy;  // Fock offset coefficients
  uint32_t nf0, nf1;         // free slot ranges (1 if absent)
  // thread order over the ket rows: the ket slots in decode order (fastest
  // first: the slot feeding the highest bra slot, so neighbouring threads
  // write neighbouring bra rows); per position its range, ket row stride,
  // bra row stride and Fock offset coefficient
  uint32_t ddim[4];
  int64_t drk[4], dob[4], dfk[4];
  uint32_t bdim[4];          // bra all-orderings dims (out-parallel form)
  int64_t wk_b[4];           // ket row stride per bra slot (out-parallel form)
  int64_t fb[4];             // Fock offset coefficient per bra slot (out-parallel form)
  int ny;
  int64_t ncol;
};

ExpandPlan make_expand_plan(const CoupleDesc& d) {
  ExpandPlan r{};
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
  for (int l = 0; l < 4; ++l) r.kdim[l] = l < d.ket.nslot ? (uint32_t)d.ket.slot_dim[l] : 1u;
  for (int k = 0; k < 4; ++k) r.bdim[k] = k < d.bra.nslot ? (uint32_t)d.bra.slot_dim[k] : 1u;
  // bra slot k fed by ket slot feed[k] (or free)
  int feed[4] = {-1, -1, -1, -1};
  for (int l = 0; l < d.ket.nslot; ++l) {
    feed[d.ket_src[l]] = l;
    r.wk_b[d.ket_src[l]] += kst[l];
  }
  int free_of[4] = {-1, -1, -1, -1}, nfree = 0;
  r.nf0 = r.nf1 = 1;
  for (int k = 0; k < d.bra.nslot; ++k) {
    if (feed[k] >= 0) {
      r.ob_k[feed[k]] += bst[k];
    } else {
      free_of[k] = nfree;
      r.ob_f[nfree] += bst[k];
      if (nfree == 0) r.nf0 = (uint32_t)d.bra.slot_dim[k];
      else r.nf1 = (uint32_t)d.bra.slot_dim[k];
      ++nfree;
    }
  }
  auto fcoef = [&](int src, int64_t c) {
    if (src == -10) {
      r.fy += c;
      return;
    }
    r.fb[src] += c;
    if (feed[src] >= 0) r.fk[feed[src]] += c;
    else r.ff[free_of[src]] += c;
  };
  fcoef(d.fx_src, d.f_stride);
  fcoef(d.fy_src, 1);
  r.ny = d.ny;
  r.ncol = d.ncol;
  // decode order: ket slots by the bra slot they feed, highest first
  int order[4] = {0, 1, 2, 3};
  const int nk = d.ket.nslot;
  std::sort(order, order + nk, [&](int x, int y) { return d.ket_src[x] > d.ket_src[y]; });
  for (int p = 0; p < 4; ++p) {
    if (p < nk) {
      const int l = order[p];
      r.ddim[p] = r.kdim[l];
      r.drk[p] = kst[l];
      r.dob[p] = r.ob_k[l];
      r.dfk[p] = r.fk[l];
    } else {
      r.ddim[p] = 1u;
      r.drk[p] = r.dob[p] = r.dfk[p] = 0;
    }
  }
  return r;
}

// ket row, bra row base and Fock offset of thread row q (decode order)
__device__ inline void expand_decode(const ExpandPlan& ep, uint32_t q, int64_t& rk, int64_t& ob, int64_t& fo) {
  rk = ob = fo = 0;
#pragma unroll
  for (int p = 0; p < 4; ++p) {
    const uint32_t v = q % ep.ddim[p];
    q /= ep.ddim[p];
    rk += (int64_t)v * ep.drk[p];
    ob += (int64_t)v * ep.dob[p];
    fo += (int64_t)v * ep.dfk[p];
  }
}

// out[bra row(z0, z1)][c0 .. c0 + NC) += sum_y f(z0, z1, y) wreg[y][.] for the
// free values z0 in [zb, ze) and every z1.  The targets of ZB consecutive
// free values are loaded together before any is written back (they are
// distinct rows), so the read latency of the read-modify-write overlaps
// instead of being paid once per free value.
template <typename T, int NC>
__device__ inline void expand_free_range(const ExpandPlan& ep, const double* __restrict__ f, int64_t fo,
                                         int64_t ob, int64_t c0, const double (&wreg)[8][NC], uint32_t zb,
                                         uint32_t ze, T* __restrict__ out) {
  constexpr int ZB = 8;
  const uint32_t nz = (ze - zb) * ep.nf1;
  const bool vec = ep.ncol % NC == 0;
  for (uint32_t zz = 0; zz < nz; zz += ZB) {
    double old[ZB][NC];
    int64_t orow[ZB], frow[ZB];
#pragma unroll
    for (int u = 0; u < ZB; ++u) {
      const uint32_t z = zz + u;
      const uint32_t z0 = zb + z / ep.nf1, z1 = z % ep.nf1;
      orow[u] = (ob + z0 * ep.ob_f[0] + z1 * ep.ob_f[1]) * ep.ncol + c0;
      frow[u] = fo + z0 * ep.ff[0] + z1 * ep.ff[1];
      if (z < nz && vec) {
        load_group<T, NC>(out + orow[u], true, old[u]);
      } else {
#pragma unroll
        for (int c = 0; c < NC; ++c) old[u][c] = (z < nz && c0 + c < ep.ncol) ? (double)out[orow[u] + c] : 0.0;
      }
    }
#pragma unroll
    for (int u = 0; u < ZB; ++u) {
      if (zz + u >= nz) break;
      const double* fr = f + frow[u];
      double acc[NC];
#pragma unroll
      for (int c = 0; c < NC; ++c) acc[c] = old[u][c];
#pragma unroll
      for (int y = 0; y < 8; ++y)
        if (y < ep.ny) {
          const double fv = fr[y * ep.fy];
#pragma unroll
          for (int c = 0; c < NC; ++c) acc[c] += fv * wreg[y][c];
        }
      if (vec) {
        store_group<T, NC>(out + orow[u], true, acc);
      } else {
#pragma unroll
        for (int c = 0; c < NC; ++c)
          if (c0 + c < ep.ncol) out[orow[u] + c] = (T)acc[c];
      }
    }
  }
}

// expand, ket-parallel form: a thread holds the W values of one ket row and
// column group (ny x NC, in registers) and loops over the free bra slots, so
// every W row is read once; out is read-modify-written NC values at a time.
template <typename T, int NC>
__global__ __launch_bounds__(256) void k_couple_expand(ExpandPlan ep, const double* __restrict__ f,
                                                       const T* __restrict__ W, T* __restrict__ out) {
  const uint32_t nrows_k = ep.kdim[0] * ep.kdim[1] * ep.kdim[2] * ep.kdim[3];
  const int64_t ng = (ep.ncol + NC - 1) / NC;
  const int64_t total = (int64_t)nrows_k * ng;
  const int64_t wlen = (int64_t)ep.ny * ep.ncol;
  for (int64_t g = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; g < total;
       g += (int64_t)gridDim.x * blockDim.x) {
    const int64_t tr = g / ng, c0 = (g - tr * ng) * NC;
    int64_t rk, ob, fo;
    expand_decode(ep, (uint32_t)tr, rk, ob, fo);
    double wreg[8][NC];
    const T* w = W + rk * wlen + c0;
    const bool vec = ep.ncol % NC == 0;
#pragma unroll
    for (int y = 0; y < 8; ++y) {
      if (y < ep.ny && vec) {
        load_group<T, NC>(w + (int64_t)y * ep.ncol, true, wreg[y]);
      } else {
#pragma unroll
        for (int c = 0; c < NC; ++c)
          wreg[y][c] = (y < ep.ny && c0 + c < ep.ncol) ? (double)w[(int64_t)y * ep.ncol + c] : 0.0;
      }
    }
    expand_free_range<T, NC>(ep, f, fo, ob, c0, wreg, 0, ep.nf0, out);
  }
}

// Up term with the active contraction fused in: W[rk][y][c] = sum_k X[rk][k]
// G[(y ncol + c)][k] is formed in registers from the ket row (G staged in
// LDS), then expanded over the free bra slots as in k_couple_expand.  The
// free range of the first free slot is split over nsplit threads when the
// ket has few rows.  Thread order: ket row fastest (a wave shares its column
// group and split, so LDS reads of G are broadcasts).
constexpr int FUSED_G_MAX = 6144;   // G entries staged in LDS (48 KB of doubles)
template <typename T, int NC>
__global__ __launch_bounds__(256) void k_couple_up_fused(ExpandPlan ep, int64_t nak, int nsplit,
                                                         const double* __restrict__ f,
                                                         const T* __restrict__ X,
                                                         const T* __restrict__ G, T* __restrict__ out) {
  __shared__ T Gs[FUSED_G_MAX];
  const int64_t glen = (int64_t)ep.ny * ep.ncol * nak;
  for (int64_t i = threadIdx.x; i < glen; i += blockDim.x) Gs[i] = G[i];
  __syncthreads();
  const uint32_t nrows_k = ep.kdim[0] * ep.kdim[1] * ep.kdim[2] * ep.kdim[3];
  const int64_t ng = (ep.ncol + NC - 1) / NC;
  const int64_t total = (int64_t)nrows_k * ng * nsplit;
  const uint32_t chunk = (ep.nf0 + nsplit - 1) / nsplit;
  for (int64_t g = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; g < total;
       g += (int64_t)gridDim.x * blockDim.x) {
    const int64_t tr = g % nrows_k;
    const int64_t rest = g / nrows_k;
    const int64_t cg = rest % ng;
    const uint32_t zs = (uint32_t)(rest / ng);
    const int64_t c0 = cg * NC;
    int64_t rk, ob, fo;
    expand_decode(ep, (uint32_t)tr, rk, ob, fo);
    double wreg[8][NC];
#pragma unroll
    for (int y = 0; y < 8; ++y)
#pragma unroll
      for (int c = 0; c < NC; ++c) wreg[y][c] = 0.0;
    const T* xr = X + rk * nak;
    // the ket row in 16-byte loads when its length allows (four values per step)
    const int64_t nak4 = (nak % 4 == 0) ? nak : 0;
    for (int64_t k = 0; k < nak4; k += 4) {
      double xv[4];
      load_group<T, 4>(xr + k, true, xv);
#pragma unroll
      for (int y = 0; y < 8; ++y)
        if (y < ep.ny) {
#pragma unroll
          for (int c = 0; c < NC; ++c)
            if (c0 + c < ep.ncol) {
              const T* g = Gs + ((int64_t)y * ep.ncol + c0 + c) * nak + k;
              wreg[y][c] += xv[0] * (double)g[0] + xv[1] * (double)g[1] + xv[2] * (double)g[2] +
                            xv[3] * (double)g[3];
            }
        }
    }
    for (int64_t k = nak4; k < nak; ++k) {
      const double xv = (double)xr[k];
#pragma unroll
      for (int y = 0; y < 8; ++y)
        if (y < ep.ny) {
#pragma unroll
          for (int c = 0; c < NC; ++c)
            if (c0 + c < ep.ncol) wreg[y][c] += xv * (double)Gs[((int64_t)y * ep.ncol + c0 + c) * nak + k];
        }
    }
    const uint32_t zb = zs * chunk, ze = zb + chunk < ep.nf0 ? zb + chunk : ep.nf0;
    expand_free_range<T, NC>(ep, f, fo, ob, c0, wreg, zb, ze, out);
  }
}

// expand, output-parallel form (for kets with few rows): a thread per bra
// row and column group; W rows are small and stay in cache.
template <typename T, int NC>
__global__ __launch_bounds__(256) void k_couple_expand_out(ExpandPlan ep, const double* __restrict__ f,
                                                           const T* __restrict__ W, T* __restrict__ out) {
  const uint32_t nrows = ep.bdim[0] * ep.bdim[1] * ep.bdim[2] * ep.bdim[3];
  const int64_t ng = (ep.ncol + NC - 1) / NC;
  const int64_t total = (int64_t)nrows * ng;
  const int64_t wlen = (int64_t)ep.ny * ep.ncol;
  for (int64_t g = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; g < total;
       g += (int64_t)gridDim.x * blockDim.x) {
    const int64_t row = g / ng, c0 = (g - row * ng) * NC;
    uint32_t q = (uint32_t)row;
    const uint32_t b3 = q % ep.bdim[3];
    q /= ep.bdim[3];
    const uint32_t b2 = q % ep.bdim[2];
    q /= ep.bdim[2];
    const uint32_t b1 = q % ep.bdim[1];
    const uint32_t b0 = q / ep.bdim[1];
    const int64_t rk = b0 * ep.wk_b[0] + b1 * ep.wk_b[1] + b2 * ep.wk_b[2] + b3 * ep.wk_b[3];
    const double* fr = f + b0 * ep.fb[0] + b1 * ep.fb[1] + b2 * ep.fb[2] + b3 * ep.fb[3];
    const T* w = W + rk * wlen + c0;
    T* op = out + row * ep.ncol + c0;
    const bool vec = ep.ncol % NC == 0;
    double acc[NC];
    if (vec) {
      load_group<T, NC>(op, true, acc);
    } else {
#pragma unroll
      for (int c = 0; c < NC; ++c) acc[c] = c0 + c < ep.ncol ? (double)op[c] : 0.0;
    }
#pragma unroll
    for (int y = 0; y < 8; ++y)
      if (y < ep.ny) {
        const double fv = fr[y * ep.fy];
        double wv[NC];
        if (vec) {
          load_group<T, NC>(w + (int64_t)y * ep.ncol, true, wv);
        } else {
#pragma unroll
          for (int c = 0; c < NC; ++c) wv[c] = c0 + c < ep.ncol ? (double)w[(int64_t)y * ep.ncol + c] : 0.0;
        }
#pragma unroll
        for (int c = 0; c < NC; ++c) acc[c] += fv * wv[c];
      }
    if (vec) {
      store_group<T, NC>(op, true, acc);
    } else {
#pragma unroll
      for (int c = 0; c < NC; ++c)
        if (c0 + c < ep.ncol) op[c] = (T)acc[c];
    }
  }
}

template <typename T>
hipError_t couple_expand(const CoupleDesc& d, const double* f, const T* W, T* out_all,
                         hipStream_t s, int mode) {
  if (d.ny > 8) return hipErrorInvalidValue;
  int64_t nrows_k = 1, nrows_b = 1;
  for (int k = 0; k < d.ket.nslot; ++k) nrows_k *= d.ket.slot_dim[k];
  for (int k = 0; k < d.bra.nslot; ++k) nrows_b *= d.bra.slot_dim[k];
  if (nrows_b * d.ncol == 0) return hipSuccess;
  if (nrows_b >= ((int64_t)1 << 31)) return hipErrorInvalidValue;
  // each ket slot feeds a distinct bra slot; at most two bra slots are free
  {
    int fed[4] = {0, 0, 0, 0};
    for (int l = 0; l < d.ket.nslot; ++l) {
      if (d.ket_src[l] < 0 || d.ket_src[l] >= d.bra.nslot || fed[d.ket_src[l]]) return hipErrorInvalidValue;
      fed[d.ket_src[l]] = 1;
    }
    if (d.bra.nslot - d.ket.nslot > 2) return hipErrorInvalidValue;
  }
  const ExpandPlan ep = make_expand_plan(d);
  const int nc = col_group(d.ncol);
  const int64_t ng = (d.ncol + nc - 1) / nc;
  const bool ket_par = mode == 1 || (mode == 0 && nrows_k * ng >= (int64_t)1 << 18);
  if (ket_par) {
    unsigned grid = cdiv(nrows_k * ng, 256);
    if (grid > 65536) grid = 65536;
    CASPT2_NC_DISPATCH(nc, k_couple_expand, dim3(grid), ep, f, W, out_all)
  } else {
    unsigned grid = cdiv(nrows_b * ng, 256);
    if (grid > 65536) grid = 65536;
    CASPT2_NC_DISPATCH(nc, k_couple_expand_out, dim3(grid), ep, f, W, out_all)
  }
  return hipGetLastError();
}

// fused only in the ket-parallel regime (many ket rows): with few ket rows
// and large free ranges the output-parallel expand of a precomputed W is
// faster
template <typename T>
bool couple_up_fusable(const CoupleDesc& d, int64_t nak) {
  int64_t nrows_k = 1;
  for (int k = 0; k < d.ket.nslot; ++k) nrows_k *= d.ket.slot_dim[k];
  const int64_t ng = (d.ncol + col_group(d.ncol) - 1) / col_group(d.ncol);
  return d.ny <= 8 && (int64_t)d.ny * d.ncol * nak <= FUSED_G_MAX && nak > 0 &&
         nrows_k * ng >= ((int64_t)1 << 18);
}

template <typename T>
hipError_t couple_up_fused(const CoupleDesc& d, const double* f, const T* X_all, int64_t nak, const T* G,
                           T* out_all, hipStream_t s) {
  if (!couple_up_fusable<T>(d, nak)) return hipErrorInvalidValue;
  int64_t nrows_k = 1, nrows_b = 1;
  for (int k = 0; k < d.ket.nslot; ++k) nrows_k *= d.ket.slot_dim[k];
  for (int k = 0; k < d.bra.nslot; ++k) nrows_b *= d.bra.slot_dim[k];
  if (nrows_b * d.ncol == 0 || nrows_k == 0) return hipSuccess;
  if (nrows_b >= ((int64_t)1 << 31)) return hipErrorInvalidValue;
  {
    int fed[4] = {0, 0, 0, 0};
    for (int l = 0; l < d.ket.nslot; ++l) {
      if (d.ket_src[l] < 0 || d.ket_src[l] >= d.bra.nslot || fed[d.ket_src[l]]) return hipErrorInvalidValue;
      fed[d.ket_src[l]] = 1;
    }
    if (d.bra.nslot - d.ket.nslot > 2) return hipErrorInvalidValue;
  }
  const ExpandPlan ep = make_expand_plan(d);
  const int nc = col_group(d.ncol);
  const int64_t ng = (d.ncol + nc - 1) / nc;
  // split the first free range until about 2M threads run, keeping >= 8
  // free values per thread
  int nsplit = 1;
  while (nsplit * 2 <= (int)ep.nf0 / 8 && nrows_k * ng * nsplit < ((int64_t)1 << 21)) nsplit *= 2;
  unsigned grid = cdiv(nrows_k * ng * nsplit, 256);
  if (grid > 65536) grid = 65536;
  CASPT2_NC_DISPATCH(nc, k_couple_up_fused, dim3(grid), ep, nak, nsplit, f, X_all, G, out_all)
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// reduce (down terms):  Y[e_b][y ncol + a] = sum_z f(e_b, z, y) X[e_k(e_b, z)][a]
// The index maps are linear in the slot values, so the host folds them into
// per-slot coefficients (ket row strides and f offsets); the kernel keeps the
// slot values in registers (no per-thread arrays indexed at run time).
// ---------------------------------------------------------------------------
struct ReducePlan {
  int nb;                 // bra slots
  uint32_t bdim[4];       // bra all-orderings dims (1 beyond nb)
  int64_t xs_b[4], xs_z[2];   // ket all-orderings row stride per bra slot / summed label
  int64_t fs_b[4], fs_z[2], fs_y;
  uint32_t nz1, nz;       // summed labels: z = z0 * nz1 + z1, nz = nz0 * nz1
  int ksrc[4];            // ket slot sources (packed ket gather): bra slot k, or -1 - s
  int ny;
  int64_t ncol;
};

ReducePlan make_reduce_plan(const CoupleDesc& d) {
  ReducePlan r{};
  r.nb = d.bra.nslot;
  for (int k = 0; k < 4; ++k) r.bdim[k] = k < d.bra.nslot ? (uint32_t)d.bra.slot_dim[k] : 1u;
  int64_t kst[4] = {0, 0, 0, 0}, st = 1;
  for (int l = d.ket.nslot - 1; l >= 0; --l) {
    kst[l] = st;
    st *= d.ket.slot_dim[l];
  }
  for (int l = 0; l < 4; ++l) r.ksrc[l] = 0;
  for (int l = 0; l < d.ket.nslot; ++l) {
    const int src = d.ket_src[l];
    r.ksrc[l] = src;
    if (src >= 0) r.xs_b[src] += kst[l];
    else r.xs_z[-1 - src] += kst[l];
  }
  auto fcoef = [&](int src, int64_t c) {
    if (src >= 0) r.fs_b[src] += c;
    else if (src == -10) r.fs_y += c;
    else r.fs_z[-1 - src] += c;
  };
  fcoef(d.fx_src, d.f_stride);
  fcoef(d.fy_src, 1);
  const uint32_t nz0 = d.nsum > 0 ? (uint32_t)d.sum_dim[0] : 1u;
  r.nz1 = d.nsum > 1 ? (uint32_t)d.sum_dim[1] : 1u;
  r.nz = nz0 * r.nz1;
  r.ny = d.ny;
  r.ncol = d.ncol;
  return r;
}

__device__ inline int pick_src(int src, int e0, int e1, int e2, int e3, int z0, int z1) {
  switch (src) {
    case 0: return e0;
    case 1: return e1;
    case 2: return e2;
    case 3: return e3;
    case -1: return z0;
    default: return z1;
  }
}

// all-orderings values x[i, j, a, b][col .. col + VC) of the ccvv amplitude
// (packed entries '+' (i >= j, a >= b) and '-' (i > j, a > b)), added with
// weight fw into acc[y][.] for the nyv Fock values fv[y]
template <typename T, int VC>
__device__ inline void gather_ccvv(const PackInfo& p, const T* __restrict__ base, int i, int j, int a, int b,
                                   int64_t col, int nvc, double v[VC]) {
  const bool s0 = i < j, s1 = a < b;
  const int hi0 = s0 ? j : i, lo0 = s0 ? i : j, hi1 = s1 ? b : a, lo1 = s1 ? a : b;
  const int64_t nv = p.slot_dim[2];
  const int64_t rp = ((int64_t)hi0 * (hi0 + 1) / 2 + lo0) * (nv * (nv + 1) / 2) + (int64_t)hi1 * (hi1 + 1) / 2 + lo1;
  const T* xp = base + p.offset[0] + rp * p.rowlen + col;
  const bool d0 = hi0 != lo0, d1 = hi1 != lo1;
#pragma unroll
  for (int c = 0; c < VC; ++c) v[c] = c < nvc ? (double)xp[c] : 0.0;
  if (d0 && d1) {
    const int64_t rm = ((int64_t)hi0 * (hi0 - 1) / 2 + lo0) * (nv * (nv - 1) / 2) + (int64_t)hi1 * (hi1 - 1) / 2 + lo1;
    const double sg = (s0 != s1) ? -1.0 : 1.0;
    const T* xm = base + p.offset[1] + rm * p.rowlen + col;
#pragma unroll
    for (int c = 0; c < VC; ++c) v[c] = 0.5 * (v[c] + (c < nvc ? sg * (double)xm[c] : 0.0));
  } else if (d0 || d1) {
#pragma unroll
    for (int c = 0; c < VC; ++c) v[c] *= 0.70710678118654752440;
  }
}

// a workgroup handles R bra rows; thread = (column group of VC columns, row,
// z part); partial sums over the summed labels are combined through LDS
template <typename T, bool PACKED, int VC>
__global__ __launch_bounds__(256) void k_couple_reduce(ReducePlan rp, PackInfo pk, int P, int CG,
                                                       const double* __restrict__ f,
                                                       const T* __restrict__ X,
                                                       T* __restrict__ Y) {
  __shared__ double part[256 * 8];
  const uint32_t nrows = rp.bdim[0] * rp.bdim[1] * rp.bdim[2] * rp.bdim[3];
  const int R = 256 / (CG * P);
  const int t = threadIdx.x;
  const int zp = t / (R * CG);
  const int rr = t % (R * CG);
  const int r = rr / CG;
  const int64_t a0 = ((int64_t)blockIdx.y * CG + rr % CG) * VC;
  const int nvc = (int)(rp.ncol - a0 < VC ? rp.ncol - a0 : VC);
  const bool acol = a0 < rp.ncol;
  const int64_t width = (int64_t)rp.ny * rp.ncol;
  for (int64_t row0 = (int64_t)blockIdx.x * R; row0 < (int64_t)nrows; row0 += (int64_t)gridDim.x * R) {
    const int64_t row = row0 + r;
    const bool live = zp < P && row < (int64_t)nrows && acol;
    double acc[8][VC];
#pragma unroll
    for (int y = 0; y < 8; ++y)
#pragma unroll
      for (int c = 0; c < VC; ++c) acc[y][c] = 0.0;
    if (live) {
      uint32_t q = (uint32_t)row;
      const uint32_t b3 = q % rp.bdim[3];
      q /= rp.bdim[3];
      const uint32_t b2 = q % rp.bdim[2];
      q /= rp.bdim[2];
      const uint32_t b1 = q % rp.bdim[1];
      const uint32_t b0 = q / rp.bdim[1];   // slots beyond nb have dim 1: value 0
      const int64_t xb = b0 * rp.xs_b[0] + b1 * rp.xs_b[1] + b2 * rp.xs_b[2] + b3 * rp.xs_b[3];
      const int64_t fb = b0 * rp.fs_b[0] + b1 * rp.fs_b[1] + b2 * rp.fs_b[2] + b3 * rp.fs_b[3];
      for (uint32_t zz = zp; zz < rp.nz; zz += P) {
        const uint32_t z0 = zz / rp.nz1, z1 = zz - z0 * rp.nz1;
        double xv[VC];
        if (PACKED) {
          const int k0 = pick_src(rp.ksrc[0], b0, b1, b2, b3, z0, z1);
          const int k1 = pick_src(rp.ksrc[1], b0, b1, b2, b3, z0, z1);
          const int k2 = pick_src(rp.ksrc[2], b0, b1, b2, b3, z0, z1);
          const int k3 = pick_src(rp.ksrc[3], b0, b1, b2, b3, z0, z1);
          gather_ccvv<T, VC>(pk, X, k0, k1, k2, k3, a0, nvc, xv);
        } else {
          const T* xp = X + (xb + z0 * rp.xs_z[0] + z1 * rp.xs_z[1]) * rp.ncol + a0;
#pragma unroll
          for (int c = 0; c < VC; ++c) xv[c] = c < nvc ? (double)xp[c] : 0.0;
        }
        const double* fr = f + fb + z0 * rp.fs_z[0] + z1 * rp.fs_z[1];
#pragma unroll
        for (int y = 0; y < 8; ++y)
          if (y < rp.ny) {
            const double fv = fr[y * rp.fs_y];
#pragma unroll
            for (int c = 0; c < VC; ++c) acc[y][c] += fv * xv[c];
          }
      }
    }
#pragma unroll
    for (int c = 0; c < VC; ++c) {
#pragma unroll
      for (int y = 0; y < 8; ++y) part[y * 256 + t] = acc[y][c];
      __syncthreads();
      if (live && zp == 0 && c < nvc) {
        for (int y = 0; y < rp.ny; ++y) {
          double sum = 0.0;
          for (int qq = 0; qq < P; ++qq) sum += part[y * 256 + t + qq * R * CG];
          Y[row * width + (int64_t)y * rp.ncol + a0 + c] = (T)sum;
        }
      }
      __syncthreads();
    }
  }
}

template <typename T, bool PACKED, int VC>
hipError_t launch_reduce_vc(const CoupleDesc& d, const PackInfo& pk, const double* f, const T* X, T* Y,
                            hipStream_t s) {
  int64_t nrows = 1;
  for (int k = 0; k < d.bra.nslot; ++k) nrows *= d.bra.slot_dim[k];
  const ReducePlan rp = make_reduce_plan(d);
  const int nz = (int)rp.nz;
  const int64_t ngroups = (d.ncol + VC - 1) / VC;
  int CG = (int)(ngroups < 64 ? ngroups : 64);
  // rows per wave first (coalesced ket rows), then z parts; with few bra
  // rows, spread the summed labels over more lanes
  auto zparts = [&](int rw) {
    int p = 1;
    while (p * 2 <= nz && p * 2 * rw * CG <= 256) p *= 2;
    return p;
  };
  int Rw = 1;
  while (Rw * 2 * CG <= 64) Rw *= 2;
  while (Rw > 1 && nrows * CG * zparts(Rw) < ((int64_t)1 << 20)) Rw /= 2;
  // few bra rows (under 64) and few threads in all (e.g. 30 rows summed
  // over 12 000 labels): fewer column groups per workgroup (the others go
  // to grid y) and more z parts, until about 2^20 threads -- while the
  // combination of the parts (P ny additions by one thread) stays within
  // 256 and a z part keeps at least two column groups
  while (Rw == 1 && CG > 2 && nrows < 64 && nrows * ngroups * zparts(1) < ((int64_t)1 << 20) &&
         zparts(1) * 2 <= nz && zparts(1) * 2 * rp.ny <= 256)
    CG /= 2;
  const int P = zparts(Rw);
  const int R = 256 / (CG * P);
  unsigned gx = cdiv(nrows, R);
  if (gx > 65536) gx = 65536;
  const unsigned gy = cdiv(ngroups, CG);
  hipLaunchKernelGGL((k_couple_reduce<T, PACKED, VC>), dim3(gx, gy), dim3(256), 0, s, rp, pk, P, CG, f, X, Y);
  return hipGetLastError();
}

template <typename T, bool PACKED>
hipError_t launch_reduce(const CoupleDesc& d, const PackInfo& pk, const double* f, const T* X, T* Y,
                         hipStream_t s) {
  if (d.ny > 8) return hipErrorInvalidValue;
  int64_t nrows = 1;
  for (int k = 0; k < d.bra.nslot; ++k) nrows *= d.bra.slot_dim[k];
  if (nrows * d.ncol == 0) return hipSuccess;
  if (nrows >= ((int64_t)1 << 31)) return hipErrorInvalidValue;
  if (d.ncol == 1) return launch_reduce_vc<T, PACKED, 1>(d, pk, f, X, Y, s);
  if (d.ncol == 2) return launch_reduce_vc<T, PACKED, 2>(d, pk, f, X, Y, s);
  return launch_reduce_vc<T, PACKED, 4>(d, pk, f, X, Y, s);
}

template <typename T>
hipError_t couple_reduce(const CoupleDesc& d, const double* f, const T* X, T* Y,
                         hipStream_t s) {
  return launch_reduce<T, false>(d, PackInfo{}, f, X, Y, s);
}

// the packed ket must be ccvv-shaped: slots (c, c, v, v), swaps (0,1) and
// (2,3), entries '+' (1, 1) and '-' (-1, -1), rows of ncol values
template <typename T>
hipError_t couple_reduce_packed(const CoupleDesc& d, const PackInfo& pk, const double* f, const T* x,
                                T* Y, hipStream_t s) {
  if (pk.rowlen != d.ncol || pk.nslot != 4 || pk.nswap != 2 || pk.nent != 2 || pk.swap_k[0] != 0 ||
      pk.swap_l[0] != 1 || pk.swap_k[1] != 2 || pk.swap_l[1] != 3 || pk.chi[0][0] != 1 || pk.chi[0][1] != 1 ||
      pk.chi[1][0] != -1 || pk.chi[1][1] != -1 || d.ket.nslot != 4)
    return hipErrorInvalidValue;
  return launch_reduce<T, true>(d, pk, f, x, Y, s);
}

template <typename T>
__global__ __launch_bounds__(256) void k_rows_small_gemm(int64_t nrows, int nab, int width,
                                                         const T* __restrict__ Y, const T* __restrict__ G,
                                                         T* __restrict__ out) {
  __shared__ double gs[64];
  for (int k = threadIdx.x; k < nab * width; k += blockDim.x) gs[k] = (double)G[k];
  __syncthreads();
  for (int64_t r = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; r < nrows;
       r += (int64_t)gridDim.x * blockDim.x) {
    double y[8];
#pragma unroll
    for (int c = 0; c < 8; ++c) y[c] = c < width ? (double)Y[r * width + c] : 0.0;
#pragma unroll
    for (int a = 0; a < 8; ++a) {
      if (a >= nab) break;
      double acc = 0.0;
#pragma unroll
      for (int c = 0; c < 8; ++c)
        if (c < width) acc += y[c] * gs[a * width + c];
      out[r * nab + a] += (T)acc;
    }
  }
}

// the same for nab = width = 4 in FP64: rows move as two 16-byte loads
__global__ __launch_bounds__(256) void k_rows_small_gemm4(int64_t nrows, const double* __restrict__ Y,
                                                          const double* __restrict__ G, double* __restrict__ out) {
  __shared__ double gs[16];
  if (threadIdx.x < 16) gs[threadIdx.x] = G[threadIdx.x];
  __syncthreads();
  for (int64_t r = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; r < nrows;
       r += (int64_t)gridDim.x * blockDim.x) {
    const double2* yp = reinterpret_cast<const double2*>(Y + r * 4);
    double2* op = reinterpret_cast<double2*>(out + r * 4);
    const double2 y01 = yp[0], y23 = yp[1];
    double2 o01 = op[0], o23 = op[1];
    const double y[4] = {y01.x, y01.y, y23.x, y23.y};
    double acc[4];
#pragma unroll
    for (int a = 0; a < 4; ++a)
      acc[a] = y[0] * gs[4 * a] + y[1] * gs[4 * a + 1] + y[2] * gs[4 * a + 2] + y[3] * gs[4 * a + 3];
    o01.x += acc[0];
    o01.y += acc[1];
    o23.x += acc[2];
    o23.y += acc[3];
    op[0] = o01;
    op[1] = o23;
  }
}

template <typename T>
hipError_t rows_small_gemm(int64_t nrows, int nab, int width, const T* Y, const T* G, T* out, hipStream_t s) {
  if (nab < 1 || nab > 8 || width < 1 || width > 8) return hipErrorInvalidValue;
  if (nrows <= 0) return hipSuccess;
  unsigned grid = cdiv(nrows, 256);
  if (grid > 65536) grid = 65536;
  const bool al16 = ((uintptr_t)Y % 16 == 0) && ((uintptr_t)out % 16 == 0);
  if (std::is_same<T, double>::value && nab == 4 && width == 4 && al16)
    hipLaunchKernelGGL(k_rows_small_gemm4, dim3(grid), dim3(256), 0, s, nrows, (const double*)Y, (const double*)G,
                       (double*)out);
  else
    hipLaunchKernelGGL(k_rows_small_gemm<T>, dim3(grid), dim3(256), 0, s, nrows, nab, width, Y, G, out);
  return hipGetLastError();
}

#define CASPT2_COUPLE_INSTANCES(T)                                                                  \
  template hipError_t rows_small_gemm<T>(int64_t, int, int, const T*, const T*, T*, hipStream_t);  \
  template hipError_t unpack_all<T>(const PackInfo&, const AllDesc&, const T*, T*, hipStream_t);   \
  template hipError_t pack_acc<T>(const TermDesc&, const AllDesc&, const T*, T*, hipStream_t);     \
  template hipError_t pack_ccvv<T>(int, int, int, const T*, T*, T*, hipStream_t);                   \
  template hipError_t unpack_ccvv<T>(int, int, int, const T*, const T*, T*, hipStream_t);           \
  template hipError_t couple_expand<T>(const CoupleDesc&, const double*, const T*, T*, hipStream_t, int); \
  template hipError_t couple_reduce<T>(const CoupleDesc&, const double*, const T*, T*, hipStream_t);  \
  template hipError_t couple_reduce_packed<T>(const CoupleDesc&, const PackInfo&, const double*,     \
                                              const T*, T*, hipStream_t);                           \
  template bool couple_up_fusable<T>(const CoupleDesc&, int64_t);                                  \
  template hipError_t couple_up_fused<T>(const CoupleDesc&, const double*, const T*, int64_t,        \
                                         const T*, T*, hipStream_t);
CASPT2_COUPLE_INSTANCES(double)
CASPT2_COUPLE_INSTANCES(float)
#undef CASPT2_COUPLE_INSTANCES

}  // namespace caspt2
