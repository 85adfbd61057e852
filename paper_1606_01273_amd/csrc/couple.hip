// Coupling kernels (Fock couplings between excitation blocks) and the
// packed <-> all-orderings conversions, for FP64 and FP32 data.
#include "device_common.hpp"
#include "kernels.hpp"

namespace caspt2 {

static inline unsigned cdiv(int64_t a, int64_t b) { return (unsigned)((a + b - 1) / b); }

template <typename T>
__global__ void k_unpack_all(PackInfo p, AllDesc a, int64_t nrows, const T* __restrict__ packed,
                             T* __restrict__ out) {
  const int64_t total = nrows * p.rowlen;
  for (int64_t g = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; g < total;
       g += (int64_t)gridDim.x * blockDim.x) {
    const int64_t row = g / p.rowlen, c = g % p.rowlen;
    int e[4] = {0, 0, 0, 0};
    decode_all(a, row, e);
    out[g] = (T)gather_all(p, packed, e, c);
  }
}

template <typename T>
hipError_t unpack_all(const PackInfo& p, const AllDesc& a, const T* packed, T* out_all,
                      hipStream_t s) {
  int64_t nrows = 1;
  for (int k = 0; k < a.nslot; ++k) nrows *= a.slot_dim[k];
  const int64_t total = nrows * p.rowlen;
  if (total == 0) return hipSuccess;
  unsigned grid = cdiv(total, 256);
  if (grid > 65536) grid = 65536;
  hipLaunchKernelGGL(k_unpack_all<T>, dim3(grid), dim3(256), 0, s, p, a, nrows, packed, out_all);
  return hipGetLastError();
}

template <typename T>
__global__ void k_pack_acc(TermDesc d, AllDesc a, const T* __restrict__ in,
                           T* __restrict__ out) {
  const int64_t total = d.nrow * d.nalpha;
  for (int64_t g = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; g < total;
       g += (int64_t)gridDim.x * blockDim.x) {
    const int64_t row = g / d.nalpha, c = g % d.nalpha;
    int e0[4] = {0, 0, 0, 0};
    decode_orbit(d, row, e0);
    int ndistinct = 0;
    for (int s = 0; s < d.nswap; ++s)
      if (e0[d.swap_k[s]] != e0[d.swap_l[s]]) ++ndistinct;
    const double w = 1.0 / sqrt((double)(1 << ndistinct));
    double acc = 0.0;
    for (int bits = 0; bits < (1 << d.nswap); ++bits) {
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
      acc += sg * (double)in[encode_all(a, e) * d.nalpha + c];
    }
    out[row * d.ldo + c] += (T)(w * acc);
  }
}

template <typename T>
hipError_t pack_acc(const TermDesc& d, const AllDesc& a, const T* in_all, T* packed,
                    hipStream_t s) {
  const int64_t total = d.nrow * d.nalpha;
  if (total == 0) return hipSuccess;
  unsigned grid = cdiv(total, 256);
  if (grid > 65536) grid = 65536;
  hipLaunchKernelGGL(k_pack_acc<T>, dim3(grid), dim3(256), 0, s, d, a, in_all, packed);
  return hipGetLastError();
}

// expand: one thread per (ket row, alpha column); the bra slots that are not
// fed from the ket (the Fock index slots) are looped inside the thread, so
// every W row is read once.
template <typename T>
__global__ void k_couple_expand(CoupleDesc d, const double* __restrict__ f,
                                const T* __restrict__ W, T* __restrict__ out) {
  int64_t nrows_k = 1;
  for (int k = 0; k < d.ket.nslot; ++k) nrows_k *= d.ket.slot_dim[k];
  const int64_t total = nrows_k * d.ncol;
  const int64_t wlen = (int64_t)d.ny * d.ncol;
  // bra slots not fed from the ket
  int free_slot[2] = {-1, -1}, nfree = 0;
  for (int k = 0; k < d.bra.nslot; ++k) {
    bool fed = false;
    for (int l = 0; l < d.ket.nslot; ++l)
      if (d.ket_src[l] == k) fed = true;
    if (!fed && nfree < 2) free_slot[nfree++] = k;
  }
  const int n0 = nfree > 0 ? d.bra.slot_dim[free_slot[0]] : 1;
  const int n1 = nfree > 1 ? d.bra.slot_dim[free_slot[1]] : 1;
  const int z[2] = {0, 0};
  for (int64_t g = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; g < total;
       g += (int64_t)gridDim.x * blockDim.x) {
    const int64_t rk = g / d.ncol, a = g % d.ncol;
    int ek[4] = {0, 0, 0, 0}, e[4] = {0, 0, 0, 0};
    decode_all(d.ket, rk, ek);
    for (int l = 0; l < d.ket.nslot; ++l) e[d.ket_src[l]] = ek[l];
    double wreg[8];
    const T* w = W + rk * wlen + a;
    for (int y = 0; y < d.ny; ++y) wreg[y] = (double)w[(int64_t)y * d.ncol];
    for (int z0 = 0; z0 < n0; ++z0) {
      if (nfree > 0) e[free_slot[0]] = z0;
      for (int z1 = 0; z1 < n1; ++z1) {
        if (nfree > 1) e[free_slot[1]] = z1;
        double acc = 0.0;
        for (int y = 0; y < d.ny; ++y)
          acc += f[(int64_t)src_value(d.fx_src, e, z, y) * d.f_stride + src_value(d.fy_src, e, z, y)] *
                 wreg[y];
        out[encode_all(d.bra, e) * d.ncol + a] += (T)acc;
      }
    }
  }
}

// expand, output-parallel form (for kets with few rows): one thread per
// (bra row, alpha column); W rows are small and stay in cache.
template <typename T>
__global__ void k_couple_expand_out(CoupleDesc d, const double* __restrict__ f,
                                    const T* __restrict__ W, T* __restrict__ out) {
  int64_t nrows = 1;
  for (int k = 0; k < d.bra.nslot; ++k) nrows *= d.bra.slot_dim[k];
  const int64_t total = nrows * d.ncol;
  const int64_t wlen = (int64_t)d.ny * d.ncol;
  const int z[2] = {0, 0};
  for (int64_t g = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; g < total;
       g += (int64_t)gridDim.x * blockDim.x) {
    const int64_t row = g / d.ncol, a = g % d.ncol;
    int e[4] = {0, 0, 0, 0}, ek[4] = {0, 0, 0, 0};
    decode_all(d.bra, row, e);
    for (int l = 0; l < d.ket.nslot; ++l) ek[l] = e[d.ket_src[l]];
    const T* w = W + encode_all(d.ket, ek) * wlen + a;
    double acc = 0.0;
    for (int y = 0; y < d.ny; ++y)
      acc += f[(int64_t)src_value(d.fx_src, e, z, y) * d.f_stride + src_value(d.fy_src, e, z, y)] *
             (double)w[(int64_t)y * d.ncol];
    out[g] += (T)acc;
  }
}

template <typename T>
hipError_t couple_expand(const CoupleDesc& d, const double* f, const T* W, T* out_all,
                         hipStream_t s) {
  if (d.ny > 8) return hipErrorInvalidValue;
  int64_t nrows_k = 1, nrows_b = 1;
  for (int k = 0; k < d.ket.nslot; ++k) nrows_k *= d.ket.slot_dim[k];
  for (int k = 0; k < d.bra.nslot; ++k) nrows_b *= d.bra.slot_dim[k];
  if (nrows_b * d.ncol == 0) return hipSuccess;
  if (nrows_k * d.ncol >= (int64_t)1 << 20) {
    unsigned grid = cdiv(nrows_k * d.ncol, 256);
    if (grid > 65536) grid = 65536;
    hipLaunchKernelGGL(k_couple_expand<T>, dim3(grid), dim3(256), 0, s, d, f, W, out_all);
  } else {
    unsigned grid = cdiv(nrows_b * d.ncol, 256);
    if (grid > 65536) grid = 65536;
    hipLaunchKernelGGL(k_couple_expand_out<T>, dim3(grid), dim3(256), 0, s, d, f, W, out_all);
  }
  return hipGetLastError();
}

// reduce: a workgroup handles R bra rows; thread = (row, alpha column, z part);
// partial sums over the summed external labels are combined through LDS.
template <typename T>
__global__ __launch_bounds__(256) void k_couple_reduce(CoupleDesc d, int P, int CT,
                                                       const double* __restrict__ f,
                                                       const T* __restrict__ X,
                                                       T* __restrict__ Y) {
  __shared__ double part[256 * 8];
  int64_t nrows = 1;
  for (int k = 0; k < d.bra.nslot; ++k) nrows *= d.bra.slot_dim[k];
  const int per_row = CT * P;
  const int R = 256 / per_row;
  const int n0 = d.nsum > 0 ? d.sum_dim[0] : 1;
  const int n1 = d.nsum > 1 ? d.sum_dim[1] : 1;
  const int nz = n0 * n1;
  const int t = threadIdx.x;
  // lanes: column fastest, then row, then z part (coalesced row reads)
  const int zp = t / (R * CT);
  const int rr = t % (R * CT);
  const int r = rr / CT;
  const int64_t a = (int64_t)blockIdx.y * CT + rr % CT;
  const bool acol = a < d.ncol;
  const int64_t width = (int64_t)d.ny * d.ncol;
  for (int64_t row0 = (int64_t)blockIdx.x * R; row0 < nrows; row0 += (int64_t)gridDim.x * R) {
    const int64_t row = row0 + r;
    const bool live = zp < P && row < nrows && acol;
    double acc[8] = {0, 0, 0, 0, 0, 0, 0, 0};
    if (live) {
      int e[4] = {0, 0, 0, 0};
      decode_all(d.bra, row, e);
      for (int zz = zp; zz < nz; zz += P) {
        const int zv[2] = {zz / n1, zz % n1};
        int ek[4] = {0, 0, 0, 0};
        for (int l = 0; l < d.ket.nslot; ++l) ek[l] = src_value(d.ket_src[l], e, zv, 0);
        const double xv = (double)X[encode_all(d.ket, ek) * d.ncol + a];
        for (int y = 0; y < d.ny; ++y)
          acc[y] += f[(int64_t)src_value(d.fx_src, e, zv, y) * d.f_stride + src_value(d.fy_src, e, zv, y)] * xv;
      }
    }
    for (int y = 0; y < 8; ++y) part[y * 256 + t] = acc[y];
    __syncthreads();
    if (live && zp == 0) {
      for (int y = 0; y < d.ny; ++y) {
        double sum = 0.0;
        for (int q = 0; q < P; ++q) sum += part[y * 256 + t + q * R * CT];
        Y[row * width + (int64_t)y * d.ncol + a] = (T)sum;
      }
    }
    __syncthreads();
  }
}

template <typename T>
hipError_t couple_reduce(const CoupleDesc& d, const double* f, const T* X, T* Y,
                         hipStream_t s) {
  if (d.ny > 8) return hipErrorInvalidValue;
  int64_t nrows = 1;
  for (int k = 0; k < d.bra.nslot; ++k) nrows *= d.bra.slot_dim[k];
  if (nrows * d.ncol == 0) return hipSuccess;
  const int n0 = d.nsum > 0 ? d.sum_dim[0] : 1;
  const int n1 = d.nsum > 1 ? d.sum_dim[1] : 1;
  const int nz = n0 * n1;
  const int CT = (int)(d.ncol < 256 ? d.ncol : 256);
  // rows per block: fill a wave with (row, column) pairs first
  int Rw = 1;
  while (Rw * 2 * CT <= 64) Rw *= 2;
  int P = 1;
  while (P * 2 <= nz && P * 2 * Rw * CT <= 256) P *= 2;
  const int R = 256 / (CT * P);
  unsigned gx = cdiv(nrows, R);
  if (gx > 65536) gx = 65536;
  const unsigned gy = cdiv(d.ncol, CT);
  hipLaunchKernelGGL(k_couple_reduce<T>, dim3(gx, gy), dim3(256), 0, s, d, P, CT, f, X, Y);
  return hipGetLastError();
}

#define CASPT2_COUPLE_INSTANCES(T)                                                                  \
  template hipError_t unpack_all<T>(const PackInfo&, const AllDesc&, const T*, T*, hipStream_t);   \
  template hipError_t pack_acc<T>(const TermDesc&, const AllDesc&, const T*, T*, hipStream_t);     \
  template hipError_t couple_expand<T>(const CoupleDesc&, const double*, const T*, T*, hipStream_t); \
  template hipError_t couple_reduce<T>(const CoupleDesc&, const double*, const T*, T*, hipStream_t);
CASPT2_COUPLE_INSTANCES(double)
CASPT2_COUPLE_INSTANCES(float)
#undef CASPT2_COUPLE_INSTANCES

}  // namespace caspt2
