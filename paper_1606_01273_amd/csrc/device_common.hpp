// Device helpers shared by the HIP kernels: decoding of packed orbit rows,
// gathering all-orderings values from packed rows, all-orderings indexing.
#pragma once
#include <hip/hip_runtime.h>

#include <cmath>

#include "kernels.hpp"

namespace caspt2 {

__device__ inline void decode_orbit(const TermDesc& d, int64_t row, int e[4]) {
  // units from the last slot backwards; a swap pair (k, k+1) is one unit
  int k = d.nslot - 1;
  int64_t rem = row;
  while (k >= 0) {
    int sw = -1;
    for (int s = 0; s < d.nswap; ++s)
      if (d.swap_l[s] == k && d.swap_k[s] == k - 1) sw = s;
    if (sw >= 0) {
      const int64_t dim = d.slot_dim[k];
      const int64_t cnt = d.strict[sw] ? dim * (dim - 1) / 2 : dim * (dim + 1) / 2;
      const int64_t p = rem % cnt;
      rem /= cnt;
      int64_t hi;
      if (d.strict[sw]) {
        hi = (int64_t)floor((sqrt(8.0 * (double)p + 1.0) + 1.0) * 0.5);
        while (hi * (hi - 1) / 2 > p) --hi;
        while ((hi + 1) * hi / 2 <= p) ++hi;
        e[k - 1] = (int)hi;
        e[k] = (int)(p - hi * (hi - 1) / 2);
      } else {
        hi = (int64_t)floor((sqrt(8.0 * (double)p + 1.0) - 1.0) * 0.5);
        while (hi * (hi + 1) / 2 > p) --hi;
        while ((hi + 1) * (hi + 2) / 2 <= p) ++hi;
        e[k - 1] = (int)hi;
        e[k] = (int)(p - hi * (hi + 1) / 2);
      }
      k -= 2;
    } else {
      const int64_t dim = d.slot_dim[k];
      e[k] = (int)(rem % dim);
      rem /= dim;
      k -= 1;
    }
  }
}

__device__ inline int64_t pair_rank(int hi, int lo, bool strict) {
  return strict ? (int64_t)hi * (hi - 1) / 2 + lo : (int64_t)hi * (hi + 1) / 2 + lo;
}

// value of the all-orderings amplitude x[e][col] from the packed rows:
// x[e] = sum_chi chi(pi_e) t_chi[orbit(e)] / sqrt(|orbit|)
template <typename T>
__device__ inline double gather_all(const PackInfo& p, const T* __restrict__ base, const int e[4],
                             int64_t col) {
  int c[4] = {e[0], e[1], e[2], e[3]};
  int swapped[2] = {0, 0}, equal[2] = {0, 0}, ndist = 0;
  for (int s = 0; s < p.nswap; ++s) {
    const int k = p.swap_k[s], l = p.swap_l[s];
    if (c[k] < c[l]) {
      const int t = c[k];
      c[k] = c[l];
      c[l] = t;
      swapped[s] = 1;
    }
    if (c[k] == c[l]) equal[s] = 1;
    else ++ndist;
  }
  const double w = 1.0 / sqrt((double)(1 << ndist));
  double acc = 0.0;
  for (int ent = 0; ent < p.nent; ++ent) {
    bool ok = true;
    double sg = 1.0;
    for (int s = 0; s < p.nswap; ++s) {
      if (equal[s] && p.chi[ent][s] < 0) ok = false;
      if (swapped[s]) sg *= p.chi[ent][s];
    }
    if (!ok) continue;
    int64_t row = 0;
    for (int k = 0; k < p.nslot; ++k) {
      int sw = -1;
      for (int s = 0; s < p.nswap; ++s)
        if (p.swap_k[s] == k) sw = s;
      const int64_t d = p.slot_dim[k];
      if (sw >= 0) {
        const bool strict = p.chi[ent][sw] < 0;
        const int64_t cnt = strict ? d * (d - 1) / 2 : d * (d + 1) / 2;
        row = row * cnt + pair_rank(c[k], c[k + 1], strict);
        ++k;
      } else {
        row = row * d + c[k];
      }
    }
    acc += sg * (double)base[p.offset[ent] + row * p.rowlen + col];
  }
  return w * acc;
}

__device__ inline int src_value(int src, const int e[4], const int z[2], int y) {
  return src >= 0 ? e[src] : (src == -10 ? y : z[-1 - src]);
}

__device__ inline void decode_all(const AllDesc& a, int64_t row, int e[4]) {
  for (int k = a.nslot - 1; k >= 0; --k) {
    e[k] = (int)(row % a.slot_dim[k]);
    row /= a.slot_dim[k];
  }
}

__device__ inline int64_t encode_all(const AllDesc& a, const int e[4]) {
  int64_t row = 0;
  for (int k = 0; k < a.nslot; ++k) row = row * a.slot_dim[k] + e[k];
  return row;
}


}  // namespace caspt2
