// Device helpers shared by the HIP kernels: decoding of packed orbit rows,
// gathering all-orderings values from packed rows, all-orderings indexing.
//
// Every loop over the (at most four) external slots has a fixed trip count
// and is unrolled, and slot positions are compile-time constants after
// unrolling, so the slot values live in registers: a per-thread array indexed
// with a run-time value would be placed in scratch memory.  Swap pairs are
// always adjacent slots (k, k + 1).  Row indices fit in 32 bits (checked by
// the host), which keeps the index divisions in 32-bit arithmetic.
#pragma once
#include <hip/hip_runtime.h>

#include <cmath>

#include "kernels.hpp"

namespace caspt2 {

// value of slot `src` of (e0..e3), of a summed label (-1 - s) or of the
// operator's active label y (-10), by selection (no indexed array)
__device__ inline int src_pick(int src, const int e[4], const int z[2], int y) {
  int v = y;
  v = src == 0 ? e[0] : v;
  v = src == 1 ? e[1] : v;
  v = src == 2 ? e[2] : v;
  v = src == 3 ? e[3] : v;
  v = src == -1 ? z[0] : v;
  v = src == -2 ? z[1] : v;
  return v;
}
__device__ inline int src_value(int src, const int e[4], const int z[2], int y) {
  return src_pick(src, e, z, y);
}

// is slot k the first slot of a swap pair of d (returns the swap or -1)
template <typename D>
__device__ inline int swap_at(const D& d, int k) {
  int s = -1;
  if (d.nswap > 0 && d.swap_k[0] == k) s = 0;
  if (d.nswap > 1 && d.swap_k[1] == k) s = 1;
  return s;
}

__device__ inline void pair_from_rank(uint32_t p, bool strict, int& hi, int& lo) {
  int64_t h;
  if (strict) {
    h = (int64_t)floor((sqrt(8.0 * (double)p + 1.0) + 1.0) * 0.5);
    while (h * (h - 1) / 2 > (int64_t)p) --h;
    while ((h + 1) * h / 2 <= (int64_t)p) ++h;
    hi = (int)h;
    lo = (int)((int64_t)p - h * (h - 1) / 2);
  } else {
    h = (int64_t)floor((sqrt(8.0 * (double)p + 1.0) - 1.0) * 0.5);
    while (h * (h + 1) / 2 > (int64_t)p) --h;
    while ((h + 1) * (h + 2) / 2 <= (int64_t)p) ++h;
    hi = (int)h;
    lo = (int)((int64_t)p - h * (h + 1) / 2);
  }
}

// orbit representative of packed row `row` of entry d: units from the last
// slot backwards; a swap pair (k, k + 1) is one unit of rank pair_rank
__device__ inline void decode_orbit(const TermDesc& d, int64_t row, int e[4]) {
  uint32_t rem = (uint32_t)row;
  e[0] = e[1] = e[2] = e[3] = 0;
  bool second = false;   // slot k is the second slot of a pair (already set)
#pragma unroll
  for (int k = 3; k >= 0; --k) {
    if (k >= d.nslot) continue;
    if (second) {
      second = false;
      continue;
    }
    // slot k closes a pair when slot k - 1 opens one
    const int sw = k >= 1 ? swap_at(d, k - 1) : -1;
    const uint32_t dim = (uint32_t)d.slot_dim[k];
    if (sw >= 0) {
      const bool strict = d.strict[sw] != 0;
      const uint32_t cnt = strict ? dim * (dim - 1) / 2 : dim * (dim + 1) / 2;
      const uint32_t p = rem % cnt;
      rem /= cnt;
      int hi, lo;
      pair_from_rank(p, strict, hi, lo);
      if (k >= 1) e[k - 1] = hi;
      e[k] = lo;
      second = true;   // skip slot k - 1
    } else {
      e[k] = (int)(rem % dim);
      rem /= dim;
    }
  }
}

__device__ inline int64_t pair_rank(int hi, int lo, bool strict) {
  return strict ? (int64_t)hi * (hi - 1) / 2 + lo : (int64_t)hi * (hi + 1) / 2 + lo;
}

// packed rows holding the all-orderings row e: for each character entry
// present, the offset of its row (from base, in elements) and the sign
// chi(pi_e) times the packing weight 1 / sqrt(|orbit|); sg = 0 marks an
// entry that has no row for e (a strict character on equal slot values)
__device__ inline void gather_rows(const PackInfo& p, const int e[4], int64_t off[2], double sg[2]) {
  int c[4] = {e[0], e[1], e[2], e[3]};
  int swapped[2] = {0, 0}, equal[2] = {0, 0}, ndist = 0;
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    const int s = swap_at(p, k);
    if (s >= 0) {
      const bool sw = c[k] < c[k + 1];
      const int hi = sw ? c[k + 1] : c[k], lo = sw ? c[k] : c[k + 1];
      c[k] = hi;
      c[k + 1] = lo;
      const int eq = hi == lo ? 1 : 0;
      if (s == 0) {
        swapped[0] = sw;
        equal[0] = eq;
      } else {
        swapped[1] = sw;
        equal[1] = eq;
      }
      ndist += 1 - eq;
    }
  }
  const double w = ndist == 0 ? 1.0 : (ndist == 1 ? 0.70710678118654752440 : 0.5);
#pragma unroll
  for (int ent = 0; ent < 2; ++ent) {
    off[ent] = 0;
    sg[ent] = 0.0;
    if (ent >= p.nent) continue;
    bool ok = true;
    double sgn = w;
#pragma unroll
    for (int s = 0; s < 2; ++s) {
      if (s >= p.nswap) continue;
      if (equal[s] && p.chi[ent][s] < 0) ok = false;
      if (swapped[s]) sgn *= p.chi[ent][s];
    }
    if (!ok) continue;
    int64_t row = 0;
    bool second = false;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      if (k >= p.nslot) continue;
      if (second) {
        second = false;
        continue;
      }
      const int s = k < 3 ? swap_at(p, k) : -1;
      const int64_t d = p.slot_dim[k];
      if (s >= 0) {
        const bool strict = p.chi[ent][s] < 0;
        const int64_t cnt = strict ? d * (d - 1) / 2 : d * (d + 1) / 2;
        row = row * cnt + pair_rank(c[k], c[k + 1], strict);
        second = true;
      } else {
        row = row * d + c[k];
      }
    }
    off[ent] = p.offset[ent] + row * p.rowlen;
    sg[ent] = sgn;
  }
}

// value of the all-orderings amplitude x[e][col] from the packed rows:
// x[e] = sum_chi chi(pi_e) t_chi[orbit(e)] / sqrt(|orbit|)
template <typename T>
__device__ inline double gather_all(const PackInfo& p, const T* __restrict__ base, const int e[4],
                                    int64_t col) {
  // canonical order of each swap pair and its flags
  int c[4] = {e[0], e[1], e[2], e[3]};
  int swapped[2] = {0, 0}, equal[2] = {0, 0}, ndist = 0;
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    const int s = swap_at(p, k);
    if (s >= 0) {
      const bool sw = c[k] < c[k + 1];
      const int hi = sw ? c[k + 1] : c[k], lo = sw ? c[k] : c[k + 1];
      c[k] = hi;
      c[k + 1] = lo;
      const int eq = hi == lo ? 1 : 0;
      if (s == 0) {
        swapped[0] = sw;
        equal[0] = eq;
      } else {
        swapped[1] = sw;
        equal[1] = eq;
      }
      ndist += 1 - eq;
    }
  }
  const double w = ndist == 0 ? 1.0 : (ndist == 1 ? 0.70710678118654752440 : 0.5);
  double acc = 0.0;
#pragma unroll
  for (int ent = 0; ent < 2; ++ent) {
    if (ent >= p.nent) continue;
    bool ok = true;
    double sg = 1.0;
#pragma unroll
    for (int s = 0; s < 2; ++s) {
      if (s >= p.nswap) continue;
      if (equal[s] && p.chi[ent][s] < 0) ok = false;
      if (swapped[s]) sg *= p.chi[ent][s];
    }
    if (!ok) continue;
    int64_t row = 0;
    bool second = false;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      if (k >= p.nslot) continue;
      if (second) {
        second = false;
        continue;
      }
      const int s = k < 3 ? swap_at(p, k) : -1;
      const int64_t d = p.slot_dim[k];
      if (s >= 0) {
        const bool strict = p.chi[ent][s] < 0;
        const int64_t cnt = strict ? d * (d - 1) / 2 : d * (d + 1) / 2;
        row = row * cnt + pair_rank(c[k], c[k + 1], strict);
        second = true;
      } else {
        row = row * d + c[k];
      }
    }
    acc += sg * (double)base[p.offset[ent] + row * p.rowlen + col];
  }
  return w * acc;
}

__device__ inline void decode_all(const AllDesc& a, int64_t row, int e[4]) {
  uint32_t q = (uint32_t)row;
  e[0] = e[1] = e[2] = e[3] = 0;
#pragma unroll
  for (int k = 3; k >= 0; --k) {
    if (k >= a.nslot) continue;
    const uint32_t dim = (uint32_t)a.slot_dim[k];
    e[k] = (int)(q % dim);
    q /= dim;
  }
}

__device__ inline int64_t encode_all(const AllDesc& a, const int e[4]) {
  int64_t row = 0;
#pragma unroll
  for (int k = 0; k < 4; ++k)
    if (k < a.nslot) row = row * a.slot_dim[k] + e[k];
  return row;
}

// e[swap pair of swap s] exchanged (the pair is adjacent: (swap_k, swap_k + 1))
template <typename D>
__device__ inline void swap_pair(const D& d, int s, int e[4]) {
  const int k = d.swap_k[s];
  int t;
  if (k == 0) { t = e[0]; e[0] = e[1]; e[1] = t; }
  if (k == 1) { t = e[1]; e[1] = e[2]; e[2] = t; }
  if (k == 2) { t = e[2]; e[2] = e[3]; e[3] = t; }
}

// first and second slot value of swap s
template <typename D>
__device__ inline void pair_values(const D& d, int s, const int e[4], int& a, int& b) {
  const int k = d.swap_k[s];
  a = k == 0 ? e[0] : (k == 1 ? e[1] : e[2]);
  b = k == 0 ? e[1] : (k == 1 ? e[2] : e[3]);
}

}  // namespace caspt2
