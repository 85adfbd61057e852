// Grouped PCG vector kernels: one launch advances every linear system of a
// solve (all states of one problem, or all systems of a batch of problems)
// by one step of the preconditioned conjugate-gradient recurrence, with the
// scalars (rz, p.Ap, alpha, beta, |r|^2) kept on the device so that a whole
// iteration runs without host synchronisation.
//
// Work decomposition: the host builds a block table (one entry per chunk of
// CHUNK elements of one system's vectors); the partial sums of a system's
// blocks are contiguous and are reduced in a fixed order by the per-system
// kernels (deterministic results).
#include "kernels.hpp"

namespace caspt2 {

namespace {

__device__ inline double block_sum(double v, double* sh) {
  sh[threadIdx.x] = v;
  __syncthreads();
  for (int w = PCG_THREADS / 2; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) sh[threadIdx.x] += sh[threadIdx.x + w];
    __syncthreads();
  }
  return sh[0];
}

// partial[b] = sum over the block's chunk of x . y
template <typename T>
__global__ __launch_bounds__(PCG_THREADS) void k_seg_dot(PcgTable tab, const PcgVecs<T>* __restrict__ v,
                                                         int which_x, int which_y,
                                                         double* __restrict__ partial) {
  __shared__ double sh[PCG_THREADS];
  const int b = blockIdx.x;
  const int s = tab.blk_sys[b];
  const T* x = v[s].vec[which_x];
  const T* y = v[s].vec[which_y];
  double acc = 0.0;
  for (int64_t i = tab.blk_start[b] + threadIdx.x; i < tab.blk_end[b]; i += PCG_THREADS)
    acc += (double)x[i] * (double)y[i];
  const double tot = block_sum(acc, sh);
  if (threadIdx.x == 0) partial[b] = tot;
}

// z = r / D, p = z; partials of r.r and r.z   (start of a (re)started solve)
template <typename T>
__global__ __launch_bounds__(PCG_THREADS) void k_seg_init(PcgTable tab, const PcgVecs<T>* __restrict__ v,
                                                          double* __restrict__ part_rr,
                                                          double* __restrict__ part_rz) {
  __shared__ double sh[PCG_THREADS];
  const int b = blockIdx.x;
  const int s = tab.blk_sys[b];
  const T* r = v[s].vec[PCG_R];
  const T* D = v[s].vec[PCG_D];
  T* p = v[s].vec[PCG_P];
  double arr = 0.0, arz = 0.0;
  for (int64_t i = tab.blk_start[b] + threadIdx.x; i < tab.blk_end[b]; i += PCG_THREADS) {
    const T ri = r[i];
    const T zi = ri / D[i];
    p[i] = zi;
    arr += (double)ri * (double)ri;
    arz += (double)ri * (double)zi;
  }
  const double trr = block_sum(arr, sh);
  __syncthreads();
  const double trz = block_sum(arz, sh);
  if (threadIdx.x == 0) {
    part_rr[b] = trr;
    part_rz[b] = trz;
  }
}

// t += alpha p, r -= alpha q, z = r / D (not stored); partials of r.r, r.z
template <typename T>
__global__ __launch_bounds__(PCG_THREADS) void k_seg_update(PcgTable tab, const PcgVecs<T>* __restrict__ v,
                                                            const PcgScalars* __restrict__ sc,
                                                            double* __restrict__ part_rr,
                                                            double* __restrict__ part_rz) {
  __shared__ double sh[PCG_THREADS];
  const int b = blockIdx.x;
  const int s = tab.blk_sys[b];
  const double alpha = sc[s].alpha;
  T* t = v[s].vec[PCG_T];
  T* r = v[s].vec[PCG_R];
  const T* p = v[s].vec[PCG_P];
  const T* q = v[s].vec[PCG_Q];
  const T* D = v[s].vec[PCG_D];
  double arr = 0.0, arz = 0.0;
  const bool step = alpha != 0.0;
  for (int64_t i = tab.blk_start[b] + threadIdx.x; i < tab.blk_end[b]; i += PCG_THREADS) {
    T ri = r[i];
    if (step) {
      t[i] += (T)(alpha * (double)p[i]);
      ri -= (T)(alpha * (double)q[i]);
      r[i] = ri;
    }
    const T zi = ri / D[i];
    arr += (double)ri * (double)ri;
    arz += (double)ri * (double)zi;
  }
  const double trr = block_sum(arr, sh);
  __syncthreads();
  const double trz = block_sum(arz, sh);
  if (threadIdx.x == 0) {
    part_rr[b] = trr;
    part_rz[b] = trz;
  }
}

// p = r / D + beta p  for systems still running
template <typename T>
__global__ __launch_bounds__(PCG_THREADS) void k_seg_xpay(PcgTable tab, const PcgVecs<T>* __restrict__ v,
                                                          const PcgScalars* __restrict__ sc) {
  const int b = blockIdx.x;
  const int s = tab.blk_sys[b];
  if (!sc[s].active) return;
  const double beta = sc[s].beta;
  const T* r = v[s].vec[PCG_R];
  const T* D = v[s].vec[PCG_D];
  T* p = v[s].vec[PCG_P];
  for (int64_t i = tab.blk_start[b] + threadIdx.x; i < tab.blk_end[b]; i += PCG_THREADS)
    p[i] = r[i] / D[i] + (T)(beta * (double)p[i]);
}

// per system (one workgroup each): reduce the partials of its blocks
// [b0, b1) with a fixed assignment and tree (deterministic)
__device__ inline double sys_sum(const double* part, int b0, int b1, double* sh) {
  double acc = 0.0;
  for (int b = b0 + (int)threadIdx.x; b < b1; b += PCG_THREADS) acc += part[b];
  return block_sum(acc, sh);
}

__global__ __launch_bounds__(PCG_THREADS) void k_sys_init(const int* __restrict__ sys_id,
                                                          const int* __restrict__ b0,
                                                          const int* __restrict__ b1,
                                                          const double* __restrict__ part_rr,
                                                          const double* __restrict__ part_rz,
                                                          PcgScalars* __restrict__ sc) {
  __shared__ double sh[PCG_THREADS];
  const int k = blockIdx.x;
  const double rr = sys_sum(part_rr, b0[k], b1[k], sh);
  __syncthreads();
  const double rz = sys_sum(part_rz, b0[k], b1[k], sh);
  if (threadIdx.x != 0) return;
  PcgScalars& c = sc[sys_id[k]];
  c.rr = rr;
  c.rz = rz;
  c.alpha = 0.0;
  c.beta = 0.0;
  c.status = PCG_RUNNING;
  c.active = 1;
  if (rr <= c.tol2) {
    c.status = PCG_CONVERGED;
    c.active = 0;
  }
}

__global__ __launch_bounds__(PCG_THREADS) void k_sys_alpha(const int* __restrict__ sys_id,
                                                           const int* __restrict__ b0,
                                                           const int* __restrict__ b1,
                                                           const double* __restrict__ part,
                                                           PcgScalars* __restrict__ sc) {
  __shared__ double sh[PCG_THREADS];
  const int k = blockIdx.x;
  const double pAp = sys_sum(part, b0[k], b1[k], sh);
  if (threadIdx.x != 0) return;
  PcgScalars& c = sc[sys_id[k]];
  if (!c.active) {
    c.alpha = 0.0;
    return;
  }
  c.pap = pAp;
  if (!(pAp > 0.0)) {
    c.status = PCG_INDEFINITE;
    c.active = 0;
    c.alpha = 0.0;
    return;
  }
  c.alpha = c.rz / pAp;
}

__global__ __launch_bounds__(PCG_THREADS) void k_sys_beta(const int* __restrict__ sys_id,
                                                          const int* __restrict__ b0,
                                                          const int* __restrict__ b1,
                                                          const double* __restrict__ part_rr,
                                                          const double* __restrict__ part_rz,
                                                          PcgScalars* __restrict__ sc) {
  __shared__ double sh[PCG_THREADS];
  const int k = blockIdx.x;
  const double rr = sys_sum(part_rr, b0[k], b1[k], sh);
  __syncthreads();
  const double rz = sys_sum(part_rz, b0[k], b1[k], sh);
  if (threadIdx.x != 0) return;
  PcgScalars& c = sc[sys_id[k]];
  if (!c.active) return;
  c.rr = rr;
  c.iters += 1;
  if (rr <= c.tol2) {
    c.status = PCG_CONVERGED;
    c.active = 0;
    c.beta = 0.0;
    return;
  }
  if (c.iters >= c.maxiter) {
    c.status = PCG_MAXITER;
    c.active = 0;
    c.beta = 0.0;
    return;
  }
  c.beta = rz / c.rz;
  c.rz = rz;
}

}  // namespace

template <typename T>
hipError_t pcg_init(const PcgTable& tab, const PcgSysTable& st, const PcgVecs<T>* v, PcgScalars* sc,
                    double* part_rr, double* part_rz, hipStream_t s) {
  if (tab.nblk <= 0 || st.nsys <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_seg_init<T>, dim3(tab.nblk), dim3(PCG_THREADS), 0, s, tab, v, part_rr, part_rz);
  hipLaunchKernelGGL(k_sys_init, dim3(st.nsys), dim3(PCG_THREADS), 0, s, st.sys_id, st.b0, st.b1,
                     part_rr, part_rz, sc);
  return hipGetLastError();
}

template <typename T>
hipError_t pcg_step(const PcgTable& tab, const PcgSysTable& st, const PcgVecs<T>* v, PcgScalars* sc,
                    double* part_a, double* part_b, hipStream_t s) {
  if (tab.nblk <= 0 || st.nsys <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_seg_dot<T>, dim3(tab.nblk), dim3(PCG_THREADS), 0, s, tab, v, (int)PCG_P,
                     (int)PCG_Q, part_a);
  hipLaunchKernelGGL(k_sys_alpha, dim3(st.nsys), dim3(PCG_THREADS), 0, s, st.sys_id, st.b0, st.b1,
                     part_a, sc);
  hipLaunchKernelGGL(k_seg_update<T>, dim3(tab.nblk), dim3(PCG_THREADS), 0, s, tab, v,
                     (const PcgScalars*)sc, part_a, part_b);
  hipLaunchKernelGGL(k_sys_beta, dim3(st.nsys), dim3(PCG_THREADS), 0, s, st.sys_id, st.b0, st.b1,
                     part_a, part_b, sc);
  hipLaunchKernelGGL(k_seg_xpay<T>, dim3(tab.nblk), dim3(PCG_THREADS), 0, s, tab, v,
                     (const PcgScalars*)sc);
  return hipGetLastError();
}

template hipError_t pcg_init<double>(const PcgTable&, const PcgSysTable&, const PcgVecs<double>*,
                                     PcgScalars*, double*, double*, hipStream_t);
template hipError_t pcg_init<float>(const PcgTable&, const PcgSysTable&, const PcgVecs<float>*,
                                    PcgScalars*, double*, double*, hipStream_t);
template hipError_t pcg_step<double>(const PcgTable&, const PcgSysTable&, const PcgVecs<double>*,
                                     PcgScalars*, double*, double*, hipStream_t);
template hipError_t pcg_step<float>(const PcgTable&, const PcgSysTable&, const PcgVecs<float>*,
                                    PcgScalars*, double*, double*, hipStream_t);

}  // namespace caspt2
