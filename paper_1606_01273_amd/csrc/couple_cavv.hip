// Coupling terms of cavv with aavv and aaav (Fock couplings of Eq. 10 with
// the f of Eq. 11), in the packed rows of cavv (+: i, a >= b; -: i, a > b)
// and aavv (+: a >= b; -: a > b) instead of the all-orderings tensors:
//   up   cavv <- aavv through f(active, closed):  sigma(i,a,b) += sum_y f(y,i)
//        [W1(a,b) + W2(b,a)](y, .),  W = X_aavv G^T (two pairings)
//   up   cavv <- aaav through f(virtual, closed): sigma(i,a,b) += f(b,i) W3(a)
//        + f(a,i) W4(b)
//   down aavv <- cavv through f(closed, active):  Y(a,b)(y,c) = sum_z f(z,y)
//        X(z,a,b)(c), sigma_aavv(a,b) += G1 Y(a,b) + G2 Y(b,a)
//   up   cavv <- caav through f(virtual, active): sigma(i,a,b) += sum_y
//        f(b,y) W5(i,a)(y, .) + f(a,y) W6(i,b)(y, .)
//   down caav <- cavv through f(active, virtual): Y(i,a)(y,c) = sum_w f(y,w)
//        X(i,w,a)(c) and sum_w f(y,w) X(i,a,w)(c)
//   down aaav <- cavv through f(closed, virtual): sum_{z,w} f(z,w) X(z,w,a)
//        and sum_{z,w} f(z,w) X(z,a,w)
// With x(i,a,b) +- x(i,b,a) = sqrt 2 x+-(i,ab) (a != b) the packed entries
// take sums and differences of the two pairings:
//   cavv +(i,ab) += f(.,i).Q+(ab) + kv [f(b,i) B+(a) + f(a,i) B+(b)]
//   cavv -(i,ab) += f(.,i).Q-(ab) + [f(b,i) B-(a) - f(a,i) B-(b)] / sqrt 2
//   aavv +-(ab)  += (G1 +- G2) Z+-(ab),  Z+-(ab)(y,c) = sum_z f(z,y) x+-(z,ab)(c)
//   cavv +(i,ab) += kv [f(b,.).C+(i,a) + f(a,.).C+(i,b)],
//   cavv -(i,ab) += [f(b,.).C-(i,a) - f(a,.).C-(i,b)] / sqrt 2
//   caav (i,a)   += [(G1 + G2) Sb(i,a) + (G1 - G2) Db(i,a)] / 2,
//        Sb = sum_w f(.,w) s_w x+(i,{w,a}),  Db = sum_w f(.,w) t_w x-(i,{w,a})
//   aaav (a)     += the same with f(z, w) and a further sum over z
// (Q+- = (G1 +- G2) x_aavv+-, B+- = (G3 +- G4) x_aaav, C+- = (G5 +- G6)
// x_caav; kv = 1/sqrt 2, or 1/2 for a = b; s_w = sqrt 2, or 2 for w = a;
// t_w = sqrt 2 sign(w - a)).  The products with G run as GEMMs in the packed
// spaces; one pass over virtual pairs adds the cavv rows and forms Z, one
// pass over closed indices forms Sb, Db and the per-index parts of the aaav
// sums.
#include <algorithm>
#include <cmath>

#include "device_common.hpp"
#include "kernels.hpp"

namespace caspt2 {

namespace {

constexpr int CV_NB = VPAIR_GROUP;   // virtual pairs (a, b0 .. b0 + 2) per workgroup
constexpr int CV_THREADS = 512;
constexpr int CV_IPT = 4;

// the packed cavv sigma element of item it = (kind, i, alpha) and pair u of
// the group (a, b0 + u), or NULL (no such pair, or the - entry of a = b)
template <typename T>
__device__ inline T* cavv_out(T* sp, T* sm, int it, int u, int nb, int nc, int nak, int a, int b0, int64_t npv,
                              int64_t nmv) {
  const int al = it % nak, i = (it / nak) % nc, kind = it / (nak * nc);
  if (u >= nb || (kind == 1 && (a == b0 + u || !sm))) return nullptr;
  return kind == 0 ? sp + ((int64_t)i * npv + (int64_t)a * (a + 1) / 2 + b0 + u) * nak + al
                   : sm + ((int64_t)i * nmv + (int64_t)a * (a - 1) / 2 + b0 + u) * nak + al;
}          // (kind, i, alpha) items per thread whose old values are loaded first

}  // namespace

// Workgroup g: virtual index a and b_u = b0 + u (u < nb, b_u <= a) from
// groups[g] = a << 16 | b0 (the table of the ccvv passes).  Shared memory
// (doubles): Qs [nb][2][nq] (Q+ and Q- of each pair, nq = ny * nak), Xs
// [nb][2][nc][nak] (x+ and x- of cavv for every closed z), Bs [1 + nb][2][nak]
// (B+ and B- of v = a, b_0 ..), fac [ny][nc] (f(y, i)), fvc [1 + nb][nc]
// (f(v, i)), fca [nc][ny] (f(z, y)).
template <typename T>
__global__ __launch_bounds__(CV_THREADS, 4) void k_cavv_vpair(CavvArgs<T> p, const uint32_t* __restrict__ groups) {
  extern __shared__ double sm[];
  const int nc = p.nc, nv = p.nv, nak = p.nak, ny = p.ny, nq = p.ny * p.nak;
  const int t = threadIdx.x;
  const uint32_t gv = groups[blockIdx.x];
  const int a = (int)(gv >> 16), b0 = (int)(gv & 0xffffu);
  const int nb = min(CV_NB, a + 1 - b0);
  const int64_t npv = (int64_t)nv * (nv + 1) / 2, nmv = (int64_t)nv * (nv - 1) / 2;
  const bool haveq = p.Qp != nullptr, haveb = p.Bp != nullptr, havez = p.Zp != nullptr, havec = p.Cp != nullptr;
  const bool up = haveq || haveb || havec;
  double* Qs = sm;                                          // [nb][2][nq]
  double* Xs = Qs + (haveq ? CV_NB * 2 * nq : 0);           // [nb][2][nc][nak]
  double* Bs = Xs + (havez ? CV_NB * 2 * nc * nak : 0);     // [1 + nb][2][nak]
  double* fac = Bs + (haveb ? (1 + CV_NB) * 2 * nak : 0);   // [ny][nc]
  double* fvc = fac + (haveq ? ny * nc : 0);                // [1 + nb][nc]
  double* fca = fvc + (haveb ? (1 + CV_NB) * nc : 0);       // [nc][ny]
  double* fva = fca + (havez ? nc * ny : 0);                // [1 + nb][ny]: f(v, y)
  auto vidx = [&](int v) { return v == 0 ? a : b0 + v - 1; };
  auto pab = [&](int u) { return (int64_t)a * (a + 1) / 2 + b0 + u; };
  auto mab = [&](int u) { return (int64_t)a * (a - 1) / 2 + b0 + u; };
  // cavv outputs: a thread takes (kind, i, alpha) (kind 0: +, 1: -) for the
  // nb pairs of the group, so the caav product row of (i, a) is read once;
  // at most CV_IPT items per thread (checked on the host)
  const int nit = up ? 2 * nc * nak : 0;
  T* const spl = p.sp;
  T* const smi = p.sm;
  double old[CV_IPT][CV_NB];
#pragma unroll
  for (int m = 0; m < CV_IPT; ++m) {
    const int it = t + m * (int)blockDim.x;
#pragma unroll
    for (int u = 0; u < CV_NB; ++u) {
      old[m][u] = 0.0;
      if (it < nit) {
        const T* q = cavv_out(spl, smi, it, u, nb, nc, nak, a, b0, npv, nmv);
        if (q) old[m][u] = (double)*q;
      }
    }
  }
  if (haveq) {
    for (int e = t; e < nb * 2 * nq; e += blockDim.x) {
      const int k = e % nq, kind = (e / nq) & 1, u = e / (2 * nq);
      double v = 0.0;
      if (kind == 0) v = (double)p.Qp[pab(u) * nq + k];
      else if (a != b0 + u && p.Qm) v = (double)p.Qm[mab(u) * nq + k];
      Qs[e] = v;
    }
    for (int e = t; e < ny * nc; e += blockDim.x) fac[e] = p.fAC[(int64_t)(e / nc) * p.fAC_stride + e % nc];
  }
  if (havez) {
    for (int e = t; e < nb * 2 * nc * nak; e += blockDim.x) {
      const int c = e % nak, z = (e / nak) % nc, kind = (e / (nak * nc)) & 1, u = e / (2 * nak * nc);
      double v = 0.0;
      if (kind == 0) v = (double)p.xp[((int64_t)z * npv + pab(u)) * nak + c];
      else if (a != b0 + u && p.xm) v = (double)p.xm[((int64_t)z * nmv + mab(u)) * nak + c];
      Xs[e] = v;
    }
    for (int e = t; e < nc * ny; e += blockDim.x) fca[e] = p.fCA[(int64_t)(e / ny) * p.fCA_stride + e % ny];
  }
  if (haveb) {
    for (int e = t; e < (1 + nb) * 2 * nak; e += blockDim.x) {
      const int c = e % nak, kind = (e / nak) & 1, v = e / (2 * nak);
      const T* B = kind == 0 ? p.Bp : p.Bm;
      Bs[e] = B ? (double)B[(int64_t)vidx(v) * nak + c] : 0.0;
    }
    for (int e = t; e < (1 + nb) * nc; e += blockDim.x)
      fvc[e] = p.fVC[(int64_t)vidx(e / nc) * p.fVC_stride + e % nc];
  }
  if (havec)
    for (int e = t; e < (1 + nb) * ny; e += blockDim.x) fva[e] = p.fVA[(int64_t)vidx(e / ny) * p.fVA_stride + e % ny];
  __syncthreads();
  // cavv rows: the additions to the nb outputs of each (kind, i, alpha)
#pragma unroll
  for (int m = 0; m < CV_IPT; ++m) {
    const int it = t + m * (int)blockDim.x;
    if (it >= nit) continue;
    const int al = it % nak, i = (it / nak) % nc, kind = it / (nak * nc);
    double ca[8] = {0, 0, 0, 0, 0, 0, 0, 0};
    if (havec) {
      const T* C = (kind == 0 ? p.Cp : p.Cm) + ((int64_t)i * nv + a) * nq + al;
#pragma unroll
      for (int y = 0; y < 8; ++y)
        if (y < ny) ca[y] = (double)C[y * nak];
    }
#pragma unroll
    for (int u = 0; u < CV_NB; ++u) {
      T* q = cavv_out(spl, smi, it, u, nb, nc, nak, a, b0, npv, nmv);
      if (!q) continue;
      const double kv = kind == 0 ? (a != b0 + u ? 0.70710678118654752440 : 0.5) : 0.70710678118654752440;
      double s = 0.0;
      if (haveq) {
        const double* qs = Qs + (u * 2 + kind) * nq + al;
        for (int y = 0; y < ny; ++y) s += fac[y * nc + i] * qs[y * nak];
      }
      if (haveb) {
        const double fbi = fvc[(1 + u) * nc + i], fai = fvc[i];
        const double ba = Bs[(0 * 2 + kind) * nak + al], bb = Bs[((1 + u) * 2 + kind) * nak + al];
        s += kv * (kind == 0 ? fbi * ba + fai * bb : fbi * ba - fai * bb);
      }
      if (havec) {
        const T* cb = (kind == 0 ? p.Cp : p.Cm) + ((int64_t)i * nv + b0 + u) * nq + al;
        const double* fa = fva;                   // f(a, y)
        const double* fb = fva + (1 + u) * ny;    // f(b, y)
        double sa = 0.0, sb = 0.0;
#pragma unroll
        for (int y = 0; y < 8; ++y) {
          if (y >= ny) break;
          sa += fb[y] * ca[y];
          sb += fa[y] * (double)cb[y * nak];
        }
        s += kv * (kind == 0 ? sa + sb : sa - sb);
      }
      *q = (T)(old[m][u] + s);
    }
  }
  // Z+- rows of the pairs: (u, kind, y, c)
  if (havez)
    for (int e = t; e < nb * 2 * nq; e += blockDim.x) {
      const int c = e % nak, y = (e / nak) % ny, kind = (e / nq) & 1, u = e / (2 * nq);
      if (kind == 1 && (a == b0 + u || !p.Zm)) continue;
      const double* xz = Xs + (int64_t)(u * 2 + kind) * nc * nak + c;
      double s = 0.0;
      for (int z = 0; z < nc; ++z) s += fca[z * ny + y] * xz[z * nak];
      if (kind == 0) p.Zp[pab(u) * nq + y * nak + c] = (T)s;
      else p.Zm[mab(u) * nq + y * nak + c] = (T)s;
    }
}

// Down terms out of cavv into caav and aaav.  A workgroup takes closed index
// i and CVC_A virtual indices a; thread (a, c) runs the sum over w from its
// own loads of the packed cavv x at (i, {w, a}), eight w at a time, with the
// Fock values at addresses uniform over the workgroup (scalar loads).
constexpr int CVC_A = 8;
template <typename T>
__global__ __launch_bounds__(256) void k_cavv_cpair(CavvArgs<T> p) {
  const int nc = p.nc, nv = p.nv, nak = p.nak, ny = p.ny, nq = p.ny * p.nak;
  const int i = blockIdx.y, a0 = blockIdx.x * CVC_A;
  const int al = threadIdx.x / nak, c = threadIdx.x % nak;
  if (al >= CVC_A || a0 + al >= nv) return;
  const int a = a0 + al;
  const int64_t npv = (int64_t)nv * (nv + 1) / 2, nmv = (int64_t)nv * (nv - 1) / 2;
  const bool haveb = p.Sb != nullptr, havec = p.Scd != nullptr;
  const double* __restrict__ fAV = p.fAV;
  const double* __restrict__ fCV = p.fCV;
  double sb[8] = {0, 0, 0, 0, 0, 0, 0, 0}, db[8] = {0, 0, 0, 0, 0, 0, 0, 0}, sc = 0.0, dc = 0.0;
  for (int w0 = 0; w0 < nv; w0 += 8) {
    double xs[8], xd[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      xs[u] = xd[u] = 0.0;
      const int w = w0 + u;
      if (w >= nv) continue;
      const int hi = max(w, a), lo = min(w, a);
      const double xp = (double)p.xp[((int64_t)i * npv + (int64_t)hi * (hi + 1) / 2 + lo) * nak + c];
      xs[u] = (w != a ? 1.41421356237309504880 : 2.0) * xp;
      if (w != a && p.xm) {
        const double xm = (double)p.xm[((int64_t)i * nmv + (int64_t)hi * (hi - 1) / 2 + lo) * nak + c];
        xd[u] = (w > a ? 1.41421356237309504880 : -1.41421356237309504880) * xm;
      }
    }
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      const int w = w0 + u;
      if (w >= nv) break;
      if (haveb) {
#pragma unroll
        for (int y = 0; y < 8; ++y) {
          if (y >= ny) break;
          const double f = fAV[(int64_t)y * p.fAV_stride + w];
          sb[y] += f * xs[u];
          db[y] += f * xd[u];
        }
      }
      if (havec) {
        const double f = fCV[(int64_t)i * p.fCV_stride + w];
        sc += f * xs[u];
        dc += f * xd[u];
      }
    }
  }
  if (haveb) {
    const int64_t row = (int64_t)i * nv + a;
#pragma unroll
    for (int y = 0; y < 8; ++y) {
      if (y >= ny) break;
      p.Sb[row * nq + y * nak + c] = (T)sb[y];
      p.Db[row * nq + y * nak + c] = (T)db[y];
    }
  }
  if (havec) {
    const int64_t per = (int64_t)nc * nv * nak;
    p.Scd[((int64_t)i * nv + a) * nak + c] = (T)sc;
    p.Scd[per + ((int64_t)i * nv + a) * nak + c] = (T)dc;
  }
}

int64_t cavv_vpair_shared(int nc, int nak, int ny, bool haveq, bool haveb, bool havez, bool havec) {
  int64_t n = havec ? (int64_t)(1 + CV_NB) * ny : 0;
  if (haveq) n += (int64_t)CV_NB * 2 * ny * nak + (int64_t)ny * nc;
  if (havez) n += (int64_t)CV_NB * 2 * nc * nak + (int64_t)nc * ny;
  if (haveb) n += (int64_t)(1 + CV_NB) * 2 * nak + (int64_t)(1 + CV_NB) * nc;
  return n * (int64_t)sizeof(double);
}

bool cavv_pass_supported(int nc, int nv, int nak, int ny) {
  if (nc <= 0 || nv <= 0 || nv > 65535 || nak <= 0 || ny < 1 || ny > 8) return false;
  if (CVC_A * nak > 256) return false;   // closed-index pass: a thread per (a, column)
  if (2 * nc * nak > CV_IPT * CV_THREADS) return false;   // virtual-pair pass: items per thread
  int dev = 0, lds_max = 0;
  if (hipGetDevice(&dev) != hipSuccess ||
      hipDeviceGetAttribute(&lds_max, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) != hipSuccess)
    return false;
  return cavv_vpair_shared(nc, nak, ny, true, true, true, true) <= lds_max;
}

// out[k][r] = sum_i in[k][i][r] (k = 0, 1; i < n)
template <typename T>
__global__ __launch_bounds__(256) void k_sum_outer(int64_t n, int64_t inner, const T* __restrict__ in, T* __restrict__ out) {
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < 2 * inner; e += (int64_t)gridDim.x * blockDim.x) {
    const int64_t k = e / inner, r = e % inner;
    double s = 0.0;
    for (int64_t i = 0; i < n; ++i) s += (double)in[(k * n + i) * inner + r];
    out[e] = (T)s;
  }
}

template <typename T>
hipError_t cavv_pass_apply(const CavvArgs<T>& p, const uint32_t* groups, int64_t ngroups, hipStream_t s) {
  if (p.nc <= 0 || p.nv <= 0) return hipSuccess;
  if (!cavv_pass_supported(p.nc, p.nv, p.nak, p.ny)) return hipErrorInvalidValue;
  CavvArgs<T> q = p;
  const bool haveq = q.Qp && q.fAC, haveb = q.Bp && q.fVC, havez = q.Zp && q.xp && q.fCA;
  const bool havec = q.Cp && q.fVA, havesb = q.Sb && q.Db && q.xp && q.fAV, havesc = q.Scd && q.Sc && q.xp && q.fCV;
  if (!haveq) q.Qp = q.Qm = nullptr;
  if (!haveb) q.Bp = q.Bm = nullptr;
  if (!havez) q.Zp = q.Zm = nullptr;
  if (!havec) q.Cp = q.Cm = nullptr;
  if (!havesb) q.Sb = q.Db = nullptr;
  if (!havesc) q.Scd = q.Sc = nullptr;
  if (haveq || haveb || havez || havec) {
    const size_t shm = (size_t)cavv_vpair_shared(q.nc, q.nak, q.ny, haveq, haveb, havez, havec);
    hipLaunchKernelGGL(k_cavv_vpair<T>, dim3((unsigned)ngroups), dim3(CV_THREADS), shm, s, q, groups);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  if (havesb || havesc) {
    if (CVC_A * q.nak > 256) return hipErrorInvalidValue;
    const dim3 grid((unsigned)((q.nv + CVC_A - 1) / CVC_A), (unsigned)q.nc);
    hipLaunchKernelGGL(k_cavv_cpair<T>, grid, dim3(256), 0, s, q);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    if (havesc) {
      const int64_t inner = (int64_t)q.nv * q.nak;
      const unsigned g2 = (unsigned)std::min<int64_t>((2 * inner + 255) / 256, 65536);
      hipLaunchKernelGGL(k_sum_outer<T>, dim3(g2), dim3(256), 0, s, (int64_t)q.nc, inner, q.Scd, q.Sc);
      e = hipGetLastError();
      if (e != hipSuccess) return e;
    }
  }
  return hipSuccess;
}

template hipError_t cavv_pass_apply<double>(const CavvArgs<double>&, const uint32_t*, int64_t, hipStream_t);
template hipError_t cavv_pass_apply<float>(const CavvArgs<float>&, const uint32_t*, int64_t, hipStream_t);

}  // namespace caspt2
