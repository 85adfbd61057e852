// C ABI of the (X)MS-CASPT2 hot path on MI355X: set-up (XMS rotation, DF
// integral classes, sources, metrics, orthonormal bases), the residual of
// the amplitude equation, PCG, the effective Hamiltonian and lambda.
// Every floating-point step on problem data runs in kernels.hip.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <cstdlib>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <map>
#include <memory>
#include <mutex>
#include <stdexcept>
#include <string>
#include <thread>
#include <vector>

#include "../../include/caspt2.h"
#include "engine.hpp"
#include "kernels.hpp"

using namespace caspt2;

static thread_local std::string g_last_error;

namespace {

struct DevError : std::runtime_error {
  int code;
  DevError(int c, const std::string& m) : std::runtime_error(m), code(c) {}
};

#define HIPCHECK(expr)                                                                   \
  do {                                                                                   \
    hipError_t _e = (expr);                                                              \
    if (_e != hipSuccess)                                                                \
      throw DevError(_e == hipErrorOutOfMemory ? CASPT2_E_NOMEM : CASPT2_E_DEVICE,       \
                     std::string(#expr) + ": " + hipGetErrorString(_e));                 \
  } while (0)

// Device blocks freed while a handle is being created are kept for the
// allocations that follow in the same creation instead of going back through
// hipFree, which waits for the whole device (a creation allocates and frees
// a few thousand temporaries: for the small problems of a batch that cost
// more than their kernels).  Every launch of a creation is ordered on the
// handle's one stream, so a block is reused only by work queued after the
// work that used it.  Sizes up to 4 MB are rounded to powers of two so that
// blocks of neighbouring sizes are shared, larger ones to 256 KB; a block is
// keyed by its own size, so one allocated before the creation is reused only
// for requests it covers.  The cache belongs to one creation on one thread; the creation returns its blocks at
// its end (or when it throws), after its last synchronisation.
struct BlockCache {
  std::multimap<size_t, void*> blocks;
  size_t held = 0;
  static constexpr size_t CAP = size_t(8) << 30;   // beyond this, freed blocks go back at once
  ~BlockCache() {
    for (auto& kv : blocks) (void)hipFree(kv.second);
  }
};
thread_local BlockCache* t_block_cache = nullptr;

size_t block_class(size_t bytes) {
  if (bytes <= (size_t(4) << 20)) {
    size_t c = 256;
    while (c < bytes) c <<= 1;
    return c;
  }
  const size_t g = size_t(256) << 10;
  return (bytes + g - 1) / g * g;
}

// a block of at least `bytes`; cap receives its size (the cache's key when
// it is freed: a block is reused only for requests of its exact class)
void* dev_alloc(size_t bytes, size_t& cap) {
  void* p = nullptr;
  if (BlockCache* c = t_block_cache) {
    bytes = block_class(bytes);
    auto it = c->blocks.find(bytes);
    if (it != c->blocks.end()) {
      p = it->second;
      c->blocks.erase(it);
      c->held -= bytes;
      cap = bytes;
      return p;
    }
  }
  HIPCHECK(hipMalloc(&p, bytes));
  cap = bytes;
  return p;
}

void dev_free(void* p, size_t cap) {
  if (!p) return;
  BlockCache* c = t_block_cache;
  if (c && c->held + cap <= BlockCache::CAP) {
    c->blocks.emplace(cap, p);
    c->held += cap;
    return;
  }
  (void)hipFree(p);
}

// the block cache of one creation on this thread (restores the previous one)
struct BlockCacheScope {
  BlockCache cache;
  BlockCache* prev;
  BlockCacheScope() : prev(t_block_cache) { t_block_cache = &cache; }
  ~BlockCacheScope() { t_block_cache = prev; }
  BlockCacheScope(const BlockCacheScope&) = delete;
  BlockCacheScope& operator=(const BlockCacheScope&) = delete;
};

// owning device buffer
template <typename T>
struct DevBuf {
  T* p = nullptr;
  int64_t n = 0;
  size_t cap = 0;   // bytes of the block
  DevBuf() = default;
  explicit DevBuf(int64_t n_) { alloc(n_); }
  void alloc(int64_t n_) {
    release();
    if (n_ > 0) p = static_cast<T*>(dev_alloc((size_t)n_ * sizeof(T), cap));
    n = n_;
  }
  void zero(hipStream_t s) {
    if (n > 0) HIPCHECK(hipMemsetAsync(p, 0, (size_t)n * sizeof(T), s));
  }
  void release() {
    dev_free(p, cap);
    p = nullptr;
    n = 0;
    cap = 0;
  }
  ~DevBuf() { release(); }
  DevBuf(const DevBuf&) = delete;
  DevBuf& operator=(const DevBuf&) = delete;
  DevBuf(DevBuf&& o) noexcept : p(o.p), n(o.n), cap(o.cap) {
    o.p = nullptr;
    o.n = 0;
    o.cap = 0;
  }
  DevBuf& operator=(DevBuf&& o) noexcept {
    release();
    p = o.p;
    n = o.n;
    cap = o.cap;
    o.p = nullptr;
    o.n = 0;
    o.cap = 0;
    return *this;
  }
};
using DBuf = DevBuf<double>;
using FBuf = DevBuf<float>;

// page-locked host buffer (hipHostMalloc): every device-to-host copy of
// scalars and small arrays lands here, so no asynchronous copy targets
// pageable memory
template <typename T>
struct PinBuf {
  T* p = nullptr;
  int64_t n = 0;
  void ensure(int64_t n_) {
    if (n_ <= n) return;
    release();
    HIPCHECK(hipHostMalloc((void**)&p, (size_t)n_ * sizeof(T), hipHostMallocDefault));
    n = n_;
  }
  void release() {
    if (p) (void)hipHostFree(p);
    p = nullptr;
    n = 0;
  }
  T& operator[](int64_t i) { return p[i]; }
  const T& operator[](int64_t i) const { return p[i]; }
  PinBuf() = default;
  ~PinBuf() { release(); }
  PinBuf(const PinBuf&) = delete;
  PinBuf& operator=(const PinBuf&) = delete;
};

struct IBuf {
  int32_t* p = nullptr;
  int64_t n = 0;
  size_t cap = 0;
  void alloc(int64_t n_) {
    dev_free(p, cap);
    p = nullptr;
    n = 0;
    cap = 0;
    if (n_ > 0) p = static_cast<int32_t*>(dev_alloc((size_t)n_ * sizeof(int32_t), cap));
    n = n_;
  }
  ~IBuf() { dev_free(p, cap); }
};

int64_t ipow(int64_t b, int e) {
  int64_t r = 1;
  for (int k = 0; k < e; ++k) r *= b;
  return r;
}

// one packed layout entry of one state's function set
struct Entry {
  int block;
  std::vector<int> chi;
  int64_t nrow = 0, nalpha = 0, offset = 0;
  int64_t nkeep = 0, ooff = 0;   // orthogonal-basis columns and offset
  DBuf S, F, X, mu, eps;          // S,F [nalpha^2]; X [nalpha][nkeep]; mu [nkeep]; eps [nrow]
  DBuf SX;                        // S X [nalpha][nkeep], made on the first warm start
  FBuf S32, F32, X32, eps32;      // FP32 copies for the inner solver (mixed precision)
  DBuf epsA, epsB;                // separable row energies: eps(m) = A[m / nB] + B[m % nB]
  FBuf epsA32, epsB32;
  int64_t nB = 1;
  double emin_kept = INFINITY, emax_dropped = -1.0;
  LaunchTune tune;                // FP64 launch choices (rule unless autotuned)
  double tune_rule_ms = -1.0, tune_best_ms = -1.0;   // autotuner timings (-1: not timed)
};

struct CoupleTerm {
  bool up;
  int bra, ket;          // block ids
  CoupleDesc d;          // ket_src, fx/fy, nsum, sum_dim, ny, f_stride filled
  int64_t f_off;         // offset of the Fock block origin in f
  DBuf G;                // up: [ny * nalpha_b][nalpha_k]; down: [nalpha_b][ny * nalpha_k]
  FBuf G32;              // FP32 copy (mixed precision)
  int fuse = -1;         // up terms (autotuned): -1 rule (fused where possible), 0 GEMM + ket-parallel
                         // expand, 1 fused, 2 GEMM + output-parallel expand
  int sg_slot = -1;      // down term of a block with itself that applies f along one bra slot of the
                         // ket tensor: that slot (batched MFMA GEMM in FP64), else -1
  bool sg_perm = false;  // ... read from the block's slot-permuted copy of x
  int ccvv_kind = -1;    // up term into ccvv applied by the packed-row passes (couple_ccvv.hip): its role
                         // (CcvvKind), else -1
  int ccvv_down = -1;    // down term out of ccvv into cavv or caav applied by the packed-row pass: its
                         // role (CcvvDownKind), else -1
  int cavv_role = -1;    // term between cavv and aavv/aaav applied in packed rows (couple_cavv.hip): its
                         // role (CavvRole), else -1
};

// roles of the up terms into ccvv in the packed-row passes, with the slot
// maps the host engine gives them (bra slots i, j, a, b = 0..3; the Fock
// indices as bra slots, -10 the active label)
enum CcvvKind { CK_CAVV1 = 0, CK_CAVV2, CK_CCAV1, CK_CCAV2, CK_CAAV1, CK_CAAV2, CK_N };
// roles of the down terms out of ccvv in the packed-row pass (cavv bra slots
// i, a, b; caav i, a; the ket ccvv slots from bra slots or summed labels -1, -2)
enum CcvvDownKind { DK_CAVV1 = 0, DK_CAVV2, DK_CAAV1, DK_CAAV2, DK_CCAV1, DK_CCAV2, DK_N };
// roles of the terms between cavv (slots i, a, b) and aavv (a, b), aaav (a),
// caav (i, a) applied in packed rows: up from aavv, up from aaav, down into
// aavv, up from caav, down into caav, down into aaav; two pairings each
enum CavvRole { CV_UA1 = 0, CV_UA2, CV_UB1, CV_UB2, CV_DA1, CV_DA2, CV_UC1, CV_UC2, CV_DB1, CV_DB2, CV_DC1, CV_DC2,
                CV_N };

// the G products of the cavv packed-row terms of one function set, summed
// and differenced over the two pairings of each role (FP64 and FP32 copies)
struct CavvG {
  DBuf g[6][2];     // per role pair (UA, UB, DA, UC, DB, DC): [0] G1 + G2, [1] G1 - G2; empty when absent
  FBuf g32[6][2];
};

// element-type selection of the per-entry and per-term operands
template <typename T>
struct Sel;
template <>
struct Sel<double> {
  static const double* S(const Entry& e) { return e.S.p; }
  static const double* F(const Entry& e) { return e.F.p; }
  static const double* X(const Entry& e) { return e.X.p; }
  static const double* eps(const Entry& e) { return e.eps.p; }
  static RowEnergy<double> rows(const Entry& e) { return RowEnergy<double>{e.epsA.p, e.epsB.p, (uint32_t)e.nB}; }
  static const double* G(const CoupleTerm& t) { return t.G.p; }
  static LaunchTune tune(const Entry& e) { return e.tune; }
};
template <>
struct Sel<float> {
  static const float* S(const Entry& e) { return e.S32.p; }
  static const float* F(const Entry& e) { return e.F32.p; }
  static const float* X(const Entry& e) { return e.X32.p; }
  static const float* eps(const Entry& e) { return e.eps32.p; }
  static RowEnergy<float> rows(const Entry& e) { return RowEnergy<float>{e.epsA32.p, e.epsB32.p, (uint32_t)e.nB}; }
  static const float* G(const CoupleTerm& t) { return t.G32.p; }
  static LaunchTune tune(const Entry&) { return LaunchTune{}; }
};

inline hipError_t gemm_t(bool nk, int64_t M, int64_t N, int64_t K, double alpha, const double* A,
                         int64_t lda, const double* B, int64_t ldb, double beta, double* C,
                         int64_t ldc, hipStream_t s) {
  return gemm_f64(nk, M, N, K, alpha, A, lda, 0, B, ldb, 0, beta, C, ldc, 0, 1, s);
}
inline hipError_t gemm_t(bool nk, int64_t M, int64_t N, int64_t K, double alpha, const float* A,
                         int64_t lda, const float* B, int64_t ldb, double beta, float* C,
                         int64_t ldc, hipStream_t s) {
  return gemm_f32(nk, M, N, K, (float)alpha, A, lda, 0, B, ldb, 0, (float)beta, C, ldc, 0, 1, s);
}
inline hipError_t residual_small_t(int64_t M, int64_t N, const double* X, const double* S,
                                   const double* F, const double* d, double dshift,
                                   const double* V, double* C, hipStream_t s, LaunchTune tu) {
  return residual_small_f64(M, N, X, S, F, d, dshift, V, C, s, tu);
}
inline hipError_t residual_small_t(int64_t M, int64_t N, const float* X, const float* S,
                                   const float* F, const float* d, double dshift, const float* V,
                                   float* C, hipStream_t s, LaunchTune) {
  return residual_small_f32(M, N, X, S, F, d, (float)dshift, V, C, s);
}
inline hipError_t residual_gemm_t(int64_t M, int64_t N, const double* X, const double* S,
                                  const double* F, const double* d, double dshift,
                                  const double* V, double* C, hipStream_t s, DBuf& ws, LaunchTune tu) {
  return residual_gemm_f64(M, N, N, X, N, S, F, d, dshift, V, N, C, N, s, ws.p, ws.n, tu);
}
inline hipError_t residual_gemm_t(int64_t M, int64_t N, const float* X, const float* S,
                                  const float* F, const float* d, double dshift, const float* V,
                                  float* C, hipStream_t s, DBuf&, LaunchTune) {
  return residual_gemm_f32(M, N, N, X, N, S, F, d, (float)dshift, V, N, C, N, s);
}

struct ProfEventRec {
  int entry;
  double bytes;
  hipEvent_t a, b;
};

struct Gather {
  IBuf src;
  DBuf sign;
  Sector to;
  int64_t dim_to;
};

}  // namespace

struct caspt2_handle {
  caspt2_dims d;
  hipStream_t s = nullptr;
  int nc, na, nv, nmo, nst, naux;
  Sector sec0;
  std::unique_ptr<ActiveSpace> as;
  int64_t ndet = 0;
  DBuf fock, hcore, B, ci_raw, ci;   // ci: rotated [nst][dim]
  FBuf fock32;                       // FP32 copy of fock (mixed precision)
  std::vector<double> h_fock, h_eps, U, e0, fref, href, eref;
  // layout per function set (one for MS-MR, nst for SS-SR)
  std::vector<std::vector<Entry>> sets;
  int64_t length = 0, olength = 0;
  // sources: src[set][N] packed
  std::vector<std::vector<DBuf>> src;
  // integrals
  std::map<std::string, DBuf> eri;
  // gather tables
  std::map<std::tuple<char, int, int, int>, std::unique_ptr<Gather>> gathers;
  // applied-string cache
  std::map<std::string, std::pair<DBuf, Sector>> vcache;
  DBuf red_partial, red_out;
  // solutions
  std::vector<DBuf> T, Tt, lam, lamt;  // packed and orthogonal
  std::vector<caspt2_info> tinfo, linfo;
  bool have_T = false, have_heff = false, have_lam = false;
  int lam_target = -1;                                 // target state P of the stored lambda
  std::vector<double> heff, ems, R;
  DBuf jws;
  PinBuf<double> hpin;   // staging of device-to-host copies (d2h)
  std::vector<std::vector<struct CoupleTerm>> couple;  // per function set
  DBuf cscratch;                                       // W / Y of the couplings
  DBuf wx, wsg;                                        // operator work vectors of the grouped solver
  DBuf splitk_ws;                                      // partial products of the split-K residual GEMMs
  DBuf* ws_cur = nullptr;                              // split-K workspace of the current stream (null: splitk_ws)
  // second work set (all-orderings tensors, coupling scratch, operator work
  // vectors), so that two streams can apply the operator with couplings of
  // two states at once; wset selects the set the launches use
  DBuf xall2[NBLOCK], sall2[NBLOCK], cscratch2, wx2, wsg2;
  int wset = 0;
  // caspt2_residual_all without couplings: states on two streams of default
  // priority, their join events and the second stream's split-K workspace
  hipStream_t slane[2] = {nullptr, nullptr};
  hipEvent_t slane_done[2] = {nullptr, nullptr};
  hipEvent_t sfork = nullptr;
  DBuf splitk_ws2;
  int residual_streams = 2;                            // 1: caspt2_residual_all on the handle's stream only
  DBuf xall[NBLOCK], sall[NBLOCK];                      // all-orderings x and sigma per block
  DBuf xperm[NBLOCK], xperm2[NBLOCK];                   // slot-permuted all-orderings x (both work sets)
  int xperm_p[NBLOCK][4] = {};                          // its slot map: copy[e] = x[e[p[0]], e[p[1]], ..]
  bool direct[NBLOCK] = {};                            // ket read from packed rows (no all-orderings x)
  std::vector<char> ccvv_fused;                        // per set: up terms into ccvv run as packed-row passes
  IBuf ccvv_groups;                                    // workgroup table of the virtual-pair pass
  IBuf cavv_groups;                                    // the same groups, b-major in per-XCD runs
  int64_t ccvv_ngroups = 0;
  int64_t ccvv_woff[CK_N] = {};                        // offsets of the W products in ccvv_w (-1: absent)
  DBuf ccvv_w, ccvv_w2;                                // W products of the ccav and caav terms (both work sets)
  std::vector<char> ccvv_down_fused;                   // per set: down terms out of ccvv into cavv, caav as a pass
  std::vector<char> cavv_fused;                        // per set: cavv - aavv/aaav terms in packed rows
  std::vector<CavvG> cavv_g;                           // per set: their summed and differenced G
  DBuf cavv_w, cavv_w2;                                // Q+-, B+-, Z+- of the cavv pass (both work sets)
  int64_t cavv_off[12] = {};                           // offsets in cavv_w: Q+, Q-, B+, B-, Z+, Z-, C+, C-, Sb, Db,
                                                       // Scd, Sc
  DBuf ccvv_t, ccvv_t2, ccvv_y, ccvv_y2;               // caav partial sums and reductions (both work sets)
  bool have_mixed = false;                             // FP32 operand copies made
  bool prof_on = false;
  bool verbose = false;
  int verbose_level = 0;
  double t_start = 0.0;
  std::vector<ProfEventRec> prof_events;
  std::vector<std::string> prof_stage;                 // names of the coupling stages timed (entries 1000 + k)
};

namespace {

using H = caspt2_handle;

const Gather& gather(H& h, char kind, int spin, Sector from) {
  auto key = std::make_tuple(kind, spin, from.na_el, from.nb_el);
  auto it = h.gathers.find(key);
  if (it != h.gathers.end()) return *it->second;
  auto g = std::make_unique<Gather>();
  std::vector<int32_t> src;
  std::vector<double> sign;
  h.as->gather_table(kind, spin, from, src, sign);
  g->to = h.as->target(kind, spin, from);
  g->dim_to = h.as->valid(g->to) ? h.as->dim(g->to) : 0;
  g->src.alloc((int64_t)src.size());
  g->sign.alloc((int64_t)sign.size());
  if (!src.empty()) {
    HIPCHECK(hipMemcpyAsync(g->src.p, src.data(), src.size() * sizeof(int32_t),
                            hipMemcpyHostToDevice, h.s));
    HIPCHECK(hipMemcpyAsync(g->sign.p, sign.data(), sign.size() * sizeof(double),
                            hipMemcpyHostToDevice, h.s));
  }
  HIPCHECK(hipStreamSynchronize(h.s));
  auto& ref = *g;
  h.gathers[key] = std::move(g);
  return ref;
}

std::string skey(const ActString& a) {
  std::string k;
  for (const auto& o : a) {
    k += o.kind;
    k += char('0' + o.spin);
  }
  return k;
}

// Apply an active string (rightmost first) to the reference CI vectors.
// Result [labels in string order][nst][dim]; returns sector, or invalid.
const std::pair<DBuf, Sector>* apply_string(H& h, const ActString& ops) {
  const std::string key = skey(ops);
  auto it = h.vcache.find(key);
  if (it != h.vcache.end()) return &it->second;
  Sector sec = h.sec0;
  int64_t lead = h.nst;
  DBuf cur(lead * h.ndet);
  HIPCHECK(hipMemcpyAsync(cur.p, h.ci.p, (size_t)lead * h.ndet * sizeof(double),
                          hipMemcpyDeviceToDevice, h.s));
  int64_t dim = h.ndet;
  for (auto o = ops.rbegin(); o != ops.rend(); ++o) {
    const Gather& g = gather(h, o->kind, o->spin, sec);
    if (g.dim_to == 0 || !h.as->valid(g.to)) return nullptr;
    DBuf nxt((int64_t)h.na * lead * g.dim_to);
    HIPCHECK(launch_gather_apply(cur.p, lead, dim, g.src.p, g.sign.p, h.na, g.dim_to, nxt.p, h.s));
    cur = std::move(nxt);
    lead *= h.na;
    dim = g.dim_to;
    sec = g.to;
  }
  auto& slot = h.vcache[key];
  slot.first = std::move(cur);
  slot.second = sec;
  return &slot;
}

// sum_sigma-free one-body operator sum_xy f_xy a+_{x s} a_{y s} applied to
// vectors V [lead][dim] in sector sec (same sector out).
void apply_onebody(H& h, const double* fact, int spin, const double* V, int64_t lead, Sector sec,
                   double* out) {
  const Gather& ga = gather(h, 'a', spin, sec);
  if (ga.dim_to == 0 || !h.as->valid(ga.to)) {
    HIPCHECK(vec_fill(lead * h.as->dim(sec), 0.0, out, h.s));
    return;
  }
  const int64_t dim = h.as->dim(sec);
  DBuf Z((int64_t)h.na * lead * ga.dim_to), Z2((int64_t)h.na * lead * ga.dim_to);
  HIPCHECK(launch_gather_apply(V, lead, dim, ga.src.p, ga.sign.p, h.na, ga.dim_to, Z.p, h.s));
  // Z2[x] = sum_y f[x][y] Z[y]
  HIPCHECK(gemm_f64(false, h.na, lead * ga.dim_to, h.na, 1.0, fact, h.na, 0, Z.p,
                    lead * ga.dim_to, 0, 0.0, Z2.p, lead * ga.dim_to, 0, 1, h.s));
  // out = sum_x a+_x Z2[x]: gather each x into a temp and accumulate
  const Gather& gc = gather(h, 'c', spin, ga.to);
  DBuf tmp((int64_t)h.na * lead * dim);
  HIPCHECK(vec_fill(lead * dim, 0.0, out, h.s));
  for (int x = 0; x < h.na; ++x) {
    // only the x-th slab of the creation table applied to Z2[x]
    HIPCHECK(launch_gather_apply(Z2.p + (int64_t)x * lead * ga.dim_to, lead, ga.dim_to,
                                 gc.src.p + (int64_t)x * dim, gc.sign.p + (int64_t)x * dim, 1, dim,
                                 tmp.p, h.s));
    HIPCHECK(vec_axpy(lead * dim, 1.0, tmp.p, out, h.s));
  }
}

struct TypeInfo {
  int nlab;       // active labels of the function
  int64_t ntup;   // na^nlab
};

// Accumulate sum_entries coeff * <bra(M)| mid ket |N> into G with layout
// [mid labels][alpha_b = (M, tb, tuple_b)][alpha_k = (N, tk, tuple_k)].
// For sources (ket_block < 0) alpha_k = N.  fock_mid: the mid string is the
// one-body operator contracted with fact (mid labels absent from G).
void accumulate_gram(H& h, const WickEntry& w, int tb, int ntypes_b, int64_t ntup_b, int tk,
                     int ntypes_k, int64_t ntup_k, bool source, const double* fact, DBuf& G,
                     int64_t nmid_lab) {
  const int nst = h.nst;
  const auto* U = apply_string(h, w.bra);
  if (!U) return;
  ActString wk = w.ket;
  int64_t nmid = 1;
  const bool fock_mid = fact != nullptr;
  if (!fock_mid) {
    wk = w.mid;
    wk.insert(wk.end(), w.ket.begin(), w.ket.end());
    nmid = ipow(h.na, (int)w.mid.size());
  }
  const auto* Wp = apply_string(h, wk);
  if (!Wp) return;
  Sector wsec = Wp->second;
  const int64_t nWlead = Wp->first.n / h.as->dim(wsec);
  const double* Wdata = Wp->first.p;
  DBuf Wf;
  if (fock_mid) {
    if (!(wsec == U->second)) return;
    Wf.alloc(Wp->first.n);
    apply_onebody(h, fact, w.mid[0].spin, Wp->first.p, nWlead, wsec, Wf.p);
    Wdata = Wf.p;
  }
  if (!(wsec == U->second)) return;
  const int64_t dim = h.as->dim(wsec);
  const int64_t nUlead = U->first.n / dim;
  DBuf Gr(nUlead * nWlead);
  HIPCHECK(gemm_f64(true, nUlead, nWlead, dim, 1.0, U->first.p, dim, 0, Wdata, dim, 0, 0.0, Gr.p,
                    nWlead, 0, 1, h.s));
  // Gram axes: [bra labels][M][mid labels][ket labels][N]
  const int nbl = (int)w.bra.size(), nml = fock_mid ? 0 : (int)w.mid.size(),
            nkl = (int)w.ket.size();
  const int64_t na_b_all = (int64_t)nst * ntypes_b * ntup_b;
  const int64_t na_k_all = source ? nst : (int64_t)nst * ntypes_k * ntup_k;
  std::vector<int64_t> dims, strides;
  for (int k = 0; k < nbl; ++k) {
    dims.push_back(h.na);
    strides.push_back(ipow(h.na, nbl - 1 - k) * na_k_all);
  }
  dims.push_back(nst);
  strides.push_back((int64_t)ntypes_b * ntup_b * na_k_all);
  for (int k = 0; k < nml; ++k) {
    dims.push_back(h.na);
    strides.push_back(ipow(h.na, nml - 1 - k) * na_b_all * na_k_all);
  }
  for (int k = 0; k < nkl; ++k) {
    dims.push_back(h.na);
    strides.push_back(ipow(h.na, nkl - 1 - k));
  }
  dims.push_back(nst);
  strides.push_back(source ? 1 : (int64_t)ntypes_k * ntup_k);
  const int64_t base = (int64_t)tb * ntup_b * na_k_all + (source ? 0 : (int64_t)tk * ntup_k);
  (void)nmid_lab;
  HIPCHECK(permute_axpy((int)dims.size(), dims.data(), strides.data(), w.coeff, Gr.p, G.p + base,
                        h.s));
}

// characters of a pairing: which swaps of the block are applied
double perm_sign(const Block& b, const Pairing& P, const std::vector<int>& chi) {
  double sg = 1.0;
  for (size_t s = 0; s < b.swaps.size(); ++s) {
    const std::string lk = b.ext[b.swaps[s].first].first + "_b";
    const std::string ll = b.ext[b.swaps[s].second].first + "_k";
    for (const auto& pr : P.pairs)
      if ((pr.first == lk && pr.second == ll) || (pr.first == ll && pr.second == lk)) sg *= chi[s];
  }
  return sg;
}

int64_t orbit_rows(const H& h, const Block& b, const std::vector<int>& chi) {
  int64_t rows = 1;
  for (size_t k = 0; k < b.ext.size(); ++k) {
    int sw = -1;
    for (size_t s = 0; s < b.swaps.size(); ++s)
      if (b.swaps[s].first == (int)k) sw = (int)s;
    const int64_t dim = b.ext[k].second == CLO ? h.nc : h.nv;
    if (sw >= 0) {
      rows *= chi[sw] < 0 ? dim * (dim - 1) / 2 : dim * (dim + 1) / 2;
      ++k;
    } else {
      rows *= dim;
    }
  }
  return rows;
}

TermDesc base_desc(const H& h, const Block& b, const Entry& e) {
  TermDesc d{};
  d.block = e.block;
  d.nslot = (int)b.ext.size();
  for (int k = 0; k < d.nslot; ++k) d.slot_dim[k] = b.ext[k].second == CLO ? h.nc : h.nv;
  d.nswap = (int)b.swaps.size();
  for (int s = 0; s < d.nswap; ++s) {
    d.swap_k[s] = b.swaps[s].first;
    d.swap_l[s] = b.swaps[s].second;
    d.chi[s] = e.chi[s];
    d.strict[s] = e.chi[s] < 0 ? 1 : 0;
  }
  d.nrow = e.nrow;
  d.nalpha = e.nalpha;
  d.ldo = e.nalpha;
  d.na = h.na;
  return d;
}

void host_sync(H& h) { HIPCHECK(hipStreamSynchronize(h.s)); }

double wall() {
  return std::chrono::duration<double>(std::chrono::steady_clock::now().time_since_epoch()).count();
}

// progress of the set-up on stderr when CASPT2_VERBOSE is set
void progress(H& h, const std::string& what) {
  if (!h.verbose) return;
  host_sync(h);
  std::fprintf(stderr, "[caspt2] %8.2f s  %s\n", wall() - h.t_start, what.c_str());
  std::fflush(stderr);
}

// device-to-host copy of a small array in stream order, through the
// handle's page-locked staging buffer; returns when the data is on the host
void d2h(H& h, void* dst, const void* src, size_t bytes, hipStream_t s) {
  if (bytes == 0) return;
  h.hpin.ensure((int64_t)((bytes + sizeof(double) - 1) / sizeof(double)));
  HIPCHECK(hipMemcpyAsync(h.hpin.p, src, bytes, hipMemcpyDeviceToHost, s));
  HIPCHECK(hipStreamSynchronize(s));
  std::memcpy(dst, h.hpin.p, bytes);
}

double dev_scalar(H& h, const double* p) {
  double v;
  d2h(h, &v, p, sizeof(double), h.s);
  return v;
}

// symmetric eigendecomposition of an n x n device matrix: values (host,
// unsorted as on the diagonal) and vectors (device, columns)
void eigh_dev(H& h, const double* A, int64_t n, std::vector<double>& w, DBuf& Vec, double abs_tol = 0.0) {
  DBuf Aw(n * n);
  HIPCHECK(hipMemcpyAsync(Aw.p, A, (size_t)(n * n) * sizeof(double), hipMemcpyDeviceToDevice, h.s));
  Vec.alloc(n * n);
  if (h.jws.n < jacobi_ws_doubles(n)) h.jws.alloc(jacobi_ws_doubles(n));
  h.hpin.ensure(std::max<int64_t>(n, 8));
  int sweeps = 0;
  // form by size: the LDS workgroup up to 64, the block form above (the
  // scalar whole-device forms remain for comparison, through the debug entry)
  HIPCHECK(jacobi_eigh((int)n, Aw.p, Vec.p, h.jws.p, 60, 1e-15, h.s, &sweeps, 0, nullptr, h.hpin.p, abs_tol));
  // the eigenvalues are the diagonal: a strided copy of n doubles
  HIPCHECK(hipMemcpy2DAsync(h.hpin.p, sizeof(double), Aw.p, (size_t)(n + 1) * sizeof(double), sizeof(double),
                            (size_t)n, hipMemcpyDeviceToHost, h.s));
  host_sync(h);
  w.assign(h.hpin.p, h.hpin.p + n);
}

// X = Q[:, keep] / sqrt(w); then rotate to diagonalise X^T F X (Sec. II.B)
void orthonormal_basis(H& h, Entry& e) {
  const int64_t n = e.nalpha;
  std::vector<double> w;
  DBuf Q;
  // the kept set is decided against an absolute threshold: converge until
  // no diagonal element can be more than 0.1 thresh from its eigenvalue (the
  // off-diagonal norm bounds that distance), where FP64 rotations attain it
  eigh_dev(h, e.S.p, n, w, Q, 0.1 * h.d.ovl_thresh);
  std::vector<int64_t> keep;
  for (int64_t i = 0; i < n; ++i) {
    if (w[i] >= h.d.ovl_thresh) {
      keep.push_back(i);
      e.emin_kept = std::min(e.emin_kept, w[i]);
    } else {
      e.emax_dropped = std::max(e.emax_dropped, w[i]);
    }
  }
  const int64_t nk = (int64_t)keep.size();
  e.nkeep = nk;
  if (nk == 0) {
    e.X.alloc(0);
    e.mu.alloc(0);
    return;
  }
  // X0[:, k] = Q[:, keep[k]] / sqrt(w[keep[k]])
  DBuf X0(n * nk), sc(nk);
  IBuf ki;
  ki.alloc(nk);
  {
    std::vector<int32_t> kk(nk);
    std::vector<double> sv(nk);
    for (int64_t k = 0; k < nk; ++k) {
      kk[k] = (int32_t)keep[k];
      sv[k] = 1.0 / std::sqrt(w[keep[k]]);
    }
    HIPCHECK(hipMemcpyAsync(ki.p, kk.data(), nk * sizeof(int32_t), hipMemcpyHostToDevice, h.s));
    HIPCHECK(hipMemcpyAsync(sc.p, sv.data(), nk * sizeof(double), hipMemcpyHostToDevice, h.s));
    HIPCHECK(select_scale_cols(n, n, Q.p, ki.p, sc.p, nk, X0.p, h.s));
    host_sync(h);
  }
  // Fo = X0^T F X0 : FX = F X0 [n][nk]; Fo = X0^T FX
  DBuf FX(n * nk), X0t(nk * n), Fo(nk * nk);
  HIPCHECK(gemm_f64(false, n, nk, n, 1.0, e.F.p, n, 0, X0.p, nk, 0, 0.0, FX.p, nk, 0, 1, h.s));
  {
    const int64_t dims[2] = {n, nk};
    const int64_t str[2] = {1, n};
    X0t.zero(h.s);
    HIPCHECK(permute_axpy(2, dims, str, 1.0, X0.p, X0t.p, h.s));
  }
  HIPCHECK(gemm_f64(false, nk, nk, n, 1.0, X0t.p, n, 0, FX.p, nk, 0, 0.0, Fo.p, nk, 0, 1, h.s));
  std::vector<double> mu;
  DBuf Z;
  eigh_dev(h, Fo.p, nk, mu, Z);
  e.X.alloc(n * nk);
  HIPCHECK(gemm_f64(false, n, nk, nk, 1.0, X0.p, nk, 0, Z.p, nk, 0, 0.0, e.X.p, nk, 0, 1, h.s));
  e.mu.alloc(nk);
  HIPCHECK(hipMemcpyAsync(e.mu.p, mu.data(), nk * sizeof(double), hipMemcpyHostToDevice, h.s));
  host_sync(h);
}

// DF integral class (sp sq | sr ss) as a contiguous [np][nq][nr][ns] tensor
const double* eri_block(H& h, char sp, char sq, char sr, char ss) {
  std::string key{sp, sq, sr, ss};
  auto it = h.eri.find(key);
  if (it != h.eri.end()) return it->second.p;
  auto off = [&](char c) { return c == CLO ? 0 : c == ACT ? h.nc : h.nc + h.na; };
  auto dim = [&](char c) { return c == CLO ? h.nc : c == ACT ? h.na : h.nv; };
  const int np = dim(sp), nq = dim(sq), nr = dim(sr), ns = dim(ss);
  DBuf A((int64_t)np * nq * h.naux), Bt((int64_t)nr * ns * h.naux);
  HIPCHECK(df_pack(h.B.p, h.naux, h.nmo, off(sp), np, off(sq), nq, A.p, h.s));
  HIPCHECK(df_pack(h.B.p, h.naux, h.nmo, off(sr), nr, off(ss), ns, Bt.p, h.s));
  DBuf out((int64_t)np * nq * nr * ns);
  HIPCHECK(gemm_f64(true, (int64_t)np * nq, (int64_t)nr * ns, h.naux, 1.0, A.p, h.naux, 0, Bt.p,
                    h.naux, 0, 0.0, out.p, (int64_t)nr * ns, 0, 1, h.s));
  auto& slot = h.eri[key];
  slot = std::move(out);
  return slot.p;
}

// row energies: sum of virtual minus closed diagonal Fock elements
void row_energies(H& h, const Block& b, Entry& e) {
  // sum over slots of +eps (virtual) / -eps (closed) on the representative
  e.eps.alloc(e.nrow);
  e.eps.zero(h.s);
  DBuf epsd((int64_t)h.nmo), one(1);
  HIPCHECK(hipMemcpyAsync(epsd.p, h.h_eps.data(), h.nmo * sizeof(double), hipMemcpyHostToDevice,
                          h.s));
  HIPCHECK(vec_fill(1, 1.0, one.p, h.s));
  for (size_t k = 0; k < b.ext.size(); ++k) {
    const bool vir = b.ext[k].second == VIR;
    TermDesc d = base_desc(h, b, e);
    d.nalpha = 1;
    d.ldo = 1;
    d.ncax = 1;
    d.c_slot[0] = (int)k;
    d.c_stride[0] = 1;
    d.nopact = 0;
    d.gcols = 1;
    d.gcol = 0;
    d.galpha = 1;
    d.goff = 0;
    d.mode_avg = 1;
    d.scale = vir ? 1.0 : -1.0;
    HIPCHECK(term_source(d, epsd.p + (vir ? h.nc + h.na : 0), one.p, e.eps.p, h.s));
  }
  // separable form: the first orbital unit (slot 0, or the swap pair (0, 1))
  // indexes A, the remaining units B
  int64_t nA = b.ext.empty() ? 1 : (b.ext[0].second == CLO ? h.nc : h.nv);
  for (size_t sw = 0; sw < b.swaps.size(); ++sw)
    if (b.swaps[sw].first == 0) {
      const int64_t d = nA;
      nA = e.chi[sw] < 0 ? d * (d - 1) / 2 : d * (d + 1) / 2;
    }
  if (nA <= 0 || e.nrow % nA != 0) throw DevError(CASPT2_E_DEVICE, "row energy split");
  e.nB = e.nrow / nA;
  e.epsA.alloc(nA);
  e.epsB.alloc(e.nB);
  HIPCHECK(split_energies(nA, e.nB, e.eps.p, e.epsA.p, e.epsB.p, h.s));
  host_sync(h);
}

}  // namespace

namespace {

std::string pair_key(const Pairing& P) {
  std::vector<std::string> v;
  for (const auto& p : P.pairs) v.push_back(std::min(p.first, p.second) + "=" + std::max(p.first, p.second));
  std::sort(v.begin(), v.end());
  std::string k;
  for (auto& s : v) k += s + ";";
  return k;
}

struct PairAcc {
  Pairing P;   // pairs only
  DBuf G;
};

// copy the (L, L) state block of an all-states alpha x alpha matrix
void state_block(H& h, const double* G, int64_t nall, int64_t n, int L, double c, double* out) {
  DBuf tmp(n * n);
  HIPCHECK(hipMemcpy2DAsync(tmp.p, (size_t)n * sizeof(double), G + (int64_t)L * n * nall + (int64_t)L * n,
                            (size_t)nall * sizeof(double), (size_t)n * sizeof(double), (size_t)n,
                            hipMemcpyDeviceToDevice, h.s));
  HIPCHECK(vec_axpy(n * n, c, tmp.p, out, h.s));
}

void setup_blocks(H& h) {
  const bool ss = h.d.scheme == CASPT2_SSSR;
  const int nst = h.nst;
  const int nsets = ss ? nst : 1;
  h.sets.clear();
  h.sets.resize(nsets);
  // active block of f on the device, contiguous [na][na]
  DBuf fact((int64_t)h.na * h.na);
  {
    std::vector<double> fa((size_t)h.na * h.na);
    for (int r = 0; r < h.na; ++r)
      for (int s = 0; s < h.na; ++s) fa[r * h.na + s] = h.h_fock[(h.nc + r) * h.nmo + h.nc + s];
    if (!fa.empty())
      HIPCHECK(hipMemcpyAsync(fact.p, fa.data(), fa.size() * sizeof(double), hipMemcpyHostToDevice,
                              h.s));
  }
  const auto& BL = blocks();
  for (int bi = 0; bi < NBLOCK; ++bi) {
    const Block& b = BL[bi];
    const int ntypes = (int)b.types.size();
    const int64_t ntup = ipow(h.na, (int)b.act.size());
    const int64_t nall = (int64_t)nst * ntypes * ntup;
    const int64_t nset = (ss ? 1 : nst) * ntypes * ntup;
    // metric and Fock-metric accumulators per pairing
    std::map<std::string, PairAcc> met, fk;
    const OpString fop = E("x_o", ACT, "y_o", ACT, "so");
    for (int tb = 0; tb < ntypes; ++tb)
      for (int tk = 0; tk < ntypes; ++tk) {
        const OpString bra = suffixed(b.types[tb], "_b"), ket = suffixed(b.types[tk], "_k");
        for (int which = 0; which < 2; ++which) {
          auto pairings = matrix_element(bra, which == 0 ? OpString{} : fop, ket);
          auto& acc = which == 0 ? met : fk;
          for (auto& P : pairings) {
            const std::string key = pair_key(P);
            auto it = acc.find(key);
            if (it == acc.end()) {
              PairAcc pa;
              pa.P.pairs = P.pairs;
              pa.G.alloc(nall * nall);
              pa.G.zero(h.s);
              it = acc.emplace(key, std::move(pa)).first;
            }
            for (const auto& w : P.entries)
              accumulate_gram(h, w, tb, ntypes, ntup, tk, ntypes, ntup, false,
                              which == 0 ? nullptr : fact.p, it->second.G, 0);
          }
        }
      }
    for (int set = 0; set < nsets; ++set) {
      for (const auto& chi : characters(b)) {
        Entry e;
        e.block = bi;
        e.chi = chi;
        e.nrow = orbit_rows(h, b, chi);
        e.nalpha = nset;
        e.S.alloc(nset * nset);
        e.F.alloc(nset * nset);
        e.S.zero(h.s);
        e.F.zero(h.s);
        for (int which = 0; which < 2; ++which) {
          auto& acc = which == 0 ? met : fk;
          DBuf& dst = which == 0 ? e.S : e.F;
          for (auto& kv : acc) {
            const double sg = perm_sign(b, kv.second.P, chi);
            if (nset == 0) continue;
            if (ss)
              state_block(h, kv.second.G.p, nall, nset, set, sg, dst.p);
            else
              HIPCHECK(vec_axpy(nset * nset, sg, kv.second.G.p, dst.p, h.s));
          }
        }
        if (e.nrow > 0 && e.nalpha > 0) {
          row_energies(h, b, e);
          orthonormal_basis(h, e);
        }
        h.sets[set].push_back(std::move(e));
      }
    }
    h.vcache.clear();
    host_sync(h);
    progress(h, "metrics and orthonormal bases of block " + b.name);
  }
  // workspace of the split-K residual GEMMs (entries with few rows)
  int64_t ws = 0;
  for (auto& es : h.sets)
    for (auto& e : es)
      if (e.nrow > 0 && e.nalpha > 64) {
        const int ns = residual_splitk(e.nrow, e.nalpha, e.nalpha);
        if (ns > 1) ws = std::max(ws, (int64_t)ns * 2 * e.nrow * e.nalpha);
      }
  h.splitk_ws.alloc(ws);
  // offsets
  for (auto& set : h.sets) {
    int64_t off = 0, ooff = 0;
    for (auto& e : set) {
      e.offset = off;
      e.ooff = ooff;
      off += e.nrow * e.nalpha;
      ooff += e.nrow * e.nkeep;
    }
    h.length = off;
    h.olength = std::max(h.olength, ooff);
  }
}

// the parts of H that act on the references with something left (closed
// creators and virtual annihilators removed): one-body h^c_pq E_pq and
// two-body 1/2 (pq|rs) a+_p a+_r a_s a_q with p, r active or virtual and
// q, s active or closed, not all active; fixed order (the one-body classes,
// then the two-body classes with p slowest)
struct SrcComp {
  OpString ops;
  std::vector<std::string> labels;
  std::vector<char> spaces;
  double scale;
};

std::vector<SrcComp> source_comps() {
  std::vector<SrcComp> comps;
  for (char sp : {ACT, VIR})
    for (char sq : {ACT, CLO}) {
      if (sp == ACT && sq == ACT) continue;
      comps.push_back({E("p_o", sp, "q_o", sq, "so"), {"p_o", "q_o"}, {sp, sq}, 1.0});
    }
  for (char sp : {ACT, VIR})
    for (char sq : {ACT, CLO})
      for (char sr : {ACT, VIR})
        for (char ss2 : {ACT, CLO}) {
          if (sp == ACT && sq == ACT && sr == ACT && ss2 == ACT) continue;
          OpString ops = {Op{'c', "p_o", sp, "so"}, Op{'c', "r_o", sr, "to"},
                          Op{'a', "s_o", ss2, "to"}, Op{'a', "q_o", sq, "so"}};
          comps.push_back({ops, {"p_o", "q_o", "r_o", "s_o"}, {sp, sq, sr, ss2}, 0.5});
        }
  return comps;
}

// Every source term: for each block, component of H, Wick pairing and
// packed entry, fn(comp index, component, term descriptor, coefficient
// tensor, active tensor G [opact][alpha_all][N], set, entry).  The active
// tensors are built per (block, component) and released afterwards.
template <typename Fn>
void for_source_terms(H& h, Fn&& fn) {
  const bool ss = h.d.scheme == CASPT2_SSSR;
  const int nst = h.nst;
  const int nsets = ss ? nst : 1;
  const std::vector<SrcComp> comps = source_comps();
  auto dim = [&](char c) { return c == CLO ? h.nc : c == ACT ? h.na : h.nv; };
  auto off = [&](char c) { return c == CLO ? 0 : c == ACT ? h.nc : h.nc + h.na; };
  const auto& BL = blocks();
  for (int bi = 0; bi < NBLOCK; ++bi) {
    const Block& b = BL[bi];
    const int ntypes = (int)b.types.size();
    const int64_t ntup = ipow(h.na, (int)b.act.size());
    const int64_t nall = (int64_t)nst * ntypes * ntup;
    const int64_t nset = (ss ? 1 : nst) * ntypes * ntup;
    if (nset == 0) continue;
    for (size_t ci = 0; ci < comps.size(); ++ci) {
      const SrcComp& c = comps[ci];
      bool empty = false;
      for (char sp : c.spaces)
        if (dim(sp) == 0) empty = true;
      if (empty) continue;
      std::map<std::string, PairAcc> acc;
      int nopact = 0;
      for (const auto& o : c.ops)
        if (o.space == ACT) ++nopact;
      const int64_t ny = ipow(h.na, nopact);
      for (int tb = 0; tb < ntypes; ++tb) {
        auto pairings = matrix_element(suffixed(b.types[tb], "_b"), c.ops, OpString{});
        for (auto& P : pairings) {
          const std::string key = pair_key(P);
          auto it = acc.find(key);
          if (it == acc.end()) {
            PairAcc pa;
            pa.P.pairs = P.pairs;
            pa.G.alloc(ny * nall * nst);
            pa.G.zero(h.s);
            it = acc.emplace(key, std::move(pa)).first;
          }
          for (const auto& w : P.entries)
            accumulate_gram(h, w, tb, ntypes, ntup, 0, 1, 1, true, nullptr, it->second.G, nopact);
        }
      }
      if (acc.empty()) continue;
      // coefficient tensor
      const double* C = nullptr;
      int64_t cstr[4] = {0, 0, 0, 0};
      if (c.labels.size() == 2) {
        C = h.hcore.p + (int64_t)off(c.spaces[0]) * h.nmo + off(c.spaces[1]);
        cstr[0] = h.nmo;
        cstr[1] = 1;
      } else {
        C = eri_block(h, c.spaces[0], c.spaces[1], c.spaces[2], c.spaces[3]);
        cstr[3] = 1;
        cstr[2] = dim(c.spaces[3]);
        cstr[1] = cstr[2] * dim(c.spaces[2]);
        cstr[0] = cstr[1] * dim(c.spaces[1]);
      }
      for (auto& kv : acc) {
        for (int set = 0; set < nsets; ++set)
          for (auto& e : h.sets[set]) {
            if (e.block != bi || e.nrow == 0) continue;
            TermDesc d = base_desc(h, b, e);
            d.ncax = (int)c.labels.size();
            // active labels index G in operator-string order
            std::vector<std::string> mid_order;
            for (const auto& o : c.ops)
              if (o.space == ACT) mid_order.push_back(o.label);
            for (int a = 0; a < d.ncax; ++a) {
              d.c_stride[a] = cstr[a];
              if (c.spaces[a] == ACT) {
                const int pos = (int)(std::find(mid_order.begin(), mid_order.end(), c.labels[a]) -
                                      mid_order.begin());
                d.c_slot[a] = -1 - pos;
              } else {
                int slot = -1;
                for (const auto& pr : kv.second.P.pairs) {
                  std::string other;
                  if (pr.first == c.labels[a]) other = pr.second;
                  if (pr.second == c.labels[a]) other = pr.first;
                  if (!other.empty())
                    for (size_t k = 0; k < b.ext.size(); ++k)
                      if (b.ext[k].first + "_b" == other) slot = (int)k;
                }
                if (slot < 0) throw DevError(CASPT2_E_DEVICE, "source pairing without bra slot");
                d.c_slot[a] = slot;
              }
            }
            d.nopact = nopact;
            d.gcols = nst;
            d.galpha = nall;
            d.goff = ss ? (int64_t)set * nset : 0;
            d.mode_avg = 0;
            d.scale = c.scale;
            fn((int)ci, c, d, C, (const double*)kv.second.G.p, set, e);
          }
      }
      host_sync(h);
    }
    h.vcache.clear();
    progress(h, "source terms of block " + b.name);
  }
  host_sync(h);
}

// sources <M~| E_Omega^+ H |N~> for every N, packed, per function set
void setup_sources(H& h) {
  const bool ss = h.d.scheme == CASPT2_SSSR;
  const int nst = h.nst;
  const int nsets = ss ? nst : 1;
  h.src.clear();
  h.src.resize(nsets);
  for (int set = 0; set < nsets; ++set)
    for (int N = 0; N < nst; ++N) {
      h.src[set].emplace_back(h.length);
      h.src[set].back().zero(h.s);
    }
  for_source_terms(h, [&](int, const SrcComp&, TermDesc d, const double* C, const double* G, int set,
                          const Entry& e) {
    for (int N = 0; N < nst; ++N) {
      d.gcol = N;
      HIPCHECK(term_source(d, C, G, h.src[set][N].p + e.offset, h.s));
    }
  });
}

// ---------------------------------------------------------------------------
// Fock couplings between blocks (closed-active, active-virtual and
// closed-virtual blocks of f): one term per Wick pairing
// ---------------------------------------------------------------------------
AllDesc all_desc(const H& h, int block) {
  const Block& b = blocks()[block];
  AllDesc a{};
  a.nslot = (int)b.ext.size();
  for (int k = 0; k < a.nslot; ++k) a.slot_dim[k] = b.ext[k].second == CLO ? h.nc : h.nv;
  return a;
}

int64_t all_rows(const H& h, int block) {
  const AllDesc a = all_desc(h, block);
  int64_t n = 1;
  for (int k = 0; k < a.nslot; ++k) n *= a.slot_dim[k];
  return n;
}

PackInfo pack_info(const H& h, int set, int block, const double* base, const std::vector<int64_t>* offs,
                   int64_t rowlen) {
  const Block& b = blocks()[block];
  PackInfo p{};
  p.nslot = (int)b.ext.size();
  for (int k = 0; k < p.nslot; ++k) p.slot_dim[k] = b.ext[k].second == CLO ? h.nc : h.nv;
  p.nswap = (int)b.swaps.size();
  for (int s2 = 0; s2 < p.nswap; ++s2) {
    p.swap_k[s2] = b.swaps[s2].first;
    p.swap_l[s2] = b.swaps[s2].second;
  }
  int ent = 0;
  for (size_t k = 0; k < h.sets[set].size(); ++k) {
    const auto& e = h.sets[set][k];
    if (e.block != block) continue;
    for (int s2 = 0; s2 < p.nswap; ++s2) p.chi[ent][s2] = e.chi[s2];
    p.offset[ent] = offs ? (*offs)[ent] : e.offset;
    ++ent;
  }
  p.nent = ent;
  p.rowlen = rowlen;
  (void)base;
  return p;
}

// Coupling terms of the blocks of f named in comps: between excitation
// blocks for a block of f between two orbital spaces, inside each
// excitation block for one within an orbital space (the operator's
// contraction with itself, the trace of that block, dropped).  One term per
// Wick pairing and function set, appended to terms[set]; used[b] marks the
// excitation blocks taking part.
void make_coupling_terms(H& h, const std::vector<std::pair<char, char>>& comps,
                         std::vector<std::vector<CoupleTerm>>& terms, bool* used) {
  const bool ss = h.d.scheme == CASPT2_SSSR;
  const int nst = h.nst;
  const int nsets = ss ? nst : 1;
  terms.resize(nsets);
  auto off = [&](char c) { return c == CLO ? 0 : c == ACT ? h.nc : h.nc + h.na; };
  const auto& BL = blocks();
  for (int bb = 0; bb < NBLOCK; ++bb)
    for (int kb = 0; kb < NBLOCK; ++kb) {
      const Block& B1 = BL[bb];
      const Block& B2 = BL[kb];
      const int nty_b = (int)B1.types.size(), nty_k = (int)B2.types.size();
      const int64_t ntup_b = ipow(h.na, (int)B1.act.size()), ntup_k = ipow(h.na, (int)B2.act.size());
      const int64_t nall_b = (int64_t)nst * nty_b * ntup_b, nall_k = (int64_t)nst * nty_k * ntup_k;
      const int64_t nset_b = (ss ? 1 : nst) * nty_b * ntup_b, nset_k = (ss ? 1 : nst) * nty_k * ntup_k;
      if (nset_b == 0 || nset_k == 0) continue;
      for (auto comp : comps) {
        // a Fock element within one orbital space keeps every block in
        // itself; one between spaces always changes the block
        if ((comp.first == comp.second) != (bb == kb)) continue;
        const OpString op = E("x_o", comp.first, "y_o", comp.second, "so");
        const int ny = (comp.first == ACT || comp.second == ACT) ? h.na : 1;
        std::map<std::string, PairAcc> acc;
        for (int tb = 0; tb < nty_b; ++tb)
          for (int tk = 0; tk < nty_k; ++tk) {
            auto pairings = matrix_element(suffixed(B1.types[tb], "_b"), op, suffixed(B2.types[tk], "_k"));
            for (auto& P : pairings) {
              // the operator contracted with itself (closed x = y) weighs
              // the trace of the off-diagonal part of f_cc: zero
              bool self = false;
              for (const auto& pr : P.pairs)
                if ((pr.first == "x_o" && pr.second == "y_o") || (pr.first == "y_o" && pr.second == "x_o"))
                  self = true;
              if (self) continue;
              const std::string key = pair_key(P);
              auto it = acc.find(key);
              if (it == acc.end()) {
                PairAcc pa;
                pa.P.pairs = P.pairs;
                pa.G.alloc((int64_t)ny * nall_b * nall_k);
                pa.G.zero(h.s);
                it = acc.emplace(key, std::move(pa)).first;
              }
              for (const auto& w : P.entries)
                accumulate_gram(h, w, tb, nty_b, ntup_b, tk, nty_k, ntup_k, false, nullptr,
                                it->second.G, 0);
            }
          }
        h.vcache.clear();
        for (auto& kv : acc) {
          const auto& pairs = kv.second.P.pairs;
          auto partner = [&](const std::string& lab) {
            for (const auto& pr : pairs) {
              if (pr.first == lab) return pr.second;
              if (pr.second == lab) return pr.first;
            }
            return std::string();
          };
          auto bra_slot = [&](const std::string& lab) {
            for (size_t k = 0; k < B1.ext.size(); ++k)
              if (B1.ext[k].first + "_b" == lab) return (int)k;
            return -1;
          };
          auto ket_slot = [&](const std::string& lab) {
            for (size_t k = 0; k < B2.ext.size(); ++k)
              if (B2.ext[k].first + "_k" == lab) return (int)k;
            return -1;
          };
          // direction: the operator's external labels pair with the bra (up)
          // or with the ket (down)
          bool up = true;
          for (const char* lab : {"x_o", "y_o"}) {
            const char sp = std::string(lab) == "x_o" ? comp.first : comp.second;
            if (sp == ACT) continue;
            if (ket_slot(partner(lab)) >= 0) up = false;
          }
          for (int set = 0; set < nsets; ++set) {
            CoupleTerm t;
            t.up = up;
            t.bra = bb;
            t.ket = kb;
            t.d = CoupleDesc{};
            t.d.ny = ny;
            t.d.f_stride = h.nmo;
            t.f_off = (int64_t)off(comp.first) * h.nmo + off(comp.second);
            int nsum = 0;
            std::map<std::string, int> sum_of;   // ket label -> summed index
            if (up) {
              for (size_t l = 0; l < B2.ext.size(); ++l)
                t.d.ket_src[l] = bra_slot(partner(B2.ext[l].first + "_k"));
            } else {
              for (size_t l = 0; l < B2.ext.size(); ++l) {
                const std::string kl = B2.ext[l].first + "_k";
                const int bs = bra_slot(partner(kl));
                if (bs >= 0) {
                  t.d.ket_src[l] = bs;
                } else {
                  sum_of[kl] = nsum;
                  t.d.sum_dim[nsum] = B2.ext[l].second == CLO ? h.nc : h.nv;
                  t.d.ket_src[l] = -1 - nsum;
                  ++nsum;
                }
              }
            }
            t.d.nsum = nsum;
            for (int which = 0; which < 2; ++which) {
              const std::string lab = which == 0 ? "x_o" : "y_o";
              const char sp = which == 0 ? comp.first : comp.second;
              int src;
              if (sp == ACT) src = -10;
              else if (up || bra_slot(partner(lab)) >= 0) src = bra_slot(partner(lab));
              else src = -1 - sum_of.at(partner(lab));
              (which == 0 ? t.d.fx_src : t.d.fy_src) = src;
            }
            // active tensor of this function set, [y][alpha_b][alpha_k]
            DBuf Gs((int64_t)ny * nset_b * nset_k);
            if (ss) {
              for (int y = 0; y < ny; ++y)
                HIPCHECK(hipMemcpy2DAsync(Gs.p + (int64_t)y * nset_b * nset_k, (size_t)nset_k * sizeof(double),
                                          kv.second.G.p + (int64_t)y * nall_b * nall_k +
                                              (int64_t)set * nset_b * nall_k + (int64_t)set * nset_k,
                                          (size_t)nall_k * sizeof(double), (size_t)nset_k * sizeof(double),
                                          (size_t)nset_b, hipMemcpyDeviceToDevice, h.s));
            } else {
              HIPCHECK(hipMemcpyAsync(Gs.p, kv.second.G.p, Gs.n * sizeof(double), hipMemcpyDeviceToDevice, h.s));
            }
            t.d.bra = all_desc(h, bb);
            t.d.ket = all_desc(h, kb);
            if (up) {
              t.G = std::move(Gs);                     // [(y, alpha_b)][alpha_k]
              t.d.ncol = nset_b;
            } else {
              t.G.alloc((int64_t)nset_b * ny * nset_k);   // [alpha_b][(y, alpha_k)]
              t.G.zero(h.s);
              const int64_t dims3[3] = {ny, nset_b, nset_k};
              const int64_t str3[3] = {nset_k, (int64_t)ny * nset_k, 1};
              HIPCHECK(permute_axpy(3, dims3, str3, 1.0, Gs.p, t.G.p, h.s));
              t.d.ncol = nset_k;
            }
            used[bb] = used[kb] = true;
            terms[set].push_back(std::move(t));
          }
        }
        host_sync(h);
      }
      progress(h, "couplings " + B1.name + " <- " + B2.name);
    }
}

// up terms into ccvv as packed-row passes (caspt2_debug_ccvv_passes turns
// them off for handles created afterwards, to compare with the term path)
bool g_ccvv_passes = true;
int64_t nalpha_of_block(const H& h, int set, int block);

// Classify the terms between cavv and aavv/aaav of every function set by
// their roles in the packed-row pass (couple_cavv.hip), and form the sums
// and differences of the two pairings' G of each role.
void classify_cavv_terms(H& h) {
  const int nsets = (int)h.couple.size();
  h.cavv_fused.assign(nsets, 0);
  h.cavv_g.clear();
  h.cavv_g.resize(nsets);
  const int64_t fac = (int64_t)h.nc * h.nmo, fvc = (int64_t)(h.nc + h.na) * h.nmo, fca = h.nc;
  const int64_t fva = fvc + h.nc, fav = fac + h.nc + h.na, fcv2 = h.nc + h.na;
  for (int set = 0; set < nsets; ++set) {
    const int64_t nak = nalpha_of_block(h, set, CAVV);
    if (!cavv_pass_supported(h.nc, h.nv, (int)nak, h.na)) continue;
    CoupleTerm* by[CV_N] = {};
    bool ok = true, any = false;
    for (auto& t : h.couple[set]) {
      const bool cand = (t.up && t.bra == CAVV && (t.ket == AAVV || t.ket == AAAV || t.ket == CAAV)) ||
                        (!t.up && t.ket == CAVV && (t.bra == AAVV || t.bra == CAAV || t.bra == AAAV));
      if (!cand) continue;
      any = true;
      const int* k = t.d.ket_src;
      int role = -1;
      if (t.d.f_stride == h.nmo && t.sg_slot < 0) {
        if (t.up && t.ket == AAVV && t.d.nsum == 0 && t.d.ny == h.na && t.f_off == fac && t.d.fx_src == -10 &&
            t.d.fy_src == 0 && t.d.ncol == nak) {
          if (k[0] == 1 && k[1] == 2) role = CV_UA1;
          else if (k[0] == 2 && k[1] == 1) role = CV_UA2;
        } else if (t.up && t.ket == AAAV && t.d.nsum == 0 && t.d.ny == 1 && t.f_off == fvc && t.d.fy_src == 0 &&
                   t.d.ncol == nak) {
          if (k[0] == 1 && t.d.fx_src == 2) role = CV_UB1;
          else if (k[0] == 2 && t.d.fx_src == 1) role = CV_UB2;
        } else if (!t.up && t.bra == AAVV && t.d.nsum == 1 && t.d.sum_dim[0] == h.nc && t.d.ny == h.na &&
                   t.f_off == fca && t.d.fx_src == -1 && t.d.fy_src == -10 && t.d.ncol == nak && k[0] == -1) {
          if (k[1] == 0 && k[2] == 1) role = CV_DA1;
          else if (k[1] == 1 && k[2] == 0) role = CV_DA2;
        } else if (t.up && t.ket == CAAV && t.d.nsum == 0 && t.d.ny == h.na && t.f_off == fva && t.d.fy_src == -10 &&
                   t.d.ncol == nak && k[0] == 0) {
          if (k[1] == 1 && t.d.fx_src == 2) role = CV_UC1;
          else if (k[1] == 2 && t.d.fx_src == 1) role = CV_UC2;
        } else if (!t.up && t.bra == CAAV && t.d.nsum == 1 && t.d.sum_dim[0] == h.nv && t.d.ny == h.na &&
                   t.f_off == fav && t.d.fx_src == -10 && t.d.fy_src == -1 && t.d.ncol == nak && k[0] == 0) {
          if (k[1] == -1 && k[2] == 1) role = CV_DB1;
          else if (k[1] == 1 && k[2] == -1) role = CV_DB2;
        } else if (!t.up && t.bra == AAAV && t.d.nsum == 2 && t.d.sum_dim[0] == h.nc && t.d.sum_dim[1] == h.nv &&
                   t.d.ny == 1 && t.f_off == fcv2 && t.d.fx_src == -1 && t.d.fy_src == -2 && t.d.ncol == nak &&
                   k[0] == -1) {
          if (k[1] == -2 && k[2] == 0) role = CV_DC1;
          else if (k[1] == 0 && k[2] == -2) role = CV_DC2;
        }
      }
      if (role < 0 || by[role]) {
        ok = false;
        break;
      }
      by[role] = &t;
    }
    if (!ok || !any) continue;
    CavvG& cg = h.cavv_g[set];
    auto combine = [&](CoupleTerm* t1, CoupleTerm* t2, DBuf (&out)[2]) {
      if (!t1 && !t2) return;
      const int64_t n = (t1 ? t1 : t2)->G.n;
      for (int s2 = 0; s2 < 2; ++s2) {
        out[s2].alloc(n);
        if (t1) HIPCHECK(vec_scale_copy(n, 1.0, t1->G.p, out[s2].p, h.s));
        else HIPCHECK(vec_fill(n, 0.0, out[s2].p, h.s));
        if (t2) HIPCHECK(vec_axpy(n, s2 == 0 ? 1.0 : -1.0, t2->G.p, out[s2].p, h.s));
      }
    };
    for (int r = 0; r < 6; ++r) combine(by[2 * r], by[2 * r + 1], cg.g[r]);
    for (int r = 0; r < CV_N; ++r)
      if (by[r]) by[r]->cavv_role = r;
    h.cavv_fused[set] = 1;
  }
  bool anyset = false;
  for (char f : h.cavv_fused) anyset = anyset || f;
  if (!anyset) return;
  int64_t nak = 0;
  for (int set = 0; set < nsets; ++set) nak = std::max(nak, nalpha_of_block(h, set, CAVV));
  const int64_t nq = (int64_t)h.na * nak;
  const int64_t npv = (int64_t)h.nv * (h.nv + 1) / 2, nmv = (int64_t)h.nv * (h.nv - 1) / 2;
  const int64_t ncv = (int64_t)h.nc * h.nv;
  const int64_t len[12] = {npv * nq, nmv * nq, h.nv * nak, h.nv * nak, npv * nq, nmv * nq,   // Q+- B+- Z+-
                           ncv * nq, ncv * nq, ncv * nq, ncv * nq, 2 * ncv * nak, 2 * h.nv * nak};   // C+- Sb Db Scd Sc
  int64_t off = 0;
  for (int k = 0; k < 12; ++k) {
    h.cavv_off[k] = off;
    off += len[k];
  }
  h.cavv_w.alloc(off);
  host_sync(h);
}

// Classify the up terms into ccvv of every function set by their roles in the
// packed-row passes; a set runs the passes when every such term has a role
// (one term per role) and the shapes fit the kernels, else the term path.
void classify_ccvv_terms(H& h) {
  const int nsets = (int)h.couple.size();
  h.ccvv_fused.assign(nsets, 0);
  if (!g_ccvv_passes || h.nc == 0 || h.nv == 0) return;
  const int64_t fac = (int64_t)h.nc * h.nmo, fvc = (int64_t)(h.nc + h.na) * h.nmo, fva = fvc + h.nc;
  for (int set = 0; set < nsets; ++set) {
    const int64_t ncol = nalpha_of_block(h, set, CCVV), nak = nalpha_of_block(h, set, CAVV);
    if (!ccvv_up_supported(h.nc, h.nv, (int)ncol, h.na, (int)(nak ? nak : h.na * ncol))) continue;
    CoupleTerm* by_kind[CK_N] = {};
    bool ok = true, any = false;
    for (auto& t : h.couple[set]) {
      if (!t.up || t.bra != CCVV) continue;
      any = true;
      const int* k = t.d.ket_src;
      int kind = -1;
      if (t.d.nsum == 0 && t.d.ncol == ncol && t.d.f_stride == h.nmo) {
        if (t.ket == CAVV && t.d.ny == h.na && t.f_off == fac && t.d.fx_src == -10 && t.d.fy_src == 1 &&
            k[0] == 0 && nak == (int64_t)h.na * ncol) {
          if (k[1] == 2 && k[2] == 3) kind = CK_CAVV1;
          else if (k[1] == 3 && k[2] == 2) kind = CK_CAVV2;
        } else if (t.ket == CCAV && t.d.ny == h.na && t.f_off == fva && t.d.fy_src == -10 && k[0] == 0 &&
                   k[1] == 1) {
          if (k[2] == 2 && t.d.fx_src == 3) kind = CK_CCAV1;
          else if (k[2] == 3 && t.d.fx_src == 2) kind = CK_CCAV2;
        } else if (t.ket == CAAV && t.d.ny == 1 && t.f_off == fvc && t.d.fy_src == 1 && k[0] == 0) {
          if (k[1] == 2 && t.d.fx_src == 3) kind = CK_CAAV1;
          else if (k[1] == 3 && t.d.fx_src == 2) kind = CK_CAAV2;
        }
      }
      if (kind < 0 || by_kind[kind]) {
        ok = false;
        break;
      }
      by_kind[kind] = &t;
    }
    if (!ok || !any) continue;
    for (int k = 0; k < CK_N; ++k)
      if (by_kind[k]) by_kind[k]->ccvv_kind = k;
    h.ccvv_fused[set] = 1;
  }
  // down terms out of ccvv into cavv and caav
  h.ccvv_down_fused.assign(nsets, 0);
  const int64_t fca = h.nc, fcv = h.nc + h.na, fav = (int64_t)h.nc * h.nmo + h.nc + h.na;
  for (int set = 0; set < nsets; ++set) {
    const int64_t ncol = nalpha_of_block(h, set, CCVV), nab = nalpha_of_block(h, set, CAVV);
    if (!ccvv_down_supported(h.nc, h.nv, (int)ncol, h.na, (int)(nab ? nab : h.na * ncol))) continue;
    CoupleTerm* by_kind[DK_N] = {};
    bool ok = true, any = false;
    for (auto& t : h.couple[set]) {
      if (t.up || t.ket != CCVV || (t.bra != CAVV && t.bra != CAAV && t.bra != CCAV)) continue;
      any = true;
      const int* k = t.d.ket_src;
      int kind = -1;
      if (t.d.ncol == ncol && t.d.f_stride == h.nmo && t.sg_slot < 0 && k[0] == -1 && k[1] == 0 &&
          t.d.fx_src == -1) {
        if (t.bra == CAVV && t.d.nsum == 1 && t.d.sum_dim[0] == h.nc && t.d.ny == h.na && t.f_off == fca &&
            t.d.fy_src == -10 && nab == (int64_t)h.na * ncol) {
          if (k[2] == 1 && k[3] == 2) kind = DK_CAVV1;
          else if (k[2] == 2 && k[3] == 1) kind = DK_CAVV2;
        } else if (t.bra == CAAV && t.d.nsum == 2 && t.d.sum_dim[0] == h.nc && t.d.sum_dim[1] == h.nv &&
                   t.d.ny == 1 && t.f_off == fcv && t.d.fy_src == -2) {
          if (k[2] == -2 && k[3] == 1) kind = DK_CAAV1;
          else if (k[2] == 1 && k[3] == -2) kind = DK_CAAV2;
        }
      }
      if (t.bra == CCAV && t.d.ncol == ncol && t.d.f_stride == h.nmo && t.sg_slot < 0 && k[0] == 0 && k[1] == 1 &&
          t.d.nsum == 1 && t.d.sum_dim[0] == h.nv && t.d.ny == h.na && t.f_off == fav && t.d.fx_src == -10 &&
          t.d.fy_src == -1 && nalpha_of_block(h, set, CCAV) == (int64_t)h.na * ncol) {
        if (k[2] == -1 && k[3] == 2) kind = DK_CCAV1;
        else if (k[2] == 2 && k[3] == -1) kind = DK_CCAV2;
      }
      if (kind < 0 || by_kind[kind]) {
        ok = false;
        break;
      }
      by_kind[kind] = &t;
    }
    if (!ok || !any) continue;
    for (int k = 0; k < DK_N; ++k)
      if (by_kind[k]) by_kind[k]->ccvv_down = k;
    h.ccvv_down_fused[set] = 1;
  }
  bool anydown = false;
  for (char f : h.ccvv_down_fused) anydown = anydown || f;
  if (anydown) {
    int64_t ncol = 0;
    for (int set = 0; set < nsets; ++set) ncol = std::max(ncol, nalpha_of_block(h, set, CCVV));
    h.ccvv_t.alloc(2 * (int64_t)h.nc * h.nv * h.nv * ncol);
    h.ccvv_y.alloc(2 * (int64_t)h.nc * h.nv * ncol);
  }
  classify_cavv_terms(h);
  bool anyset = false;
  for (char f : h.ccvv_fused) anyset = anyset || f;
  bool anycavv = false;
  for (char f : h.cavv_fused) anycavv = anycavv || f;
  if (!anyset && !anydown && !anycavv) return;
  if (anyset) {
    // W products of the ccav and caav roles, one region per role
    int64_t ncol = 0;
    for (int set = 0; set < nsets; ++set) ncol = std::max(ncol, nalpha_of_block(h, set, CCVV));
    const int64_t wccav = all_rows(h, CCAV) * h.na * ncol, wcaav = all_rows(h, CAAV) * ncol;
    h.ccvv_woff[CK_CAVV1] = h.ccvv_woff[CK_CAVV2] = -1;
    h.ccvv_woff[CK_CCAV1] = 0;
    h.ccvv_woff[CK_CCAV2] = wccav;
    h.ccvv_woff[CK_CAAV1] = 2 * wccav;
    h.ccvv_woff[CK_CAAV2] = 2 * wccav + wcaav;
    h.ccvv_w.alloc(2 * (wccav + wcaav));
  }
  // workgroup table of the virtual-pair passes (up and down)
  const std::vector<uint32_t> groups = ccvv_up_groups(h.nv);
  h.ccvv_ngroups = (int64_t)groups.size();
  h.ccvv_groups.alloc(h.ccvv_ngroups);
  HIPCHECK(hipMemcpyAsync(h.ccvv_groups.p, groups.data(), groups.size() * sizeof(uint32_t), hipMemcpyHostToDevice,
                          h.s));
  const std::vector<uint32_t> bgroups = ccvv_up_groups(h.nv, true);
  h.cavv_groups.alloc(h.ccvv_ngroups);
  HIPCHECK(hipMemcpyAsync(h.cavv_groups.p, bgroups.data(), bgroups.size() * sizeof(uint32_t), hipMemcpyHostToDevice,
                          h.s));
  host_sync(h);
}

void setup_couplings(H& h) {
  const bool ss = h.d.scheme == CASPT2_SSSR;
  const int nst = h.nst;
  const int nsets = ss ? nst : 1;
  h.couple.clear();
  h.couple.resize(nsets);
  auto off = [&](char c) { return c == CLO ? 0 : c == ACT ? h.nc : h.nc + h.na; };
  auto dim = [&](char c) { return c == CLO ? h.nc : c == ACT ? h.na : h.nv; };
  // Fock blocks between orbital classes that are present
  std::vector<std::pair<char, char>> comps;
  for (auto pr : std::vector<std::pair<char, char>>{{ACT, CLO}, {CLO, ACT}, {VIR, ACT}, {ACT, VIR},
                                                    {VIR, CLO}, {CLO, VIR}}) {
    bool nz = false;
    for (int x = 0; x < dim(pr.first) && !nz; ++x)
      for (int y = 0; y < dim(pr.second); ++y)
        if (h.h_fock[(off(pr.first) + x) * h.nmo + off(pr.second) + y] != 0.0) {
          nz = true;
          break;
        }
    if (nz) comps.push_back(pr);
  }
  // off-diagonal closed-closed and virtual-virtual Fock elements (orbitals not
  // canonical in those spaces): terms of each block with itself; the
  // diagonal stays in the row energies, so the device copy of f has it zeroed
  for (char c : {CLO, VIR}) {
    bool nz = false;
    for (int x = 0; x < dim(c) && !nz; ++x)
      for (int y = 0; y < dim(c); ++y)
        if (x != y && h.h_fock[(off(c) + x) * h.nmo + off(c) + y] != 0.0) {
          nz = true;
          break;
        }
    if (nz) comps.push_back({c, c});
  }
  if (comps.empty()) return;
  bool used[NBLOCK] = {false, false, false, false, false, false, false, false};
  const auto& BL = blocks();
  make_coupling_terms(h, comps, h.couple, used);
  // merge terms that act identically (same blocks, index maps, Fock block
  // and shapes): their active tensors add.  A ccvv ket is symmetric under the
  // joint exchange (i, a) <-> (j, b) of its slots, so its slot map is first
  // brought to a canonical form.
  for (int set = 0; set < nsets; ++set) {
    auto& cs = h.couple[set];
    std::vector<CoupleTerm> merged;
    std::map<std::vector<int64_t>, size_t> seen;
    for (auto& t : cs) {
      int* ks = t.d.ket_src;
      canonical_term(t.up, t.bra, t.ket, t.d.bra.nslot, t.d.ket.nslot, t.d.nsum, t.d.ny, ks, &t.d.fx_src,
                     &t.d.fy_src);
      const std::vector<int64_t> key = {t.up, t.bra, t.ket, ks[0], ks[1], ks[2], ks[3], t.d.fx_src, t.d.fy_src,
                                        t.f_off, t.d.nsum, t.d.sum_dim[0], t.d.sum_dim[1], t.d.ny, t.d.ncol,
                                        t.G.n};
      auto it = seen.find(key);
      if (it == seen.end()) {
        seen.emplace(key, merged.size());
        merged.push_back(std::move(t));
      } else {
        HIPCHECK(vec_axpy(t.G.n, 1.0, t.G.p, merged[it->second].G.p, h.s));
      }
    }
    host_sync(h);
    if (h.verbose)
      std::fprintf(stderr, "[caspt2] coupling terms of set %d: %zu merged into %zu\n", set, cs.size(),
                   merged.size());
    cs = std::move(merged);
  }
  // ccvv is unpacked to all orderings once per operator application like the
  // other blocks, so the down terms that read it run on coalesced rows
  // (measured at the full workload: 13.8 ms for the six ccvv down terms
  // against 22.4 ms gathering from the packed rows, for 3.5 ms more
  // unpacking); when that copy would exceed 16 GiB the reduce reads the packed
  // rows instead (ccvv is never the ket of an up term)
  if (used[CCVV]) {
    const int64_t na_ccvv = (ss ? 1 : nst) * (int64_t)BL[CCVV].types.size();
    h.direct[CCVV] = all_rows(h, CCVV) * na_ccvv * (int64_t)sizeof(double) > ((int64_t)16 << 30);
  }
  // slot GEMMs (within-block terms of non-semicanonical orbitals): the ket
  // tensor, slot-permuted where the term needs it, in all-orderings form
  for (auto& cs : h.couple)
    for (auto& t : cs) {
      t.sg_slot = -1;
      t.sg_perm = false;
      int sb, perm[4];
      if (t.up || t.bra != t.ket || t.d.nsum != 1 || t.d.ny != 1 ||
          !slot_form(t.d.ket_src, t.d.fx_src, t.d.fy_src, t.d.ket.nslot, &sb, perm))
        continue;
      int64_t P = 1;
      for (int l = 0; l < sb; ++l) P *= t.d.ket.slot_dim[l];
      if (P > 65535) continue;   // batch limit of the batched GEMM: the reduce runs it
      const int b = t.ket;
      if (b == CCVV && t.d.ket.nslot == 4) {
        // x[e_p0, e_p1, e_p2, e_p3] = x[e_p1, e_p0, e_p3, e_p2]: the two slot
        // maps read the same tensor; keep the smaller
        const int alt[4] = {perm[1], perm[0], perm[3], perm[2]};
        if (std::lexicographical_compare(alt, alt + 4, perm, perm + 4)) std::copy(alt, alt + 4, perm);
      }
      if (!perm_trivial(b, perm, t.d.ket.nslot)) {
        bool have = false, same = true;
        for (auto& cs2 : h.couple)
          for (auto& t2 : cs2)
            if (t2.sg_perm && t2.ket == b) have = true;
        if (have)
          for (int l = 0; l < t.d.ket.nslot; ++l) same = same && h.xperm_p[b][l] == perm[l];
        if (have && !same) continue;   // one permuted copy per block
        std::copy(perm, perm + 4, h.xperm_p[b]);
        t.sg_perm = true;
      }
      t.sg_slot = sb;
      h.direct[b] = false;
    }
  classify_ccvv_terms(h);
  int64_t scratch = 0;
  bool sall_need[NBLOCK] = {false, false, false, false, false, false, false, false};
  bool xall_need[NBLOCK] = {false, false, false, false, false, false, false, false};
  for (auto& cs : h.couple)
    for (auto& t : cs) {
      if (t.cavv_role >= 0) continue;   // the cavv pass reads and writes packed rows only
      if (t.ccvv_down < 0) xall_need[t.ket] = true;   // the ccvv down passes read the packed rows
      if (t.ccvv_kind >= 0) continue;   // packed-row passes: no all-orderings sigma, no scratch
      if (t.ccvv_down >= 0) {
        // into packed rows, except caav (its reduction, in a buffer of its own, then a GEMM)
        if (t.ccvv_down == DK_CAAV1 || t.ccvv_down == DK_CAAV2) sall_need[t.bra] = true;
        continue;
      }
      sall_need[t.bra] = true;
      if (t.up && h.direct[t.ket]) throw DevError(CASPT2_E_NOTIMPL, "up coupling from a packed ket");
      if (t.up)
        scratch = std::max(scratch, all_rows(h, t.ket) * t.d.ny * t.d.ncol);
      else
        scratch = std::max(scratch, all_rows(h, t.bra) * t.d.ny * t.d.ncol);
    }
  h.cscratch.alloc(scratch);
  // all-orderings copies of the blocks taking part (one function set at a time)
  const int64_t nset_of = ss ? 1 : nst;
  for (int b = 0; b < NBLOCK; ++b) {
    if (!used[b]) continue;
    const int64_t na_b = nset_of * (int64_t)BL[b].types.size() * ipow(h.na, (int)BL[b].act.size());
    if (!h.direct[b] && xall_need[b]) h.xall[b].alloc(all_rows(h, b) * na_b);
    if (sall_need[b]) h.sall[b].alloc(all_rows(h, b) * na_b);
  }
  for (auto& cs : h.couple)
    for (auto& t : cs)
      if (t.sg_perm && !h.xperm[t.ket].n) h.xperm[t.ket].alloc(h.xall[t.ket].n);
}

// sigma += (Fock couplings between blocks) x, through all-orderings tensors:
// unpack the blocks, run every term (GEMM over the compound active index and
// an index-mapped expand or reduce with the Fock block), pack once per block.
// (T = float in the inner solver of the mixed-precision mode: the
// all-orderings buffers, sized for doubles, then hold floats.)
// coupling GEMMs: FP64 products split over K (in the current work set's
// split-K workspace) when they have few tiles; FP32 as gemm_t
inline hipError_t gemm_c(H& h, bool nk, int64_t M, int64_t N, int64_t K, double alpha, const double* A, int64_t lda,
                         const double* B, int64_t ldb, double beta, double* C, int64_t ldc) {
  DBuf& ws = h.ws_cur ? *h.ws_cur : h.splitk_ws;
  return gemm_f64_ws(nk, M, N, K, alpha, A, lda, B, ldb, beta, C, ldc, ws.p, ws.n, h.s);
}
inline hipError_t gemm_c(H& h, bool nk, int64_t M, int64_t N, int64_t K, double alpha, const float* A, int64_t lda,
                         const float* B, int64_t ldb, double beta, float* C, int64_t ldc) {
  return gemm_t(nk, M, N, K, alpha, A, lda, B, ldb, beta, C, ldc, h.s);
}

// the current work set's buffers
DBuf& xall_of(H& h, int b) { return h.wset ? h.xall2[b] : h.xall[b]; }
DBuf& xperm_of(H& h, int b) { return h.wset ? h.xperm2[b] : h.xperm[b]; }
DBuf& sall_of(H& h, int b) { return h.wset ? h.sall2[b] : h.sall[b]; }
DBuf& cscratch_of(H& h) { return h.wset ? h.cscratch2 : h.cscratch; }

// allocate the second work set like the first (once)
void ensure_work_set2(H& h) {
  for (int b = 0; b < NBLOCK; ++b) {
    if (h.xall[b].n && h.xall2[b].n != h.xall[b].n) h.xall2[b].alloc(h.xall[b].n);
    if (h.sall[b].n && h.sall2[b].n != h.sall[b].n) h.sall2[b].alloc(h.sall[b].n);
    if (h.xperm[b].n && h.xperm2[b].n != h.xperm[b].n) h.xperm2[b].alloc(h.xperm[b].n);
  }
  if (h.cscratch.n && h.cscratch2.n != h.cscratch.n) h.cscratch2.alloc(h.cscratch.n);
  if (h.ccvv_w.n && h.ccvv_w2.n != h.ccvv_w.n) h.ccvv_w2.alloc(h.ccvv_w.n);
  if (h.ccvv_t.n && h.ccvv_t2.n != h.ccvv_t.n) h.ccvv_t2.alloc(h.ccvv_t.n);
  if (h.ccvv_y.n && h.ccvv_y2.n != h.ccvv_y.n) h.ccvv_y2.alloc(h.ccvv_y.n);
  if (h.cavv_w.n && h.cavv_w2.n != h.cavv_w.n) h.cavv_w2.alloc(h.cavv_w.n);
  if (h.splitk_ws2.n != h.splitk_ws.n) h.splitk_ws2.alloc(h.splitk_ws.n);
}

int64_t nalpha_of_block(const H& h, int set, int block) {
  for (auto& e : h.sets[set])
    if (e.block == block) return e.nalpha;
  return 0;
}

// Y[p][e][q] = sum_z f(e, z) X[p][z][q] along slot sg_slot of the ket's
// all-orderings tensor (p: the slots before it, q: the slots after it and the
// alpha columns): a batched FP64 GEMM on MFMA (the FP32 operator of the
// mixed mode: the FP32 GEMM with the FP32 copy of f).
void prof_begin(H& h, hipEvent_t* a);
void prof_end(H& h, int entry, double bytes, hipEvent_t a);
bool slot_gemm(H& h, const CoupleTerm& t, int64_t nak, const double* X, double* Y, int prof_entry) {
  const int s = t.sg_slot;
  int64_t P = 1, Q = nak;
  for (int l = 0; l < s; ++l) P *= t.d.ket.slot_dim[l];
  for (int l = s + 1; l < t.d.ket.nslot; ++l) Q *= t.d.ket.slot_dim[l];
  const int64_t D = t.d.ket.slot_dim[s];
  const int which = t.ket == CCVV ? 0 : t.ket == CAVV ? 1 : t.ket == CCAV ? 2 : -1;
  const bool timed = which >= 0;
  hipEvent_t ev = nullptr;
  if (timed) prof_begin(h, &ev);
  // f is symmetric: f(e, z) = f(z, e) whichever of the two labels is summed
  HIPCHECK(gemm_f64_batched(D, Q, D, h.fock.p + t.f_off, t.d.f_stride, 0, X, Q, D * Q, Y, Q, D * Q, (int)P, h.s));
  if (timed) prof_end(h, prof_entry + which, 2.0 * (double)D * D * P * Q, ev);
  return true;
}
bool slot_gemm(H& h, const CoupleTerm& t, int64_t nak, const float* X, float* Y, int) {
  if (!h.fock32.p) return false;
  const int s = t.sg_slot;
  int64_t P = 1, Q = nak;
  for (int l = 0; l < s; ++l) P *= t.d.ket.slot_dim[l];
  for (int l = s + 1; l < t.d.ket.nslot; ++l) Q *= t.d.ket.slot_dim[l];
  const int64_t D = t.d.ket.slot_dim[s];
  HIPCHECK(gemm_f32(false, D, Q, D, 1.f, h.fock32.p + t.f_off, t.d.f_stride, 0, X, Q, D * Q, 0.f, Y, Q, D * Q,
                    (int)P, h.s));
  return true;
}

// one coupling term into the all-orderings sigma of its bra (x: the packed
// vector, read directly for a packed ket; the other kets' all-orderings
// copies are current).  fuse: the term's own choice, or -1/0/1 to override.
template <typename T>
void couple_term(H& h, int set, const CoupleTerm& t, const T* x, int fuse) {
  if (t.ccvv_kind >= 0 || t.ccvv_down >= 0 || t.cavv_role >= 0)
    throw DevError(CASPT2_E_ARG, "term applied by a packed-row pass");
  T* scratch = reinterpret_cast<T*>(cscratch_of(h).p);
  T* xk = reinterpret_cast<T*>(xall_of(h, t.ket).p);
  T* sb = reinterpret_cast<T*>(sall_of(h, t.bra).p);
  const double* f = h.fock.p + t.f_off;
  const int64_t nab = nalpha_of_block(h, set, t.bra), nak = nalpha_of_block(h, set, t.ket);
  if (t.up && couple_up_fusable<T>(t.d, nak) && (fuse == -1 || fuse == 1)) {
    HIPCHECK(couple_up_fused(t.d, f, (const T*)xk, nak, Sel<T>::G(t), sb, h.s));
  } else if (t.up) {
    const int64_t width = (int64_t)t.d.ny * nab;
    HIPCHECK(gemm_c(h, true, all_rows(h, t.ket), width, nak, 1.0, xk, nak, Sel<T>::G(t), nak, 0.0, scratch, width));
    HIPCHECK(couple_expand(t.d, f, (const T*)scratch, sb, h.s, fuse == 0 ? 1 : fuse == 2 ? 2 : 0));
  } else {
    const int64_t width = (int64_t)t.d.ny * nak;
    if (t.sg_slot >= 0 &&
        slot_gemm(h, t, nak, reinterpret_cast<const T*>(t.sg_perm ? xperm_of(h, t.ket).p : xall_of(h, t.ket).p),
                  scratch, (int)h.sets[set].size() + 1)) {
      // done: f applied along one slot by a batched GEMM
    } else if (h.direct[t.ket])
      HIPCHECK(couple_reduce_packed(t.d, pack_info(h, set, t.ket, nullptr, nullptr, nak), f, x, scratch, h.s));
    else
      HIPCHECK(couple_reduce(t.d, f, (const T*)xk, scratch, h.s));
    if (nab <= 8 && width <= 8)
      HIPCHECK(rows_small_gemm(all_rows(h, t.bra), (int)nab, (int)width, (const T*)scratch, Sel<T>::G(t), sb, h.s));
    else
      HIPCHECK(gemm_c(h, true, all_rows(h, t.bra), nab, width, 1.0, scratch, width, Sel<T>::G(t), width, 1.0, sb,
                      nab));
  }
}

// the up terms into ccvv of a set whose roles were classified: the W
// products of the ccav and caav terms by GEMM, then the two packed-row passes
// (the cavv terms contract with their active tensors inside the first)
template <typename T>
void ccvv_up_passes(H& h, int set, T* sig) {
  const CoupleTerm* tk[CK_N] = {};
  for (auto& t : h.couple[set])
    if (t.ccvv_kind >= 0) tk[t.ccvv_kind] = &t;
  T* wbuf = reinterpret_cast<T*>((h.wset ? h.ccvv_w2 : h.ccvv_w).p);
  CcvvUpArgs<T> a;
  a.nc = h.nc;
  a.nv = h.nv;
  a.ny = h.na;
  a.ncol = (int)nalpha_of_block(h, set, CCVV);
  a.nak = a.ny * a.ncol;
  for (int k : {CK_CCAV1, CK_CCAV2, CK_CAAV1, CK_CAAV2}) {
    const CoupleTerm* t = tk[k];
    if (!t) continue;
    const int64_t nak = nalpha_of_block(h, set, t->ket);
    const int64_t width = (int64_t)t->d.ny * a.ncol;
    HIPCHECK(gemm_c(h, true, all_rows(h, t->ket), width, nak, 1.0, reinterpret_cast<const T*>(xall_of(h, t->ket).p),
                    nak, Sel<T>::G(*t), nak, 0.0, wbuf + h.ccvv_woff[k], width));
  }
  auto W = [&](int k) { return tk[k] ? (const T*)(wbuf + h.ccvv_woff[k]) : nullptr; };
  const CoupleTerm* tA = tk[CK_CAVV1] ? tk[CK_CAVV1] : tk[CK_CAVV2];
  const CoupleTerm* tB = tk[CK_CCAV1] ? tk[CK_CCAV1] : tk[CK_CCAV2];
  const CoupleTerm* tC = tk[CK_CAAV1] ? tk[CK_CAAV1] : tk[CK_CAAV2];
  if (tA) {
    a.X = reinterpret_cast<const T*>(xall_of(h, CAVV).p);
    a.G1 = tk[CK_CAVV1] ? Sel<T>::G(*tk[CK_CAVV1]) : nullptr;
    a.G2 = tk[CK_CAVV2] ? Sel<T>::G(*tk[CK_CAVV2]) : nullptr;
    a.fA = h.fock.p + tA->f_off;
    a.fA_stride = h.nmo;
  }
  if (tB) {
    a.W3 = W(CK_CCAV1);
    a.W4 = W(CK_CCAV2);
    a.fV = h.fock.p + tB->f_off;
    a.fV_stride = h.nmo;
  }
  if (tC) {
    a.W5 = W(CK_CAAV1);
    a.W6 = W(CK_CAAV2);
    a.fC = h.fock.p + tC->f_off;
    a.fC_stride = h.nmo;
  }
  for (auto& e : h.sets[set])
    if (e.block == CCVV && e.nrow > 0) (e.chi.empty() || e.chi[0] > 0 ? a.plus : a.minus) = sig + e.offset;
  if (!a.plus) return;
  HIPCHECK(ccvv_up_apply<T>(a, reinterpret_cast<const uint32_t*>(h.ccvv_groups.p), h.ccvv_ngroups, h.s));
}

// the down terms out of ccvv into cavv and caav of a set whose roles were
// classified: one packed-row pass (cavv straight into its packed rows, caav
// through the reduction buffer Y), then Y times each caav term's G into the
// all-orderings caav sigma
template <typename T>
void ccvv_down_pass(H& h, int set, const T* x, T* sig) {
  const CoupleTerm* tk[DK_N] = {};
  for (auto& t : h.couple[set])
    if (t.ccvv_down >= 0) tk[t.ccvv_down] = &t;
  CcvvDownArgs<T> d;
  d.nc = h.nc;
  d.nv = h.nv;
  d.ny = h.na;
  d.ncol = (int)nalpha_of_block(h, set, CCVV);
  d.nab = d.ny * d.ncol;
  for (auto& e : h.sets[set]) {
    if (e.nrow == 0) continue;
    const bool pl = e.chi.empty() || e.chi[0] > 0;
    if (e.block == CCVV) (pl ? d.xp : d.xm) = x + e.offset;
    if (e.block == CAVV) (pl ? d.sp : d.sm) = sig + e.offset;
  }
  if (!d.xp) return;
  const CoupleTerm* tD = tk[DK_CAVV1] ? tk[DK_CAVV1] : tk[DK_CAVV2];
  const CoupleTerm* tE = tk[DK_CAAV1] ? tk[DK_CAAV1] : tk[DK_CAAV2];
  const CoupleTerm* tF = tk[DK_CCAV1] ? tk[DK_CCAV1] : tk[DK_CCAV2];
  if (tF) {
    for (auto& e : h.sets[set])
      if (e.block == CCAV && e.nrow > 0) (e.chi.empty() || e.chi[0] > 0 ? d.cp : d.cm) = sig + e.offset;
    d.nab3 = (int)nalpha_of_block(h, set, CCAV);
    d.G3 = tk[DK_CCAV1] ? Sel<T>::G(*tk[DK_CCAV1]) : nullptr;
    d.G4 = tk[DK_CCAV2] ? Sel<T>::G(*tk[DK_CCAV2]) : nullptr;
    d.fV = h.fock.p + tF->f_off;
    d.fV_stride = h.nmo;
  }
  if (tD && d.sp) {
    d.G1 = tk[DK_CAVV1] ? Sel<T>::G(*tk[DK_CAVV1]) : nullptr;
    d.G2 = tk[DK_CAVV2] ? Sel<T>::G(*tk[DK_CAVV2]) : nullptr;
    d.fA = h.fock.p + tD->f_off;
    d.fA_stride = h.nmo;
  } else {
    d.sp = d.sm = nullptr;
  }
  T* Y = reinterpret_cast<T*>((h.wset ? h.ccvv_y2 : h.ccvv_y).p);
  if (tE) {
    d.fC = h.fock.p + tE->f_off;
    d.fC_stride = h.nmo;
    d.Tw = reinterpret_cast<T*>((h.wset ? h.ccvv_t2 : h.ccvv_t).p);
    d.Y = Y;
  }
  HIPCHECK(ccvv_down_apply<T>(d, reinterpret_cast<const uint32_t*>(h.ccvv_groups.p), h.ccvv_ngroups, h.s));
  if (!tE) return;
  const int64_t rows = (int64_t)h.nc * h.nv, nab = nalpha_of_block(h, set, CAAV);
  T* sb = reinterpret_cast<T*>(sall_of(h, CAAV).p);
  for (int k : {DK_CAAV1, DK_CAAV2}) {
    if (!tk[k]) continue;
    const T* Yk = Y + (k == DK_CAAV1 ? 0 : rows * d.ncol);
    if (nab <= 8 && d.ncol <= 8)
      HIPCHECK(rows_small_gemm(rows, (int)nab, d.ncol, Yk, Sel<T>::G(*tk[k]), sb, h.s));
    else
      HIPCHECK(gemm_c(h, true, rows, nab, d.ncol, 1.0, Yk, d.ncol, Sel<T>::G(*tk[k]), d.ncol, 1.0, sb, nab));
  }
}

// the terms between cavv and aavv/aaav of a set whose roles were classified:
// GEMMs of the packed aavv and aaav rows with the summed and differenced G
// of the up terms, the packed-row pass over virtual pairs, and the GEMM of
// its Z rows with the down terms' G into the packed aavv rows
const double* cavv_gp(const CavvG& g, int which, int s, const double*) { return g.g[which][s].p; }
const float* cavv_gp(const CavvG& g, int which, int s, const float*) { return g.g32[which][s].p; }
template <typename T>
void cavv_pass(H& h, int set, const T* x, T* sig) {
  const CoupleTerm* tr[CV_N] = {};
  for (auto& t : h.couple[set])
    if (t.cavv_role >= 0) tr[t.cavv_role] = &t;
  const CavvG& cg = h.cavv_g[set];
  const T* tag = nullptr;
  T* w = reinterpret_cast<T*>((h.wset ? h.cavv_w2 : h.cavv_w).p);
  CavvArgs<T> c;
  c.nc = h.nc;
  c.nv = h.nv;
  c.ny = h.na;
  c.nak = (int)nalpha_of_block(h, set, CAVV);
  const int64_t nq = (int64_t)c.ny * c.nak;
  const T *xa[2] = {nullptr, nullptr}, *xaaav = nullptr, *xcaav = nullptr;
  T* sa[2] = {nullptr, nullptr};
  T *scaav = nullptr, *saaav = nullptr;
  int64_t ra[2] = {0, 0}, naa = 0, naaav = 0, ncaav = 0;
  for (auto& e : h.sets[set]) {
    if (e.nrow == 0) continue;
    const int k = e.chi.empty() || e.chi[0] > 0 ? 0 : 1;
    if (e.block == CAVV) (k == 0 ? c.sp : c.sm) = sig + e.offset;
    if (e.block == CAVV) (k == 0 ? c.xp : c.xm) = x + e.offset;
    if (e.block == AAVV) {
      xa[k] = x + e.offset;
      sa[k] = sig + e.offset;
      ra[k] = e.nrow;
      naa = e.nalpha;
    }
    if (e.block == AAAV) {
      xaaav = x + e.offset;
      saaav = sig + e.offset;
      naaav = e.nalpha;
    }
    if (e.block == CAAV) {
      xcaav = x + e.offset;
      scaav = sig + e.offset;
      ncaav = e.nalpha;
    }
  }
  if (!c.sp) return;
  if ((tr[CV_UA1] || tr[CV_UA2]) && xa[0]) {
    const CoupleTerm* t = tr[CV_UA1] ? tr[CV_UA1] : tr[CV_UA2];
    for (int k = 0; k < 2; ++k) {
      if (!xa[k]) continue;
      T* Q = w + h.cavv_off[k];
      HIPCHECK(gemm_c(h, true, ra[k], nq, naa, 1.0, xa[k], naa, cavv_gp(cg, 0, k, tag), naa, 0.0, Q, nq));
      (k == 0 ? c.Qp : c.Qm) = Q;
    }
    c.fAC = h.fock.p + t->f_off;
    c.fAC_stride = h.nmo;
  }
  if ((tr[CV_UB1] || tr[CV_UB2]) && xaaav) {
    const CoupleTerm* t = tr[CV_UB1] ? tr[CV_UB1] : tr[CV_UB2];
    for (int k = 0; k < 2; ++k) {
      T* B = w + h.cavv_off[2 + k];
      HIPCHECK(gemm_c(h, true, h.nv, c.nak, naaav, 1.0, xaaav, naaav, cavv_gp(cg, 1, k, tag), naaav, 0.0, B, c.nak));
      (k == 0 ? c.Bp : c.Bm) = B;
    }
    c.fVC = h.fock.p + t->f_off;
    c.fVC_stride = h.nmo;
  }
  const int64_t ncv = (int64_t)h.nc * h.nv;
  if ((tr[CV_UC1] || tr[CV_UC2]) && xcaav) {
    const CoupleTerm* t = tr[CV_UC1] ? tr[CV_UC1] : tr[CV_UC2];
    for (int k = 0; k < 2; ++k) {
      T* C = w + h.cavv_off[6 + k];
      HIPCHECK(gemm_c(h, true, ncv, nq, ncaav, 1.0, xcaav, ncaav, cavv_gp(cg, 3, k, tag), ncaav, 0.0, C, nq));
      (k == 0 ? c.Cp : c.Cm) = C;
    }
    c.fVA = h.fock.p + t->f_off;
    c.fVA_stride = h.nmo;
  }
  const bool down = (tr[CV_DA1] || tr[CV_DA2]) && sa[0];
  if (down) {
    const CoupleTerm* t = tr[CV_DA1] ? tr[CV_DA1] : tr[CV_DA2];
    c.Zp = w + h.cavv_off[4];
    if (sa[1]) c.Zm = w + h.cavv_off[5];
    c.fCA = h.fock.p + t->f_off;
    c.fCA_stride = h.nmo;
  }
  const bool downb = (tr[CV_DB1] || tr[CV_DB2]) && scaav;
  if (downb) {
    const CoupleTerm* t = tr[CV_DB1] ? tr[CV_DB1] : tr[CV_DB2];
    c.Sb = w + h.cavv_off[8];
    c.Db = w + h.cavv_off[9];
    c.fAV = h.fock.p + t->f_off;
    c.fAV_stride = h.nmo;
  }
  const bool downc = (tr[CV_DC1] || tr[CV_DC2]) && saaav;
  if (downc) {
    const CoupleTerm* t = tr[CV_DC1] ? tr[CV_DC1] : tr[CV_DC2];
    c.Scd = w + h.cavv_off[10];
    c.Sc = w + h.cavv_off[11];
    c.fCV = h.fock.p + t->f_off;
    c.fCV_stride = h.nmo;
  }
  if (!down && !downb && !downc) c.xp = c.xm = nullptr;
  HIPCHECK(cavv_pass_apply<T>(c, reinterpret_cast<const uint32_t*>(h.cavv_groups.p), h.ccvv_ngroups, h.s));
  if (down)
    for (int k = 0; k < 2; ++k) {
      if (!sa[k]) continue;
      const T* Z = k == 0 ? c.Zp : c.Zm;
      HIPCHECK(gemm_c(h, true, ra[k], naa, nq, 1.0, Z, nq, cavv_gp(cg, 2, k, tag), nq, 1.0, sa[k], naa));
    }
  // caav += [(G1 + G2) Sb + (G1 - G2) Db] / 2, aaav likewise with Sc, Dc
  if (downb)
    for (int k = 0; k < 2; ++k)
      HIPCHECK(gemm_c(h, true, ncv, ncaav, nq, 0.5, k == 0 ? c.Sb : c.Db, nq, cavv_gp(cg, 4, k, tag), nq, 1.0, scaav,
                      ncaav));
  if (downc)
    for (int k = 0; k < 2; ++k)
      HIPCHECK(gemm_c(h, true, h.nv, naaav, c.nak, 0.5, c.Sc + k * h.nv * c.nak, c.nak, cavv_gp(cg, 5, k, tag), c.nak,
                      1.0, saaav, naaav));
}

template <typename T>
void apply_couplings(H& h, int set, const T* x, T* sig) {
  auto nalpha_of = [&](int block) { return nalpha_of_block(h, set, block); };
  auto xall = [&](int b) { return reinterpret_cast<T*>(xall_of(h, b).p); };
  auto sall = [&](int b) { return reinterpret_cast<T*>(sall_of(h, b).p); };
  const bool diag = h.verbose_level >= 2;   // per-stage timing on stderr
  double t_prev = diag ? (host_sync(h), wall()) : 0.0;
  auto stage = [&](const char* what) {
    if (!diag) return;
    host_sync(h);
    const double now = wall();
    std::fprintf(stderr, "[caspt2] coupling %s %.3f ms\n", what, 1e3 * (now - t_prev));
    t_prev = now;
  };
  // stage timing (profiling on): pseudo entries 1000 + k, k the stage's
  // index in h.prof_stage
  auto stage_id = [&](const std::string& name) {
    for (size_t k = 0; k < h.prof_stage.size(); ++k)
      if (h.prof_stage[k] == name) return 1000 + (int)k;
    h.prof_stage.push_back(name);
    return 999 + (int)h.prof_stage.size();
  };
  hipEvent_t sev = nullptr;
  prof_begin(h, &sev);
  for (int b = 0; b < NBLOCK; ++b) {
    if (!sall_of(h, b).p && !xall_of(h, b).p) continue;
    const int64_t na_b = nalpha_of(b);
    if (xall_of(h, b).p) {
      if (b == CCVV && na_b <= 4) {
        // both characters in one tiled pass (the transpose of the pack below)
        const T* plus = nullptr;
        const T* minus = nullptr;
        for (auto& e : h.sets[set])
          if (e.block == b && e.nrow > 0) (e.chi.empty() || e.chi[0] > 0 ? plus : minus) = x + e.offset;
        if (plus) HIPCHECK(unpack_ccvv(h.nc, h.nv, (int)na_b, plus, minus, xall(b), h.s));
      } else {
        HIPCHECK(unpack_all(pack_info(h, set, b, nullptr, nullptr, na_b), all_desc(h, b), x, xall(b), h.s));
      }
    }
    if (xperm_of(h, b).p) {
      // copy[e] = x[e[p[0]], e[p[1]], ...]: scatter x's element at k to the
      // position e with e[p[l]] = k[l]
      const AllDesc ad = all_desc(h, b);
      int64_t dims[5], dst[5], st[5];
      st[ad.nslot] = 1;
      for (int k = ad.nslot - 1; k >= 0; --k) st[k] = st[k + 1] * (k + 1 < ad.nslot ? ad.slot_dim[k + 1] : na_b);
      for (int l = 0; l < ad.nslot; ++l) {
        dims[l] = ad.slot_dim[l];
        dst[l] = st[h.xperm_p[b][l]];
      }
      dims[ad.nslot] = na_b;
      dst[ad.nslot] = 1;
      HIPCHECK(permute_copy(ad.nslot + 1, dims, dst, (const T*)xall(b), reinterpret_cast<T*>(xperm_of(h, b).p),
                            h.s));
    }
    // fill kernel, not a memset: this sequence is recorded into HIP graphs
    if (sall_of(h, b).p) HIPCHECK(vec_fill(sall_of(h, b).n, 0.0, sall_of(h, b).p, h.s));
  }
  stage("unpack");
  if (h.prof_on) prof_end(h, stage_id("unpack"), 0.0, sev);
  for (auto& t : h.couple[set]) {
    if (t.ccvv_kind >= 0 || t.ccvv_down >= 0 || t.cavv_role >= 0) continue;   // below, in the packed-row passes
    if (h.prof_on) prof_begin(h, &sev);
    if (diag) {
      stage("stage");
      std::fprintf(stderr, "[caspt2] term %s %s <- %s ny %d nsum %d slot %d%s: ", t.up ? "up" : "down",
                   blocks()[t.bra].name.c_str(), blocks()[t.ket].name.c_str(), t.d.ny, t.d.nsum, t.sg_slot,
                   t.sg_perm ? " permuted" : "");
    }
    couple_term<T>(h, set, t, x, t.fuse);
    if (h.prof_on)
      prof_end(h, stage_id(std::string(t.up ? "up " : "down ") + blocks()[t.bra].name + " <- " +
                           blocks()[t.ket].name),
               0.0, sev);
  }
  stage("last term");
  if (set < (int)h.ccvv_fused.size() && h.ccvv_fused[set]) {
    if (h.prof_on) prof_begin(h, &sev);
    ccvv_up_passes<T>(h, set, sig);
    stage("ccvv up passes");
    if (h.prof_on) prof_end(h, stage_id("up ccvv passes"), 0.0, sev);
  }
  if (set < (int)h.ccvv_down_fused.size() && h.ccvv_down_fused[set]) {
    if (h.prof_on) prof_begin(h, &sev);
    ccvv_down_pass<T>(h, set, x, sig);
    stage("ccvv down pass");
    if (h.prof_on) prof_end(h, stage_id("down ccvv pass"), 0.0, sev);
  }
  if (set < (int)h.cavv_fused.size() && h.cavv_fused[set]) {
    if (h.prof_on) prof_begin(h, &sev);
    cavv_pass<T>(h, set, x, sig);
    stage("cavv pass");
    if (h.prof_on) prof_end(h, stage_id("cavv pass"), 0.0, sev);
  }
  if (h.prof_on) prof_begin(h, &sev);
  for (int b = 0; b < NBLOCK; ++b) {
    if (!sall_of(h, b).p) continue;
    if (b == CCVV && nalpha_of(b) <= 4) {
      // both characters in one tiled pass
      T* plus = nullptr;
      T* minus = nullptr;
      for (auto& e : h.sets[set])
        if (e.block == b && e.nrow > 0) (e.chi.empty() || e.chi[0] > 0 ? plus : minus) = sig + e.offset;
      if (plus)
        HIPCHECK(pack_ccvv(h.nc, h.nv, (int)nalpha_of(b), (const T*)sall(b), plus, minus, h.s));
      continue;
    }
    for (auto& e : h.sets[set]) {
      if (e.block != b || e.nrow == 0) continue;
      TermDesc d = base_desc(h, blocks()[b], e);
      HIPCHECK(pack_acc(d, all_desc(h, b), (const T*)sall(b), sig + e.offset, h.s));
    }
  }
  stage("pack");
  if (h.prof_on) prof_end(h, stage_id("pack"), 0.0, sev);
}

// ---------------------------------------------------------------------------
// residual and solver
// ---------------------------------------------------------------------------
int set_of(const H& h, int L) { return h.d.scheme == CASPT2_SSSR ? L : 0; }

// Profiling: HIP events around every entry's residual launch (entry index
// of the packed layout) with the algorithmic bytes of the launch (read x,
// read the source if added, write sigma), accumulated until read.
void prof_begin(H& h, hipEvent_t* a) {
  if (!h.prof_on) return;
  HIPCHECK(hipEventCreate(a));
  HIPCHECK(hipEventRecord(*a, h.s));
}

void prof_end(H& h, int entry, double bytes, hipEvent_t a) {
  if (!h.prof_on) return;
  hipEvent_t b;
  HIPCHECK(hipEventCreate(&b));
  HIPCHECK(hipEventRecord(b, h.s));
  h.prof_events.push_back({entry, bytes, a, b});
}

// true if entry k of the set shares one streaming launch with entry k + 1
// (the '+' and '-' entries of a block with nalpha <= 4)
bool paired_rows(const std::vector<Entry>& es, size_t k) {
  const Entry& e = es[k];
  return e.nalpha <= 4 && k + 1 < es.size() && es[k + 1].block == e.block && es[k + 1].nalpha == e.nalpha;
}

// within-block part of the residual for entry k (and k + 1 when paired):
// sig = ((eps + dshift) S + F) x (+ V), with the launch choices tu
template <typename T>
void launch_entry(H& h, const std::vector<Entry>& es, size_t k, LaunchTune tu, const T* x, const T* V,
                  T* sig, double dshift) {
  const Entry& e = es[k];
  if (paired_rows(es, k)) {
    const Entry& e2 = es[k + 1];
    HIPCHECK(residual_rows<T>((int)e.nalpha, e.nrow, e2.nrow, x + e.offset, Sel<T>::S(e), Sel<T>::F(e),
                              e2.nrow ? Sel<T>::S(e2) : nullptr, e2.nrow ? Sel<T>::F(e2) : nullptr,
                              Sel<T>::rows(e), e2.nrow ? Sel<T>::rows(e2) : RowEnergy<T>{nullptr, nullptr, 1},
                              (T)dshift, V ? V + e.offset : nullptr, sig + e.offset, h.s, tu));
  } else if (e.nalpha <= 4) {
    HIPCHECK(residual_rows<T>((int)e.nalpha, e.nrow, 0, x + e.offset, Sel<T>::S(e), Sel<T>::F(e), nullptr,
                              nullptr, Sel<T>::rows(e), RowEnergy<T>{nullptr, nullptr, 1}, (T)dshift,
                              V ? V + e.offset : nullptr, sig + e.offset, h.s, tu));
  } else if (e.nalpha <= 64) {
    HIPCHECK(residual_small_t(e.nrow, e.nalpha, x + e.offset, Sel<T>::S(e), Sel<T>::F(e), Sel<T>::eps(e),
                              dshift, V ? V + e.offset : nullptr, sig + e.offset, h.s, tu));
  } else {
    HIPCHECK(residual_gemm_t(e.nrow, e.nalpha, x + e.offset, Sel<T>::S(e), Sel<T>::F(e), Sel<T>::eps(e),
                             dshift, V ? V + e.offset : nullptr, sig + e.offset, h.s,
                             h.ws_cur ? *h.ws_cur : h.splitk_ws, tu));
  }
}

// sigma_L = A_L x (+ V^(L)) in the packed layout (Eq. 10).  T = double is
// the FP64 operator; T = float the FP32 operator of the mixed-precision
// inner solver (FP32 copies of S, F, eps and of the coupling matrices).
// reverse: launch the entries last to first (a second stream then starts
// with the MFMA-bound entries while the first streams the HBM-bound ones)
template <typename T>
void residual(H& h, int L, const T* x, T* sig, bool with_source, bool reverse = false) {
  const int set = set_of(h, L);
  const double dshift = h.d.shift - h.e0[L];
  const double esz = (double)sizeof(T);
  auto& es = h.sets[set];
  const T* V = nullptr;
  if (with_source) {
    if (sizeof(T) != sizeof(double)) throw DevError(CASPT2_E_ARG, "source only in FP64");
    V = reinterpret_cast<const T*>(h.src[set][L].p);
  }
  std::vector<size_t> units;   // first entry of each launch
  for (size_t k = 0; k < es.size(); ++k) {
    if (es[k].nrow == 0 || es[k].nalpha == 0) continue;
    units.push_back(k);
    if (paired_rows(es, k)) ++k;
  }
  if (reverse) std::reverse(units.begin(), units.end());
  for (size_t k : units) {
    auto& e = es[k];
    const bool pair = paired_rows(es, k);
    const double rows = (double)(e.nrow + (pair ? es[k + 1].nrow : 0));
    hipEvent_t ev = nullptr;
    prof_begin(h, &ev);
    launch_entry<T>(h, es, k, Sel<T>::tune(e), x, V, sig, dshift);
    prof_end(h, (int)k, (with_source ? 3.0 : 2.0) * esz * rows * e.nalpha, ev);
  }
  if (!h.couple.empty() && !h.couple[set].empty()) {
    hipEvent_t ev = nullptr;
    prof_begin(h, &ev);
    apply_couplings<T>(h, set, x, sig);
    prof_end(h, (int)es.size(), 0.0, ev);   // pseudo entry: all couplings
  }
}

// packed -> orthonormal kept basis of every entry: o = v X (Sec. II.B)
template <typename T>
void to_orth(H& h, int set, const T* v, T* o) {
  for (auto& e : h.sets[set]) {
    if (e.nrow == 0 || e.nkeep == 0) continue;
    if (e.nalpha <= 8)
      HIPCHECK(transform_rows<T>(e.nrow, (int)e.nalpha, (int)e.nkeep, v + e.offset, Sel<T>::X(e),
                                 (int)e.nkeep, 1, o + e.ooff, h.s));
    else
      HIPCHECK(gemm_t(false, e.nrow, e.nkeep, e.nalpha, 1.0, v + e.offset, e.nalpha, Sel<T>::X(e), e.nkeep,
                      0.0, o + e.ooff, e.nkeep, h.s));
  }
}

// orthonormal -> packed: v = o X^T
template <typename T>
void from_orth(H& h, int set, const T* o, T* v) {
  for (auto& e : h.sets[set]) {
    if (e.nrow == 0 || e.nalpha == 0) continue;
    if (e.nkeep == 0) {
      HIPCHECK(vec_fill(e.nrow * e.nalpha, 0.0, v + e.offset, h.s));
      continue;
    }
    if (e.nalpha <= 8)
      HIPCHECK(transform_rows<T>(e.nrow, (int)e.nkeep, (int)e.nalpha, o + e.ooff, Sel<T>::X(e), 1,
                                 (int)e.nkeep, v + e.offset, h.s));
    else
      HIPCHECK(gemm_t(true, e.nrow, e.nalpha, e.nkeep, 1.0, o + e.ooff, e.nkeep, Sel<T>::X(e), e.nkeep, 0.0,
                      v + e.offset, e.nalpha, h.s));
  }
}

// coefficients in the orthonormal kept basis of a packed amplitude-like
// vector (T or lambda): t~ = X^T S v per entry, so that X t~ is the
// S-orthogonal projection of v on the kept space (X^T S X = 1); used for
// warm starts
void amp_to_orth(H& h, int set, const double* v, double* o) {
  for (auto& e : h.sets[set]) {
    if (e.nrow == 0 || e.nkeep == 0) continue;
    if (e.SX.n != e.nalpha * e.nkeep) {
      e.SX.alloc(e.nalpha * e.nkeep);
      HIPCHECK(gemm_f64(false, e.nalpha, e.nkeep, e.nalpha, 1.0, e.S.p, e.nalpha, 0, e.X.p, e.nkeep, 0, 0.0,
                        e.SX.p, e.nkeep, 0, 1, h.s));
    }
    if (e.nalpha <= 8)
      HIPCHECK(transform_rows<double>(e.nrow, (int)e.nalpha, (int)e.nkeep, v + e.offset, e.SX.p, (int)e.nkeep,
                                      1, o + e.ooff, h.s));
    else
      HIPCHECK(gemm_t(false, e.nrow, e.nkeep, e.nalpha, 1.0, v + e.offset, e.nalpha, e.SX.p, e.nkeep, 0.0,
                      o + e.ooff, e.nkeep, h.s));
  }
}

int64_t olen(const H& h, int set) {
  int64_t n = 0;
  for (auto& e : h.sets[set]) n += e.nrow * e.nkeep;
  return n;
}

template <typename T>
double ddot(H& h, int64_t n, const T* x, const T* y) {
  HIPCHECK(vec_dot(n, x, y, h.red_partial.p, h.red_out.p, h.s));
  return dev_scalar(h, h.red_out.p);
}

// denominators D[row][k] = eps[row] + E_s - E_L + mu[k]
void build_denoms(H& h, int L, DBuf& D, double* dmin) {
  const int set = set_of(h, L);
  const int64_t n = olen(h, set);
  D.alloc(n);
  DBuf ones_mu, tmp;
  double mn = INFINITY;
  for (auto& e : h.sets[set]) {
    if (e.nrow == 0 || e.nkeep == 0) continue;
    // D = eps (x) 1 + 1 (x) mu + shift via two rank-1 GEMMs
    DBuf one_r(e.nrow), one_k(e.nkeep);
    HIPCHECK(vec_fill(e.nrow, 1.0, one_r.p, h.s));
    HIPCHECK(vec_fill(e.nkeep, 1.0, one_k.p, h.s));
    double* Dp = D.p + e.ooff;
    HIPCHECK(gemm_f64(false, e.nrow, e.nkeep, 1, 1.0, e.eps.p, 1, 0, one_k.p, e.nkeep, 0, 0.0, Dp,
                      e.nkeep, 0, 1, h.s));
    HIPCHECK(gemm_f64(false, e.nrow, e.nkeep, 1, 1.0, one_r.p, 1, 0, e.mu.p, e.nkeep, 0, 1.0, Dp,
                      e.nkeep, 0, 1, h.s));
    HIPCHECK(vec_fill(1, h.d.shift - h.e0[L], one_r.p, h.s));
    DBuf shiftv(e.nrow * e.nkeep);
    HIPCHECK(vec_fill(e.nrow * e.nkeep, h.d.shift - h.e0[L], shiftv.p, h.s));
    HIPCHECK(vec_axpy(e.nrow * e.nkeep, 1.0, shiftv.p, Dp, h.s));
    HIPCHECK(vec_min(e.nrow * e.nkeep, Dp, h.red_partial.p, h.red_out.p, h.s));
    mn = std::min(mn, dev_scalar(h, h.red_out.p));
  }
  *dmin = mn;
}

// FP32 copies of the operands of the inner solver (mixed precision)
void setup_mixed(H& h) {
  if (h.have_mixed) return;
  for (auto& es : h.sets)
    for (auto& e : es) {
      auto cast = [&](const DBuf& src, FBuf& dst) {
        dst.alloc(src.n);
        HIPCHECK(vec_scale_copy(src.n, 1.0, src.p, dst.p, h.s));
      };
      cast(e.S, e.S32);
      cast(e.F, e.F32);
      cast(e.X, e.X32);
      cast(e.eps, e.eps32);
      cast(e.epsA, e.epsA32);
      cast(e.epsB, e.epsB32);
    }
  for (auto& cs : h.couple)
    for (auto& t : cs) {
      t.G32.alloc(t.G.n);
      HIPCHECK(vec_scale_copy(t.G.n, 1.0, t.G.p, t.G32.p, h.s));
    }
  for (auto& cg : h.cavv_g)
    for (int r = 0; r < 6; ++r)
      for (int k = 0; k < 2; ++k)
        if (cg.g[r][k].n) {
          cg.g32[r][k].alloc(cg.g[r][k].n);
          HIPCHECK(vec_scale_copy(cg.g[r][k].n, 1.0, cg.g[r][k].p, cg.g32[r][k].p, h.s));
        }
  h.fock32.alloc(h.fock.n);
  HIPCHECK(vec_scale_copy(h.fock.n, 1.0, h.fock.p, h.fock32.p, h.s));
  h.have_mixed = true;
}

// ---------------------------------------------------------------------------
// Grouped PCG.  Every linear system of a solve (all states of one problem,
// or all amplitude and lambda systems of a batch of problems) advances in
// lockstep.  Per system, the operator application q = A p (from_orth,
// residual, to_orth) is one captured HIP graph; the recurrence runs in the
// grouped kernels with device-resident scalars; the host reads the scalars
// every few iterations only (then retires finished systems and may add new
// ones).
//
// Mixed precision: the same engine runs the recurrence in FP32 (operator,
// transforms, couplings and vectors in FP32, dot products accumulated in
// FP64) as the inner solver of an FP64 iterative refinement.  Per system
// the FP64 solution t and the true residual r = -b - A t (FP64 operator, a
// second captured graph) are kept; each inner solve runs on A d = r / |r|
// until its residual drops by inner_tol (or by what the FP64 tolerance
// still needs), then t += |r| d and r is recomputed.  A system ends when
// |r| meets the FP64 tolerance, when a refinement no longer reduces |r|,
// or when the inner iterations reach maxiter.  The inputs (sources,
// metrics, bases, denominators) are the FP64 ones, rounded once.
// ---------------------------------------------------------------------------
constexpr double MIXED_INNER_TOL = 1e-5;   // relative reduction per inner solve
constexpr int MIXED_INNER_CAP = 200;       // FP32 iterations per inner solve

struct PcgSystem {
  H* h = nullptr;
  int L = 0, set = 0, kind = 0;   // kind 0: amplitudes, 1: lambda
  int64_t n = 0;
  DBuf t, r, p, q, D;             // FP64 mode: the recurrence vectors; mixed: t and true residual r
  FBuf t32, r32, p32, q32, D32;   // mixed: inner correction d, its residual, p, q = A p, denominators
  DBuf b;                         // mixed: right-hand side (for the true residual)
  hipGraphExec_t graph = nullptr;     // q = A p in the recurrence's precision
  hipGraphExec_t graph64 = nullptr;   // mixed: r = A t in FP64
  int id = -1;
  int lane = 0, wset = 0;         // stream of the operator graphs and the handle's work set they use
  int status = PCG_IDLE;
  double tol = 0.0, rn = 0.0;     // mixed: FP64 tolerance and current |r|
  int maxiter = 0;
  caspt2_info info{};
  PcgSystem() = default;
  PcgSystem(const PcgSystem&) = delete;
  PcgSystem& operator=(const PcgSystem&) = delete;
  ~PcgSystem() {
    if (graph) (void)hipGraphExecDestroy(graph);
    if (graph64) (void)hipGraphExecDestroy(graph64);
  }
};

void ensure_work(H& h) {
  if (h.wx.n != h.length) {
    h.wx.alloc(h.length);
    h.wsg.alloc(h.length);
  }
  if (h.wset && h.wx2.n != h.length) {
    h.wx2.alloc(h.length);
    h.wsg2.alloc(h.length);
  }
}

// capture out = A in (orthonormal basis, precision T) of state L into a
// graph recorded on stream s (the handle's own launches are redirected to s
// while recording), using work set wset (its packed work vectors,
// all-orderings tensors, coupling scratch and split-K workspace): the work
// vectors serve both precisions, and graphs of one work set never run
// concurrently (they share a stream)
template <typename T>
hipGraphExec_t capture_operator(H& h, int L, const T* in, T* out, hipStream_t s, int wset = 0) {
  const int keep_wset = h.wset;
  h.wset = wset;
  if (wset) ensure_work_set2(h);
  ensure_work(h);
  const int set = set_of(h, L);
  T* wx = reinterpret_cast<T*>((wset ? h.wx2 : h.wx).p);
  T* wsg = reinterpret_cast<T*>((wset ? h.wsg2 : h.wsg).p);
  const hipStream_t keep = h.s;
  const bool prof = h.prof_on;
  const int vl = h.verbose_level;
  DBuf* keep_ws = h.ws_cur;
  auto restore = [&]() {
    h.s = keep;
    h.prof_on = prof;
    h.verbose_level = vl;
    h.wset = keep_wset;
    h.ws_cur = keep_ws;
  };
  h.ws_cur = wset ? &h.splitk_ws2 : &h.splitk_ws;
  h.s = s;
  h.prof_on = false;
  h.verbose_level = std::min(vl, 1);   // no host synchronisation while recording
  hipGraph_t g = nullptr;
  HIPCHECK(hipStreamBeginCapture(s, hipStreamCaptureModeRelaxed));
  try {
    from_orth(h, set, in, wx);
    residual(h, L, (const T*)wx, wsg, false);
    to_orth(h, set, (const T*)wsg, out);
  } catch (...) {
    (void)hipStreamEndCapture(s, &g);
    if (g) (void)hipGraphDestroy(g);
    restore();
    throw;
  }
  const hipError_t e1 = hipStreamEndCapture(s, &g);
  restore();
  HIPCHECK(e1);
  hipGraphExec_t ex = nullptr;
  const hipError_t e2 = hipGraphInstantiate(&ex, g, nullptr, nullptr, 0);
  (void)hipGraphDestroy(g);
  HIPCHECK(e2);
  return ex;
}

struct PcgEngine {
  hipStream_t s = nullptr;
  bool mixed = false;
  // operator applications of different problems run concurrently on these
  // streams (default priority); all systems of one problem share one stream,
  // as they share its work set (measured: spreading one problem's systems
  // over its two work sets and two streams costs more in set-up than the
  // overlap of its coupling kernels returns); the recurrence waits for all
  // of them
  std::vector<hipStream_t> lanes;
  std::vector<hipEvent_t> lane_done;
  hipEvent_t fork = nullptr;
  std::map<std::pair<const H*, int>, int> lane_of;
  int capacity = 0;
  int check_every = 4;
  std::vector<std::unique_ptr<PcgSystem>> sys;
  std::vector<int> active;             // ids the host still launches
  std::vector<int> stopped;            // ids retired by the last poll
  DevBuf<PcgScalars> sc;
  DevBuf<PcgVecs<double>> vecs;
  DevBuf<PcgVecs<float>> vecs32;
  PinBuf<PcgScalars> hsc;              // host copy of sc (page-locked)
  PinBuf<double> hrr;                  // mixed: squared true-residual norms
  DevBuf<int32_t> blk_sys, sys_id, b0, b1;
  DevBuf<int64_t> blk_start, blk_end;
  DBuf part_a, part_b;
  DBuf dot_part, dot_out;              // mixed: norms of the true residuals
  PcgTable tab{};
  PcgSysTable st{};

  PcgEngine(int cap, int nlanes, bool mixed_) : mixed(mixed_), capacity(cap) {
    HIPCHECK(hipStreamCreateWithFlags(&s, hipStreamNonBlocking));
    HIPCHECK(hipEventCreateWithFlags(&fork, hipEventDisableTiming));
    for (int k = 0; k < std::max(1, nlanes); ++k) {
      hipStream_t ls;
      hipEvent_t ev;
      HIPCHECK(hipStreamCreateWithFlags(&ls, hipStreamNonBlocking));
      lanes.push_back(ls);
      HIPCHECK(hipEventCreateWithFlags(&ev, hipEventDisableTiming));
      lane_done.push_back(ev);
    }
    sc.alloc(cap);
    if (mixed) {
      vecs32.alloc(cap);
      dot_part.alloc(1024);
      dot_out.alloc(cap);
    } else {
      vecs.alloc(cap);
    }
    hsc.ensure(cap);
    for (int k = 0; k < cap; ++k) hsc[k] = PcgScalars{};
  }
  ~PcgEngine() {
    if (s) (void)hipStreamSynchronize(s);
    for (auto ls : lanes) (void)hipStreamSynchronize(ls);
    sys.clear();
    for (auto ev : lane_done) (void)hipEventDestroy(ev);
    for (auto ls : lanes) (void)hipStreamDestroy(ls);
    if (fork) (void)hipEventDestroy(fork);
    if (s) (void)hipStreamDestroy(s);
  }
  int lane(const H* h, int wset) {
    const auto key = std::make_pair(h, wset);
    auto it = lane_of.find(key);
    if (it != lane_of.end()) return it->second;
    const int k = (int)(lane_of.size() % lanes.size());
    lane_of.emplace(key, k);
    return k;
  }
  PcgEngine(const PcgEngine&) = delete;
  PcgEngine& operator=(const PcgEngine&) = delete;

  // in stream order on s (the recurrence kernels read sc on s); waits for
  // the copy so the host may change hsc[id] afterwards
  void upload_scalars(int id) {
    HIPCHECK(hipMemcpyAsync(sc.p + id, hsc.p + id, sizeof(PcgScalars), hipMemcpyHostToDevice, s));
    HIPCHECK(hipStreamSynchronize(s));
  }

  // inner solve of a mixed system from its current true residual (|r| = rn):
  // r32 = r / rn, d = 0, stop at the relative reduction the refinement needs
  void arm_inner(PcgSystem& S) {
    HIPCHECK(vec_scale_copy(S.n, 1.0 / S.rn, S.r.p, S.r32.p, s));
    HIPCHECK(vec_fill(S.n, 0.0, S.t32.p, s));
    PcgScalars& c = hsc[S.id];
    const double goal = std::max(MIXED_INNER_TOL, 0.5 * S.tol / S.rn);
    c.tol2 = goal * goal;
    c.maxiter = std::min(c.iters + MIXED_INNER_CAP, S.maxiter);
    c.status = PCG_IDLE;
    c.active = 0;
    upload_scalars(S.id);
    S.status = PCG_IDLE;
  }

  // new system A x = -b (b in the orthonormal basis, device, on h.s); t0
  // (orthonormal basis, device, nullable): starting solution instead of 0
  PcgSystem& add(H& h, int L, int kind, const double* b, double tol, int maxiter, const double* t0 = nullptr) {
    if ((int)sys.size() >= capacity) throw DevError(CASPT2_E_ARG, "pcg engine capacity");
    if (mixed != (h.d.precision == CASPT2_MIXED)) throw DevError(CASPT2_E_ARG, "pcg engine precision");
    auto S = std::make_unique<PcgSystem>();
    S->h = &h;
    S->L = L;
    S->kind = kind;
    S->set = set_of(h, L);
    S->n = olen(h, S->set);
    S->id = (int)sys.size();
    S->tol = tol;
    S->maxiter = maxiter;
    S->wset = 0;
    S->lane = lane(&h, S->wset);
    caspt2_info& info = S->info;
    double dmin = INFINITY;
    build_denoms(h, L, S->D, &dmin);
    info.min_denom = dmin;
    info.e0 = h.e0[L];
    info.emin_kept = INFINITY;
    info.emax_dropped = -1.0;
    for (auto& e : h.sets[S->set]) {
      info.emin_kept = std::min(info.emin_kept, e.emin_kept);
      info.emax_dropped = std::max(info.emax_dropped, e.emax_dropped);
    }
    S->t.alloc(S->n);
    S->r.alloc(S->n);
    if (t0 && S->n > 0)
      HIPCHECK(hipMemcpyAsync(S->t.p, t0, S->n * sizeof(double), hipMemcpyDeviceToDevice, h.s));
    else
      HIPCHECK(vec_fill(S->n, 0.0, S->t.p, h.s));
    HIPCHECK(vec_scale_copy(S->n, -1.0, b, S->r.p, h.s));
    const bool warm = t0 && S->n > 0 && dmin > 0.0;
    PcgScalars& c = hsc[S->id];
    c = PcgScalars{};
    c.tol2 = tol * tol;
    c.maxiter = maxiter;
    if (!mixed) {
      S->p.alloc(S->n);
      S->q.alloc(S->n);
      host_sync(h);
      S->status = dmin > 0.0 ? PCG_IDLE : PCG_INDEFINITE;
      c.status = S->status;
      PcgVecs<double> v{};
      v.vec[PCG_T] = S->t.p;
      v.vec[PCG_R] = S->r.p;
      v.vec[PCG_P] = S->p.p;
      v.vec[PCG_Q] = S->q.p;
      v.vec[PCG_D] = S->D.p;
      HIPCHECK(hipMemcpy(vecs.p + S->id, &v, sizeof(v), hipMemcpyHostToDevice));
      upload_scalars(S->id);
      if (S->status == PCG_IDLE && S->n > 0)
        S->graph = capture_operator<double>(h, L, S->p.p, S->q.p, s, S->wset);
      if (warm) {
        // r = -(b + A t0): the operator graph maps p to q
        HIPCHECK(hipMemcpyAsync(S->p.p, S->t.p, S->n * sizeof(double), hipMemcpyDeviceToDevice, s));
        HIPCHECK(hipGraphLaunch(S->graph, s));
        HIPCHECK(hipMemcpyAsync(S->r.p, S->q.p, S->n * sizeof(double), hipMemcpyDeviceToDevice, s));
        HIPCHECK(vec_negsum(S->n, b, S->r.p, s));
        HIPCHECK(hipStreamSynchronize(s));
      }
      if (S->n == 0 && S->status == PCG_IDLE) S->status = PCG_CONVERGED;
    } else {
      S->b.alloc(S->n);
      S->t32.alloc(S->n);
      S->r32.alloc(S->n);
      S->p32.alloc(S->n);
      S->q32.alloc(S->n);
      S->D32.alloc(S->n);
      HIPCHECK(hipMemcpyAsync(S->b.p, b, S->n * sizeof(double), hipMemcpyDeviceToDevice, h.s));
      HIPCHECK(vec_scale_copy(S->n, 1.0, S->D.p, S->D32.p, h.s));
      if (warm) {
        // r = -(b + A t0) with the FP64 operator graph (t -> r)
        host_sync(h);
        S->graph64 = capture_operator<double>(h, L, S->t.p, S->r.p, s, S->wset);
        HIPCHECK(hipGraphLaunch(S->graph64, s));
        HIPCHECK(vec_negsum(S->n, S->b.p, S->r.p, s));
        HIPCHECK(hipStreamSynchronize(s));
      }
      S->rn = S->n > 0 ? std::sqrt(ddot(h, S->n, S->r.p, S->r.p)) : 0.0;
      S->D.release();
      PcgVecs<float> v{};
      v.vec[PCG_T] = S->t32.p;
      v.vec[PCG_R] = S->r32.p;
      v.vec[PCG_P] = S->p32.p;
      v.vec[PCG_Q] = S->q32.p;
      v.vec[PCG_D] = S->D32.p;
      HIPCHECK(hipMemcpy(vecs32.p + S->id, &v, sizeof(v), hipMemcpyHostToDevice));
      c.rr = S->rn * S->rn;
      if (!(dmin > 0.0)) {
        S->status = c.status = PCG_INDEFINITE;
        upload_scalars(S->id);
      } else if (S->n == 0 || S->rn <= tol) {
        S->status = c.status = PCG_CONVERGED;
        upload_scalars(S->id);
      } else {
        S->graph = capture_operator<float>(h, L, S->p32.p, S->q32.p, s, S->wset);
        if (!S->graph64) S->graph64 = capture_operator<double>(h, L, S->t.p, S->r.p, s, S->wset);
        arm_inner(*S);
        HIPCHECK(hipStreamSynchronize(s));
      }
    }
    sys.push_back(std::move(S));
    return *sys.back();
  }

  // block and system tables over the given ids (device upload, synchronous;
  // waits for the stream first: queued kernels may still read the tables)
  void build_tables(const std::vector<int>& ids) {
    HIPCHECK(hipStreamSynchronize(s));
    std::vector<int32_t> hb_sys, h_sys, h_b0, h_b1;
    std::vector<int64_t> hb_start, hb_end;
    for (int id : ids) {
      const PcgSystem& S = *sys[id];
      h_sys.push_back(id);
      h_b0.push_back((int32_t)hb_sys.size());
      for (int64_t a = 0; a < S.n; a += PCG_CHUNK) {
        hb_sys.push_back(id);
        hb_start.push_back(a);
        hb_end.push_back(std::min(S.n, a + PCG_CHUNK));
      }
      h_b1.push_back((int32_t)hb_sys.size());
    }
    const int64_t nb = (int64_t)hb_sys.size(), ns = (int64_t)h_sys.size();
    if (nb > INT32_MAX) throw DevError(CASPT2_E_ARG, "pcg block table too large");
    auto up = [](auto& buf, const auto& hv) {
      using E = typename std::decay_t<decltype(hv)>::value_type;
      if (buf.n < (int64_t)hv.size()) buf.alloc(std::max<int64_t>((int64_t)hv.size(), 2 * buf.n));
      if (!hv.empty()) HIPCHECK(hipMemcpy(buf.p, hv.data(), hv.size() * sizeof(E), hipMemcpyHostToDevice));
    };
    up(blk_sys, hb_sys);
    up(blk_start, hb_start);
    up(blk_end, hb_end);
    up(sys_id, h_sys);
    up(b0, h_b0);
    up(b1, h_b1);
    if (part_a.n < nb) {
      part_a.alloc(std::max<int64_t>(nb, 2 * part_a.n));
      part_b.alloc(part_a.n);
    }
    tab = PcgTable{(int)nb, blk_sys.p, blk_start.p, blk_end.p};
    st = PcgSysTable{(int)ns, sys_id.p, b0.p, b1.p};
  }

  // initialise (z, p, rz, rr) and activate the given systems
  void start(const std::vector<int>& ids) {
    std::vector<int> go;
    for (int id : ids)
      if (sys[id]->status == PCG_IDLE) go.push_back(id);
    if (go.empty()) return;
    build_tables(go);
    if (mixed)
      HIPCHECK(pcg_init<float>(tab, st, vecs32.p, sc.p, part_a.p, part_b.p, s));
    else
      HIPCHECK(pcg_init<double>(tab, st, vecs.p, sc.p, part_a.p, part_b.p, s));
    for (int id : go) {
      sys[id]->status = PCG_RUNNING;
      active.push_back(id);
    }
    build_tables(active);
  }

  // copy the scalars to the host; retire systems that stopped on the device
  bool poll() {
    HIPCHECK(hipMemcpyAsync(hsc.p, sc.p, sys.size() * sizeof(PcgScalars), hipMemcpyDeviceToHost, s));
    HIPCHECK(hipStreamSynchronize(s));
    std::vector<int> still;
    stopped.clear();
    for (int id : active) {
      if (hsc[id].status == PCG_RUNNING) {
        still.push_back(id);
      } else {
        sys[id]->status = hsc[id].status;
        stopped.push_back(id);
      }
    }
    const bool changed = still.size() != active.size();
    active.swap(still);
    return changed;
  }

  // mixed: fold the inner corrections of the stopped systems into their
  // FP64 solutions, recompute the true residuals (FP64 operator graphs on
  // the lanes) and restart the inner solve of every system not yet done
  void refine() {
    std::vector<int> ids;
    for (int id : stopped)
      if (sys[id]->status == PCG_CONVERGED || sys[id]->status == PCG_MAXITER) ids.push_back(id);
    if (ids.empty()) return;
    std::vector<int> used(lanes.size(), 0);
    for (int id : ids) {
      PcgSystem& S = *sys[id];
      HIPCHECK(vec_axpy(S.n, S.rn, S.t32.p, S.t.p, s));   // t += |r| d
      used[S.lane] = 1;
    }
    HIPCHECK(hipEventRecord(fork, s));
    for (size_t l = 0; l < lanes.size(); ++l)
      if (used[l]) HIPCHECK(hipStreamWaitEvent(lanes[l], fork, 0));
    for (int id : ids) HIPCHECK(hipGraphLaunch(sys[id]->graph64, lanes[sys[id]->lane]));   // r = A t
    for (size_t l = 0; l < lanes.size(); ++l)
      if (used[l]) {
        HIPCHECK(hipEventRecord(lane_done[l], lanes[l]));
        HIPCHECK(hipStreamWaitEvent(s, lane_done[l], 0));
      }
    for (int id : ids) {
      PcgSystem& S = *sys[id];
      HIPCHECK(vec_negsum(S.n, S.b.p, S.r.p, s));   // r = -(b + A t)
      HIPCHECK(vec_dot(S.n, S.r.p, S.r.p, dot_part.p, dot_out.p + id, s));
    }
    PinBuf<double>& rr = hrr;
    rr.ensure((int64_t)sys.size());
    HIPCHECK(hipMemcpyAsync(rr.p, dot_out.p, sys.size() * sizeof(double), hipMemcpyDeviceToHost, s));
    HIPCHECK(hipStreamSynchronize(s));
    std::vector<int> again;
    for (int id : ids) {
      PcgSystem& S = *sys[id];
      PcgScalars& c = hsc[id];
      const double rn_new = std::sqrt(std::max(rr[id], 0.0));
      S.info.refinements += 1;
      const bool reduced = rn_new < S.rn;
      S.rn = rn_new;
      if (rn_new <= S.tol) {
        S.status = PCG_CONVERGED;
      } else if (!reduced || c.iters >= S.maxiter) {
        S.status = PCG_MAXITER;   // refinement stalled, or the iteration budget is spent
      } else {
        arm_inner(S);
        again.push_back(id);
      }
      c.status = S.status;
    }
    start(again);
  }

  // iterate until no system runs; on_poll (called after every poll, and
  // once before the first iteration) may start new systems
  //
  // Polling interval: a system that stops inside a block of check_every
  // iterations still has its operator graph launched until the next poll
  // (the graph cannot see the device-side status), so long iterations are
  // polled every iteration and short ones (launch- and latency-bound, where
  // a host synchronisation per iteration would dominate) every few.
  template <typename F>
  void run(F&& on_poll) {
    on_poll(*this);
    check_every = 1;
    while (!active.empty()) {
      const double t_block = wall();
      std::vector<int> used(lanes.size(), 0);
      for (int id : active) used[sys[id]->lane] = 1;
      for (int k = 0; k < check_every; ++k) {
        // fork: the lanes wait for the previous recurrence step
        HIPCHECK(hipEventRecord(fork, s));
        for (size_t l = 0; l < lanes.size(); ++l)
          if (used[l]) HIPCHECK(hipStreamWaitEvent(lanes[l], fork, 0));
        for (int id : active) HIPCHECK(hipGraphLaunch(sys[id]->graph, lanes[sys[id]->lane]));
        // join
        for (size_t l = 0; l < lanes.size(); ++l)
          if (used[l]) {
            HIPCHECK(hipEventRecord(lane_done[l], lanes[l]));
            HIPCHECK(hipStreamWaitEvent(s, lane_done[l], 0));
          }
        if (mixed)
          HIPCHECK(pcg_step<float>(tab, st, vecs32.p, sc.p, part_a.p, part_b.p, s));
        else
          HIPCHECK(pcg_step<double>(tab, st, vecs.p, sc.p, part_a.p, part_b.p, s));
      }
      poll();
      const double per_iter = (wall() - t_block) / check_every;
      check_every = per_iter > 1e-3 ? 1 : per_iter > 2.5e-4 ? 2 : 4;
      if (mixed) refine();
      on_poll(*this);
      if (!active.empty()) build_tables(active);
    }
  }

  // free the work vectors and the graphs of a system that has finished
  void retire(PcgSystem& S) {
    S.r.release();
    S.p.release();
    S.q.release();
    S.D.release();
    S.b.release();
    S.t32.release();
    S.r32.release();
    S.p32.release();
    S.q32.release();
    S.D32.release();
    if (S.graph) (void)hipGraphExecDestroy(S.graph);
    if (S.graph64) (void)hipGraphExecDestroy(S.graph64);
    S.graph = S.graph64 = nullptr;
  }

  // final scalars into the system's info; solution stays in S.t
  void finish(PcgSystem& S) {
    const PcgScalars& c = hsc[S.id];
    S.info.iters = c.iters;
    S.info.resnorm = mixed ? S.rn : std::sqrt(std::max(c.rr, 0.0));
    S.info.flags = S.status == PCG_CONVERGED ? 1 : 0;
    if (!mixed) S.info.refinements = 0;
  }
};

// first failure wins, E_INDEFINITE over E_NOCONV
int merge_status(int a, int b) {
  if (a == CASPT2_E_INDEFINITE || b == CASPT2_E_INDEFINITE) return CASPT2_E_INDEFINITE;
  return a != CASPT2_OK ? a : b;
}

int status_code(int pcg_status) {
  switch (pcg_status) {
    case PCG_CONVERGED: return CASPT2_OK;
    case PCG_INDEFINITE: return CASPT2_E_INDEFINITE;
    default: return CASPT2_E_NOCONV;
  }
}

// right-hand sides in the orthonormal basis (device, on h.s)
void amplitude_rhs(H& h, int L, double* b) { to_orth(h, set_of(h, L), (const double*)h.src[set_of(h, L)][L].p, b); }

// b = R_LP sum_N R_NP X^T V^(N) - 2 E_s R_LP^2 t_L   (Eq. 20; X^T S X = 1)
void lambda_rhs(H& h, int L, int P, double* b) {
  const int set = set_of(h, L);
  const int nst = h.nst;
  const int64_t n = olen(h, set);
  DBuf tmp(n);
  HIPCHECK(vec_fill(n, 0.0, b, h.s));
  for (int N = 0; N < nst; ++N) {
    to_orth(h, set, (const double*)h.src[set][N].p, tmp.p);
    HIPCHECK(vec_axpy(n, h.R[L * nst + P] * h.R[N * nst + P], tmp.p, b, h.s));
  }
  HIPCHECK(vec_axpy(n, -2.0 * h.d.shift * h.R[L * nst + P] * h.R[L * nst + P], h.Tt[L].p, b, h.s));
  host_sync(h);
}

// H_eff (Eq. 15) from the amplitudes and its eigenpairs (Eqs. 16-17)
void compute_heff(H& h) {
  const int nst = h.nst;
  std::vector<double> Hm(h.href);
  for (int L = 0; L < nst; ++L) {
    for (int Lp = 0; Lp < nst; ++Lp) {
      const double a = ddot(h, h.length, h.T[L].p, h.src[set_of(h, L)][Lp].p);
      const double b = ddot(h, h.length, h.T[Lp].p, h.src[set_of(h, Lp)][L].p);
      Hm[L * nst + Lp] += 0.5 * (a + b);
    }
    const int64_t n = olen(h, set_of(h, L));
    Hm[L * nst + L] -= h.d.shift * ddot(h, n, h.Tt[L].p, h.Tt[L].p);
  }
  DBuf Hd(nst * nst), wv(nst), Rd(nst * nst);
  HIPCHECK(hipMemcpyAsync(Hd.p, Hm.data(), nst * nst * sizeof(double), hipMemcpyHostToDevice, h.s));
  HIPCHECK(small_eigh(nst, Hd.p, wv.p, Rd.p, h.s));
  h.heff = Hm;
  h.ems.resize(nst);
  h.R.resize(nst * nst);
  d2h(h, h.ems.data(), wv.p, nst * sizeof(double), h.s);
  d2h(h, h.R.data(), Rd.p, nst * nst * sizeof(double), h.s);
  h.have_heff = true;
}

// move a finished system's solution into the handle (packed and orthonormal)
void store_solution(PcgSystem& S, std::vector<DBuf>& packed, std::vector<DBuf>& orth) {
  H& h = *S.h;
  DBuf T(h.length);
  from_orth(h, S.set, (const double*)S.t.p, T.p);
  host_sync(h);
  packed[S.L] = std::move(T);
  orth[S.L] = std::move(S.t);
}

// all states of one handle in one grouped solve (FP64, or mixed with FP64
// refinement, by the handle's precision); kind 0 amplitudes, 1 lambda for
// target P
int grouped_solve(H& h, int kind, int P, double tol, int maxiter, std::vector<DBuf>& packed,
                  std::vector<DBuf>& orth, std::vector<caspt2_info>& infos, const double* x0 = nullptr) {
  const int nst = h.nst;
  PcgEngine eng(nst, 1, h.d.precision == CASPT2_MIXED);
  for (int L = 0; L < nst; ++L) {
    DBuf b(olen(h, set_of(h, L)));
    if (kind == 0)
      amplitude_rhs(h, L, b.p);
    else
      lambda_rhs(h, L, P, b.p);
    DBuf t0(x0 ? b.n : 0);
    if (x0) amp_to_orth(h, set_of(h, L), x0 + (int64_t)L * h.length, t0.p);
    host_sync(h);
    eng.add(h, L, kind, b.p, tol, maxiter, x0 ? t0.p : nullptr);
  }
  std::vector<int> ids(nst);
  for (int L = 0; L < nst; ++L) ids[L] = L;
  eng.start(ids);
  eng.run([](PcgEngine&) {});
  int status = CASPT2_OK;
  packed.resize(nst);
  orth.resize(nst);
  infos.assign(nst, caspt2_info{});
  for (auto& S : eng.sys) {
    eng.finish(*S);
    infos[S->L] = S->info;
    const int rc = status_code(S->status);
    if (rc == CASPT2_E_INDEFINITE) {
      char msg[200];
      const PcgScalars& c = eng.hsc[S->id];
      std::snprintf(msg, sizeof msg, "state %d: %s (min denominator %.6g, p.Ap %.6g after %d iterations)",
                    S->L, S->info.min_denom > 0.0 ? "operator not positive definite" : "non-positive denominator",
                    S->info.min_denom, c.pap, c.iters);
      g_last_error = msg;
      return rc;
    }
    if (rc != CASPT2_OK) status = rc;
  }
  for (auto& S : eng.sys) {
    store_solution(*S, packed, orth);
    eng.retire(*S);
  }
  return status;
}

// ---------------------------------------------------------------------------
// Autotuner of the FP64 residual launches.  Per entry, every candidate
// launch choice -- the K split count and the tile order (plain or
// XCD-grouped) of the residual GEMM, the workgroup-count cap of the
// streaming kernels -- is timed on the entry's own operands and the fastest
// kept; the rule's choice is always a candidate, so tuning never picks a
// slower launch than the rule on the timing run.  Choices are cached per
// shape in the process and, when a path is given, in a text file (one line
// per shape: the key, then splitk order grid), so handles of equal shapes
// time once.  Every candidate computes the same residual; split counts
// differ from each other only in the order of the K summation.
// ---------------------------------------------------------------------------
std::mutex g_tune_mu;
std::map<std::string, LaunchTune> g_tune_cache;

std::string tune_key(const std::vector<Entry>& es, size_t k) {
  const Entry& e = es[k];
  char buf[160];
  if (paired_rows(es, k))
    std::snprintf(buf, sizeof buf, "rows2 %lld %lld %lld", (long long)e.nalpha, (long long)e.nrow,
                  (long long)es[k + 1].nrow);
  else if (e.nalpha <= 4)
    std::snprintf(buf, sizeof buf, "rows %lld %lld", (long long)e.nalpha, (long long)e.nrow);
  else if (e.nalpha <= 64)
    std::snprintf(buf, sizeof buf, "small %lld %lld", (long long)e.nalpha, (long long)e.nrow);
  else
    std::snprintf(buf, sizeof buf, "gemm %lld %lld", (long long)e.nalpha, (long long)e.nrow);
  return buf;
}

std::vector<LaunchTune> tune_candidates(const std::vector<Entry>& es, size_t k, int64_t ws_cap) {
  const Entry& e = es[k];
  std::vector<LaunchTune> c;
  c.push_back(LaunchTune{});   // the rule
  if (e.nalpha <= 64) {
    const int64_t rows = e.nrow + (paired_rows(es, k) ? es[k + 1].nrow : 0);
    const int64_t natural = e.nalpha <= 4 ? (rows + 255) / 256
                            : e.nalpha <= 16 ? (rows * e.nalpha + 255) / 256
                                             : ((rows + 15) / 16 + 3) / 4;
    const bool mfma = e.nalpha > 16;   // the streaming MFMA kernel (plain, prefetch, prefetch + B in registers)
    for (int form : {0, 1, 2}) {
      if (form && !mfma) continue;
      if (form == 2 && e.nalpha > 32) continue;
      if (form) {
        LaunchTune t;
        t.plain = form == 1;
        t.breg = form == 2;
        c.push_back(t);
      }
      for (unsigned g : {512u, 1024u, 2048u, 4096u, 8192u, 16384u, 32768u})
        if ((int64_t)g < natural) {
          LaunchTune t;
          t.grid = g;
          t.plain = form == 1;
          t.breg = form == 2;
          c.push_back(t);
        }
    }
    return c;
  }
  const int64_t M = e.nrow, N = e.nalpha, K = e.nalpha;
  for (int order : {-1, 2})
    for (int ns : {1, 2, 4, 8, 16, 32, 64}) {
      if (ns > 1 && ((int64_t)ns * BK_RESIDUAL > K || (int64_t)ns * 2 * M * N > ws_cap)) continue;
      for (int tile : {64, 128})
        for (int kb : {16, 32})
          for (int occ : {0, 1}) {   // the rule's occupancy, or one wave per SIMD
            if ((tile == 128 || kb == 32 || occ == 1) && ns > 1) continue;
            if (tile == 128 && M < 4 * 128) continue;
            if (occ == 1 && tile == 128 && kb == 32) continue;
            LaunchTune t;
            t.splitk = ns;
            t.order = order;
            t.tile = tile;
            t.kb = kb;
            t.occ = occ;
            c.push_back(t);
          }
    }
  return c;
}

double time_entry(H& h, const std::vector<Entry>& es, size_t k, const LaunchTune& tu, const double* x,
                  const double* V, double* out, double dshift, hipEvent_t a, hipEvent_t b) {
  launch_entry<double>(h, es, k, tu, x, V, out, dshift);   // warm-up
  HIPCHECK(hipEventRecord(a, h.s));
  launch_entry<double>(h, es, k, tu, x, V, out, dshift);
  HIPCHECK(hipEventRecord(b, h.s));
  HIPCHECK(hipEventSynchronize(b));
  float ms1 = 0.0f;
  HIPCHECK(hipEventElapsedTime(&ms1, a, b));
  const int reps = std::max(2, std::min(20, (int)(2.0 / std::max(ms1, 1e-3f))));
  HIPCHECK(hipEventRecord(a, h.s));
  for (int r = 0; r < reps; ++r) launch_entry<double>(h, es, k, tu, x, V, out, dshift);
  HIPCHECK(hipEventRecord(b, h.s));
  HIPCHECK(hipEventSynchronize(b));
  float ms = 0.0f;
  HIPCHECK(hipEventElapsedTime(&ms, a, b));
  return ms / reps;
}

void load_tune_file(const char* path) {
  if (!path) return;
  FILE* f = std::fopen(path, "r");
  if (!f) return;
  char line[256];
  while (std::fgets(line, sizeof line, f)) {
    char* tab = std::strchr(line, '\t');
    if (!tab) continue;
    *tab = 0;
    LaunchTune t;
    const int got = std::sscanf(tab + 1, "%d %d %u %d %d %d %d %d", &t.splitk, &t.order, &t.grid, &t.tile, &t.kb,
                                &t.occ, &t.plain, &t.breg);
    if (got < 3) continue;
    if (got < 4) t.tile = 0;
    if (got < 5) t.kb = 0;
    if (got < 6) t.occ = 0;
    if (got < 7) t.plain = 0;
    if (got < 8) t.breg = 0;
    g_tune_cache[line] = t;
  }
  std::fclose(f);
}

void save_tune_file(const char* path) {
  if (!path) return;
  const std::string tmp = std::string(path) + ".tmp";
  FILE* f = std::fopen(tmp.c_str(), "w");
  if (!f) throw DevError(CASPT2_E_ARG, "cannot write the tuning cache file");
  for (auto& kv : g_tune_cache)
    std::fprintf(f, "%s\t%d %d %u %d %d %d %d %d\n", kv.first.c_str(), kv.second.splitk, kv.second.order,
                 kv.second.grid, kv.second.tile, kv.second.kb, kv.second.occ, kv.second.plain, kv.second.breg);
  std::fclose(f);
  if (std::rename(tmp.c_str(), path) != 0) throw DevError(CASPT2_E_ARG, "cannot replace the tuning cache file");
}

void autotune(H& h, const char* cache_path, bool force) {
  std::lock_guard<std::mutex> lock(g_tune_mu);
  load_tune_file(cache_path);
  ensure_work(h);
  const int64_t ws_cap = std::max<int64_t>(h.splitk_ws.n, (int64_t)1 << 26);   // 512 MB of partials
  hipEvent_t a, b;
  HIPCHECK(hipEventCreate(&a));
  HIPCHECK(hipEventCreate(&b));
  try {
    for (size_t set = 0; set < h.sets.size(); ++set) {
      auto& es = h.sets[set];
      const int L = h.d.scheme == CASPT2_SSSR ? (int)set : 0;
      // x, the source V and the output in three distinct buffers, as in the
      // solver (values do not matter for timing)
      const double* V = h.src[set][L].p;
      HIPCHECK(hipMemcpyAsync(h.wx.p, V, h.length * sizeof(double), hipMemcpyDeviceToDevice, h.s));
      const double* x = h.wx.p;
      const double dshift = h.d.shift - h.e0[L];
      for (size_t k = 0; k < es.size(); ++k) {
        Entry& e = es[k];
        const bool pair = paired_rows(es, k);
        if (e.nrow == 0 || e.nalpha == 0) continue;
        const std::string key = tune_key(es, k);
        auto it = g_tune_cache.find(key);
        if (it != g_tune_cache.end() && !force) {
          e.tune = it->second;
          e.tune_rule_ms = e.tune_best_ms = -1.0;
        } else {
          const auto cands = tune_candidates(es, k, ws_cap);
          int64_t need = h.splitk_ws.n;
          for (auto& c : cands)
            if (c.splitk > 1) need = std::max(need, (int64_t)c.splitk * 2 * e.nrow * e.nalpha);
          if (need > h.splitk_ws.n) h.splitk_ws.alloc(need);
          double best = INFINITY, rule = INFINITY;
          LaunchTune pick;
          for (size_t c = 0; c < cands.size(); ++c) {
            const double ms = time_entry(h, es, k, cands[c], x, V, h.wsg.p, dshift, a, b);
            if (c == 0) rule = ms;
            if (ms < best) {
              best = ms;
              pick = cands[c];
            }
          }
          e.tune = pick;
          e.tune_rule_ms = rule;
          e.tune_best_ms = best;
          g_tune_cache[key] = pick;
          if (h.verbose)
            std::fprintf(stderr,
                         "[caspt2] tune %-28s splitk %d order %d grid %u tile %d kb %d occ %d plain %d breg %d: "
                         "%.4f ms (rule %.4f ms)\n",
                         key.c_str(), pick.splitk, pick.order, pick.grid, pick.tile, pick.kb, pick.occ, pick.plain,
                         pick.breg, best, rule);
        }
        if (pair) es[k + 1].tune = e.tune;
        if (pair) ++k;
      }
    }
    // up coupling terms that can run fused: fused against GEMM + expand
    for (size_t set = 0; set < h.couple.size(); ++set)
      for (auto& t : h.couple[set]) {
        const int64_t nak = nalpha_of_block(h, (int)set, t.ket);
        if (!t.up || t.d.ny > 8 || t.ccvv_kind >= 0 || t.ccvv_down >= 0 || t.cavv_role >= 0) continue;
        const bool fusable = couple_up_fusable<double>(t.d, nak);
        int64_t rows_k = 1;
        for (int k = 0; k < t.d.ket.nslot; ++k) rows_k *= t.d.ket.slot_dim[k];
        char kb[200];
        std::snprintf(kb, sizeof kb, "term %d %d %d %lld %lld %lld %d %d %d %d %d %d", t.bra, t.ket, t.d.ny,
                      (long long)t.d.ncol, (long long)nak, (long long)rows_k, t.d.ket_src[0], t.d.ket_src[1],
                      t.d.ket_src[2], t.d.ket_src[3], t.d.fx_src, t.d.fy_src);
        const std::string key = kb;
        auto it = g_tune_cache.find(key);
        if (it != g_tune_cache.end() && !force) {
          t.fuse = it->second.splitk;   // the first field holds the fused flag for term keys
          continue;
        }
        double best = INFINITY;
        int pick = -1;
        for (int fz : {1, 0, 2}) {
          if (fz == 1 && !fusable) continue;
          couple_term<double>(h, (int)set, t, h.wx.p, fz);   // warm-up
          HIPCHECK(hipEventRecord(a, h.s));
          for (int r = 0; r < 2; ++r) couple_term<double>(h, (int)set, t, h.wx.p, fz);
          HIPCHECK(hipEventRecord(b, h.s));
          HIPCHECK(hipEventSynchronize(b));
          float ms = 0.0f;
          HIPCHECK(hipEventElapsedTime(&ms, a, b));
          if (ms / 2 < best) {
            best = ms / 2;
            pick = fz;
          }
        }
        t.fuse = pick;
        LaunchTune lt;
        lt.splitk = pick;
        g_tune_cache[key] = lt;
        if (h.verbose)
          std::fprintf(stderr, "[caspt2] tune %s: %s %.4f ms\n", key.c_str(),
                       pick == 1 ? "fused" : pick == 2 ? "GEMM + output-parallel expand" : "GEMM + ket-parallel expand",
                       best);
      }
    // workspace for the chosen split counts
    int64_t ws = 0;
    for (auto& es : h.sets)
      for (auto& e : es)
        if (e.nrow > 0 && e.nalpha > 64) {
          const int ns = e.tune.splitk >= 1 ? e.tune.splitk : residual_splitk(e.nrow, e.nalpha, e.nalpha);
          if (ns > 1) ws = std::max(ws, (int64_t)ns * 2 * e.nrow * e.nalpha);
        }
    if (ws != h.splitk_ws.n) h.splitk_ws.alloc(ws);
    save_tune_file(cache_path);
  } catch (...) {
    (void)hipEventDestroy(a);
    (void)hipEventDestroy(b);
    throw;
  }
  HIPCHECK(hipEventDestroy(a));
  HIPCHECK(hipEventDestroy(b));
}

void validate(const caspt2_dims* d, const std::vector<double>& f, const std::vector<double>& hc,
              int nmo, int nc, int na) {
  auto bad = [](const char* m) { throw DevError(CASPT2_E_ARG, m); };
  for (double v : f)
    if (!std::isfinite(v)) bad("non-finite fock");
  for (double v : hc)
    if (!std::isfinite(v)) bad("non-finite hcore");
  for (int i = 0; i < nmo; ++i)
    for (int j = 0; j < nmo; ++j) {
      if (std::fabs(f[i * nmo + j] - f[j * nmo + i]) > 1e-12) bad("fock not symmetric");
      if (std::fabs(hc[i * nmo + j] - hc[j * nmo + i]) > 1e-12) bad("hcore not symmetric");
    }
  (void)d;
  (void)na;
  (void)nc;
}

}  // namespace

// ===========================================================================
// C ABI
// ===========================================================================
#define ABI_GUARD(...)                                                       \
  try {                                                                      \
    __VA_ARGS__                                                              \
  } catch (const DevError& ex) {                                             \
    g_last_error = ex.what();                                                \
    return ex.code;                                                          \
  } catch (const std::exception& ex) {                                       \
    g_last_error = ex.what();                                                \
    return CASPT2_E_DEVICE;                                                  \
  }


// ---------------------------------------------------------------------------
// Correlated density matrices (Sec. II.D) for the target state P of the
// stored lambda.  With the mixed states |P> = sum_M |M~> R_MP and
// T_PN = sum_M T_MN R_MP:
//   d1_xy   = sum_M <M~|T_PM^+ E_xy|P> + sum_MN <M~|lambda_NM^+ E_xy|N~>
//   D1_xyzw = the same with E_xy,zw = E_xy E_zw - delta_yz E_xw
//   dbar2_xy = sum_LMN <M~|lambda_LM^+ E_xy T_LN|N~>,  N_L = <lambda_L|T_L>
//   d2 = dbar2 - sum_L N_L <L~|E|L~> on the active block, dbar2 elsewhere.
// Each is the derivative of a matrix element the amplitude equation already
// evaluates with respect to its coefficient: d1 and D1 run the source terms
// transposed (weights W_N = sum_L R_LP R_NP T_L + lambda_N in place of the
// integrals); dbar2 runs the operator's f-dependence transposed: the row
// energies (diagonal of the closed and virtual blocks of f, with N_L), the
// active Fock metric (Gram tensors with the active E_xy explicit, contracted
// with sum_rows lambda^T T) and the coupling terms of every other block of f
// (also those whose f values vanish).
// D1 holds the classes of the two-body part of H that acts on the
// references (creators active or virtual, annihilators active or closed, not
// all active), [p][q][r][s] per class, classes in a fixed order.
// ---------------------------------------------------------------------------
struct D2Class {
  char sp[4];
  int64_t offset, size;
};

std::vector<D2Class> d2_classes(const H& h) {
  auto dim = [&](char c) -> int64_t { return c == CLO ? h.nc : c == ACT ? h.na : h.nv; };
  std::vector<D2Class> out;
  int64_t off = 0;
  for (const auto& c : source_comps()) {
    if (c.labels.size() != 4) continue;
    D2Class k{};
    int64_t n = 1;
    for (int a = 0; a < 4; ++a) {
      k.sp[a] = c.spaces[a];
      n *= dim(c.spaces[a]);
    }
    k.offset = off;
    k.size = n;
    off += n;
    out.push_back(k);
  }
  return out;
}

// The transposed form of a coupling term of f within one orbital space whose
// one summed label z replaces bra slot sb (every other bra slot feeding one
// ket slot, the active label absent): gf[e][z] += sum_{p, q} L[p][e][q]
// X[p][z][q], L = lambda_all G in bra order and X the ket read with its slots
// in bra order.  Both are copied with slot sb outermost, [D][R], and
// multiplied in one MFMA GEMM (K = R); the result is added into gf at the
// term's block of f (transposed when f's first index is the summed one),
// diagonal left out.  False when the term is not of this form.
bool slot_grad(H& h, const CoupleTerm& t, int64_t nak, const double* Lb, const double* Xk, double* gf,
               int64_t nmo, int skip, DBuf& ta, DBuf& tb, DBuf& tg) {
  const CoupleDesc& d = t.d;
  if (t.up || t.bra != t.ket || d.nsum != 1 || d.ny != 1 || d.bra.nslot != d.ket.nslot) return false;
  const int ns = d.bra.nslot;
  int sb = -1;
  bool z_first;
  if (d.fx_src >= 0 && d.fy_src == -1) {
    sb = d.fx_src;
    z_first = false;
  } else if (d.fy_src >= 0 && d.fx_src == -1) {
    sb = d.fy_src;
    z_first = true;
  } else {
    return false;
  }
  int fed[4] = {0, 0, 0, 0}, lz = -1;
  for (int l = 0; l < ns; ++l) {
    if (d.ket_src[l] == -1) {
      if (lz >= 0) return false;
      lz = l;
    } else if (d.ket_src[l] >= 0 && d.ket_src[l] < ns && d.ket_src[l] != sb) {
      if (fed[d.ket_src[l]]++) return false;
    } else {
      return false;
    }
  }
  if (lz < 0 || d.ket.slot_dim[lz] != d.bra.slot_dim[sb]) return false;
  const int64_t D = d.bra.slot_dim[sb];
  // strides of [D][other bra slots in order][alpha]
  int64_t st[4] = {0, 0, 0, 0}, R = nak;
  for (int k = ns - 1; k >= 0; --k) {
    if (k == sb) continue;
    st[k] = R;
    R *= d.bra.slot_dim[k];
  }
  st[sb] = R;
  const int64_t n = D * R;
  if (ta.n < n) ta.alloc(n);
  if (tb.n < n) tb.alloc(n);
  if (tg.n < D * D) tg.alloc(D * D);
  int64_t dims[5], dst[5];
  for (int k = 0; k < ns; ++k) {
    dims[k] = d.bra.slot_dim[k];
    dst[k] = st[k];
  }
  dims[ns] = nak;
  dst[ns] = 1;
  HIPCHECK(permute_copy(ns + 1, dims, dst, Lb, ta.p, h.s));
  for (int l = 0; l < ns; ++l) {
    dims[l] = d.ket.slot_dim[l];
    dst[l] = l == lz ? st[sb] : st[d.ket_src[l]];
  }
  HIPCHECK(permute_copy(ns + 1, dims, dst, Xk, tb.p, h.s));
  // split K over nb chunks (batched GEMM into partial products, the ragged
  // rest into one more), then one GEMM with a row of ones adds the partials
  const int64_t tiles = ((D + 63) / 64) * ((D + 63) / 64);
  int64_t nb = std::max<int64_t>(1, std::min<int64_t>((1024 + tiles - 1) / tiles, R / 4096));
  nb = std::min<int64_t>(nb, 65535);
  const int64_t kc = R / nb, krest = R - nb * kc;
  const int64_t nparts = nb + (krest > 0 ? 1 : 0);
  DBuf parts(nparts * D * D), ones(nparts);
  HIPCHECK(vec_fill(nparts, 1.0, ones.p, h.s));
  HIPCHECK(gemm_f64(true, D, D, kc, 1.0, ta.p, R, kc, tb.p, R, kc, 0.0, parts.p, D, D * D, (int)nb, h.s));
  if (krest > 0)
    HIPCHECK(gemm_f64(true, D, D, krest, 1.0, ta.p + nb * kc, R, 0, tb.p + nb * kc, R, 0, 0.0,
                      parts.p + nb * D * D, D, 0, 1, h.s));
  HIPCHECK(gemm_f64(false, 1, D * D, nparts, 1.0, ones.p, nparts, 0, parts.p, D * D, 0, 0.0, tg.p, D * D, 0, 1,
                    h.s));
  HIPCHECK(add_block((int)D, tg.p, gf + t.f_off, nmo, z_first ? 1 : 0, skip, h.s));
  return true;
}

void compute_densities(H& h, DBuf& d1, DBuf& D1, DBuf& gf, DBuf& d2, DBuf& NLd) {
  const bool ss = h.d.scheme == CASPT2_SSSR;
  const int nst = h.nst, nmo = h.nmo;
  const int nsets = ss ? nst : 1;
  const int P = h.lam_target;
  auto off = [&](char c) { return c == CLO ? 0 : c == ACT ? h.nc : h.nc + h.na; };
  auto dim = [&](char c) { return c == CLO ? h.nc : c == ACT ? h.na : h.nv; };
  auto Rm = [&](int a, int b) { return h.R[(size_t)a * nst + b]; };
  // ---- weights of the source terms: W[set] = [N][length] ----------------
  std::vector<DBuf> W(nsets);
  for (int set = 0; set < nsets; ++set) {
    W[set].alloc((int64_t)nst * h.length);
    W[set].zero(h.s);
  }
  for (int L = 0; L < nst; ++L) {
    const int set = set_of(h, L);
    for (int N = 0; N < nst; ++N)
      HIPCHECK(vec_axpy(h.length, Rm(L, P) * Rm(N, P), h.T[L].p, W[set].p + (int64_t)N * h.length, h.s));
    HIPCHECK(vec_axpy(h.length, 1.0, h.lam[L].p, W[set].p + (int64_t)L * h.length, h.s));
  }
  // ---- d1, D1: source terms transposed ------------------------------------
  const auto classes = d2_classes(h);
  int64_t d2len = 0;
  for (const auto& k : classes) d2len += k.size;
  d1.alloc((int64_t)nmo * nmo);
  d1.zero(h.s);
  D1.alloc(d2len);
  D1.zero(h.s);
  int nonebody = 0;
  for (const auto& c : source_comps())
    if (c.labels.size() == 2) ++nonebody;
  for_source_terms(h, [&](int ci, const SrcComp& c, TermDesc d, const double*, const double* G, int set,
                          const Entry& e) {
    double* out = c.labels.size() == 2 ? d1.p + (int64_t)off(c.spaces[0]) * nmo + off(c.spaces[1])
                                       : D1.p + classes[ci - nonebody].offset;
    d.scale = 1.0;
    HIPCHECK(term_density(d, out, G, W[set].p + e.offset, h.length, nst, h.s));
  });
  W.clear();
  progress(h, "densities: d1, D1 from the source terms");
  // ---- dbar2: row energies (closed and virtual diagonal) and N_L ----------
  gf.alloc((int64_t)nmo * nmo);
  gf.zero(h.s);
  NLd.alloc(nst);
  NLd.zero(h.s);
  {
    int64_t ymax = 0;
    for (auto& es : h.sets)
      for (auto& e : es) ymax = std::max(ymax, e.nrow * e.nalpha);
    DBuf Y(ymax);
    for (int L = 0; L < nst; ++L)
      for (auto& e : h.sets[set_of(h, L)]) {
        if (e.nrow == 0 || e.nalpha == 0) continue;
        const Block& b = blocks()[e.block];
        HIPCHECK(gemm_f64(false, e.nrow, e.nalpha, e.nalpha, 1.0, h.lam[L].p + e.offset, e.nalpha, 0, e.S.p,
                          e.nalpha, 0, 0.0, Y.p, e.nalpha, 0, 1, h.s));
        int mask = 0;
        for (size_t k = 0; k < b.ext.size(); ++k)
          if (b.ext[k].second == VIR) mask |= 1 << k;
        HIPCHECK(row_metric(base_desc(h, b, e), Y.p, h.T[L].p + e.offset, mask, h.nc + h.na, nmo, gf.p, nmo,
                            NLd.p + L, h.s));
      }
    host_sync(h);
  }
  progress(h, "densities: row energies, N_L");
  // ---- dbar2: active block through the Gram tensors with E_xy explicit ----
  if (h.na > 0) {
    const OpString fop = E("x_o", ACT, "y_o", ACT, "so");
    const int64_t na2 = (int64_t)h.na * h.na;
    DBuf part(1024), dxy(na2);
    for (int bi = 0; bi < NBLOCK; ++bi) {
      const Block& b = blocks()[bi];
      const int ntypes = (int)b.types.size();
      const int64_t ntup = ipow(h.na, (int)b.act.size());
      const int64_t nall = (int64_t)nst * ntypes * ntup;
      const int64_t nset = (ss ? 1 : nst) * ntypes * ntup;
      bool any = false;
      for (auto& e : h.sets[0])
        if (e.block == bi && e.nrow > 0) any = true;
      if (nset == 0 || !any) continue;
      std::map<std::string, PairAcc> fk;
      for (int tb = 0; tb < ntypes; ++tb)
        for (int tk = 0; tk < ntypes; ++tk) {
          auto pairings = matrix_element(suffixed(b.types[tb], "_b"), fop, suffixed(b.types[tk], "_k"));
          for (auto& Pr : pairings) {
            const std::string key = pair_key(Pr);
            auto it = fk.find(key);
            if (it == fk.end()) {
              PairAcc pa;
              pa.P.pairs = Pr.pairs;
              pa.G.alloc(na2 * nall * nall);
              pa.G.zero(h.s);
              it = fk.emplace(key, std::move(pa)).first;
            }
            for (const auto& w : Pr.entries)
              accumulate_gram(h, w, tb, ntypes, ntup, tk, ntypes, ntup, false, nullptr, it->second.G, 0);
          }
        }
      h.vcache.clear();
      // Q_chi = sum_L lambda_L^T T_L over the rows of each entry
      std::vector<DBuf> Q;
      std::vector<const Entry*> ents;
      std::vector<int> eset;
      for (int set = 0; set < nsets; ++set)
        for (auto& e : h.sets[set]) {
          if (e.block != bi || e.nrow == 0) continue;
          Q.emplace_back(nset * nset);
          Q.back().zero(h.s);
          ents.push_back(&e);
          eset.push_back(set);
          for (int L = 0; L < nst; ++L)
            if (set_of(h, L) == set)
              HIPCHECK(outer_rows(e.nrow, nset, nset, h.lam[L].p + e.offset, h.T[L].p + e.offset,
                                  Q.back().p, h.s));
        }
      DBuf Qsum(nall * nall);
      for (auto& kv : fk) {
        Qsum.zero(h.s);
        for (size_t k = 0; k < ents.size(); ++k) {
          const double sg = perm_sign(b, kv.second.P, ents[k]->chi);
          if (ss) {
            const int64_t dims2[2] = {nset, nset};
            const int64_t str2[2] = {nall, 1};
            HIPCHECK(permute_axpy(2, dims2, str2, sg, Q[k].p,
                                  Qsum.p + (int64_t)eset[k] * nset * nall + (int64_t)eset[k] * nset, h.s));
          } else {
            HIPCHECK(vec_axpy(nall * nall, sg, Q[k].p, Qsum.p, h.s));
          }
        }
        // d[x][y] = sum_{alpha beta} G[x][y][alpha][beta] Qsum[alpha][beta]
        for (int64_t xy = 0; xy < na2; ++xy)
          HIPCHECK(vec_dot(nall * nall, kv.second.G.p + xy * nall * nall, (const double*)Qsum.p, part.p,
                           dxy.p + xy, h.s));
        const int64_t dims2[2] = {h.na, h.na};
        const int64_t str2[2] = {nmo, 1};
        HIPCHECK(permute_axpy(2, dims2, str2, 1.0, dxy.p, gf.p + (int64_t)h.nc * nmo + h.nc, h.s));
        host_sync(h);
      }
    }
  }
  progress(h, "densities: active block");
  // ---- dbar2: every other block of f through the coupling terms -----------
  {
    std::vector<std::pair<char, char>> comps;
    for (auto pr : std::vector<std::pair<char, char>>{{ACT, CLO}, {CLO, ACT}, {VIR, ACT}, {ACT, VIR},
                                                      {VIR, CLO}, {CLO, VIR}, {CLO, CLO}, {VIR, VIR}})
      if (dim(pr.first) > 0 && dim(pr.second) > 0 && !(pr.first == pr.second && dim(pr.first) < 2))
        comps.push_back(pr);
    std::vector<std::vector<CoupleTerm>> terms;
    bool used[NBLOCK] = {false, false, false, false, false, false, false, false};
    make_coupling_terms(h, comps, terms, used);
    std::vector<DBuf> lall(NBLOCK), tall(NBLOCK);
    int64_t scr = 0;
    for (int b = 0; b < NBLOCK; ++b)
      if (used[b]) {
        const int64_t na_b = nalpha_of_block(h, 0, b);
        lall[b].alloc(all_rows(h, b) * na_b);
        tall[b].alloc(all_rows(h, b) * na_b);
      }
    for (auto& ts : terms)
      for (auto& t : ts)
        scr = std::max(scr, (t.up ? all_rows(h, t.ket) : all_rows(h, t.bra)) * t.d.ny * t.d.ncol);
    DBuf scratch(scr);
    // permuted copies and the f-block product of the slot-GEMM form
    DBuf slot_a, slot_b, slot_g;
    for (int L = 0; L < nst; ++L) {
      const int set = set_of(h, L);
      for (int b = 0; b < NBLOCK; ++b)
        if (used[b]) {
          const int64_t na_b = nalpha_of_block(h, set, b);
          HIPCHECK(unpack_all(pack_info(h, set, b, nullptr, nullptr, na_b), all_desc(h, b),
                              (const double*)h.lam[L].p, lall[b].p, h.s));
          HIPCHECK(unpack_all(pack_info(h, set, b, nullptr, nullptr, na_b), all_desc(h, b),
                              (const double*)h.T[L].p, tall[b].p, h.s));
        }
      for (auto& t : terms[set]) {
        const int64_t nab = nalpha_of_block(h, set, t.bra), nak = nalpha_of_block(h, set, t.ket);
        const int skip = t.bra == t.ket ? 1 : 0;   // f within one orbital space: diagonal from the row energies
        if (t.up) {
          const int64_t width = (int64_t)t.d.ny * nab;
          HIPCHECK(gemm_f64(true, all_rows(h, t.ket), width, nak, 1.0, tall[t.ket].p, nak, 0, t.G.p, nak, 0, 0.0,
                            scratch.p, width, 0, 1, h.s));
          HIPCHECK(fock_grad(t.d, lall[t.bra].p, nab, 0, scratch.p, width, nab, nab, gf.p + t.f_off, nmo, skip,
                             h.s));
        } else {
          const int64_t width = (int64_t)t.d.ny * nak;
          HIPCHECK(gemm_f64(false, all_rows(h, t.bra), width, nab, 1.0, lall[t.bra].p, nab, 0, t.G.p, width, 0,
                            0.0, scratch.p, width, 0, 1, h.s));
          if (!slot_grad(h, t, nak, scratch.p, tall[t.ket].p, gf.p, nmo, skip, slot_a, slot_b, slot_g))
            HIPCHECK(fock_grad(t.d, scratch.p, width, nak, tall[t.ket].p, nak, 0, nak, gf.p + t.f_off, nmo, skip,
                               h.s));
        }
      }
      host_sync(h);
    }
  }
  progress(h, "densities: coupling terms");
  // ---- <L~|E_rs|L~> and the finished dbar2, d2 ----------------------------
  DBuf gam((int64_t)nst * h.na * h.na);
  gam.zero(h.s);
  if (h.na > 0)
    for (int spin = 0; spin < 2; ++spin) {
      const auto* v = apply_string(h, ActString{ActOp{'a', "r", spin}});
      if (!v) continue;
      const int64_t dimv = h.as->dim(v->second);
      for (int L = 0; L < nst; ++L)
        HIPCHECK(gemm_f64(true, h.na, h.na, dimv, 1.0, v->first.p + (int64_t)L * dimv, (int64_t)nst * dimv, 0,
                          v->first.p + (int64_t)L * dimv, (int64_t)nst * dimv, 0, 1.0,
                          gam.p + (int64_t)L * h.na * h.na, h.na, 0, 1, h.s));
    }
  h.vcache.clear();
  d2.alloc((int64_t)nmo * nmo);
  HIPCHECK(density_finish(nmo, h.nc, h.na, nst, NLd.p, gam.p, gf.p, d2.p, h.s));
  host_sync(h);
}

extern "C" {

const char* caspt2_last_error(void) { return g_last_error.c_str(); }

const char* caspt2_strerror(int code) {
  switch (code) {
    case CASPT2_OK: return "ok";
    case CASPT2_E_ARG: return "invalid argument";
    case CASPT2_E_NOMEM: return "device out of memory";
    case CASPT2_E_DEVICE: return "HIP device error";
    case CASPT2_E_NOCONV: return "not converged";
    case CASPT2_E_INDEFINITE: return "operator not positive definite";
    case CASPT2_E_NOTIMPL: return "not implemented";
    case CASPT2_E_STATE: return "call out of order";
    default: return "unknown status";
  }
}

int caspt2_create(const caspt2_dims* dims, const caspt2_inputs* in, int on_device, void* stream,
                  caspt2_handle** out) {
  if (!dims || !in || !out) return CASPT2_E_ARG;
  *out = nullptr;
  std::unique_ptr<caspt2_handle> hp(new caspt2_handle());
  H& h = *hp;
  ABI_GUARD({
    BlockCacheScope cache;   // temporaries of this creation reuse each other's blocks
    h.d = *dims;
    h.s = (hipStream_t)stream;
    h.verbose = std::getenv("CASPT2_VERBOSE") != nullptr;
    h.verbose_level = h.verbose ? std::atoi(std::getenv("CASPT2_VERBOSE")) : 0;
    h.t_start = wall();
    h.nc = dims->nclosed;
    h.na = dims->nact;
    h.nv = dims->nvirt;
    h.naux = dims->naux;
    h.nst = dims->nstates;
    h.nmo = h.nc + h.na + h.nv;
    if (h.nc < 0 || h.na < 0 || h.nv < 0 || h.naux <= 0 || h.nst <= 0 || h.nst > 16 ||
        h.nmo <= 0 || dims->nelec < 0 || dims->nelec > 2 * h.na ||
        (dims->scheme != CASPT2_MSMR && dims->scheme != CASPT2_SSSR) ||
        (dims->precision != CASPT2_FP64 && dims->precision != CASPT2_MIXED) || !(dims->ovl_thresh > 0.0) || !std::isfinite(dims->shift))
      throw DevError(CASPT2_E_ARG, "bad dimensions");
    if (!in->fock || !in->hcore || !in->dfB || !in->ci || !in->eref)
      throw DevError(CASPT2_E_ARG, "null input");
    h.as = std::make_unique<ActiveSpace>(h.na);
    h.sec0 = Sector{(dims->nelec + 1) / 2, dims->nelec / 2};
    h.ndet = h.as->dim(h.sec0);
    if (h.nst > h.ndet) throw DevError(CASPT2_E_ARG, "more states than determinants");
    const int64_t n2 = (int64_t)h.nmo * h.nmo;
    const hipMemcpyKind kind = on_device ? hipMemcpyDeviceToHost : hipMemcpyHostToHost;
    h.h_fock.resize(n2);
    std::vector<double> hc(n2);
    h.eref.resize(h.nst);
    HIPCHECK(hipMemcpy(h.h_fock.data(), in->fock, n2 * sizeof(double), kind));
    HIPCHECK(hipMemcpy(hc.data(), in->hcore, n2 * sizeof(double), kind));
    HIPCHECK(hipMemcpy(h.eref.data(), in->eref, h.nst * sizeof(double), kind));
    validate(dims, h.h_fock, hc, h.nmo, h.nc, h.na);
    for (double v : h.eref)
      if (!std::isfinite(v)) throw DevError(CASPT2_E_ARG, "non-finite eref");
    // the diagonal of f enters through the row energies; the coupling terms
    // read the device copy, whose closed and virtual diagonals are zero
    h.h_eps.resize(h.nmo);
    for (int i = 0; i < h.nmo; ++i) h.h_eps[i] = h.h_fock[i * h.nmo + i];
    std::vector<double> fdev(h.h_fock);
    for (int i = 0; i < h.nmo; ++i)
      if (i < h.nc || i >= h.nc + h.na) fdev[(size_t)i * h.nmo + i] = 0.0;
    // device copies
    const hipMemcpyKind k2 = on_device ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice;
    h.fock.alloc(n2);
    h.hcore.alloc(n2);
    h.B.alloc((int64_t)h.naux * n2);
    h.ci_raw.alloc((int64_t)h.nst * h.ndet);
    h.ci.alloc((int64_t)h.nst * h.ndet);
    HIPCHECK(hipMemcpyAsync(h.fock.p, fdev.data(), n2 * sizeof(double), hipMemcpyHostToDevice, h.s));
    HIPCHECK(hipMemcpyAsync(h.hcore.p, hc.data(), n2 * sizeof(double), hipMemcpyHostToDevice, h.s));
    HIPCHECK(hipMemcpyAsync(h.B.p, in->dfB, (size_t)h.naux * n2 * sizeof(double), k2, h.s));
    HIPCHECK(hipMemcpyAsync(h.ci_raw.p, in->ci, (size_t)h.nst * h.ndet * sizeof(double), k2, h.s));
    h.red_partial.alloc(1024);
    h.red_out.alloc(4);
    // ---- XMS (Eqs. 3-5): F^ref_MN = <M| f_act |N> -------------------------
    const int nst = h.nst;
    DBuf fact((int64_t)h.na * h.na), W((int64_t)nst * h.ndet), W2((int64_t)nst * h.ndet), Fr(nst * nst);
    {
      std::vector<double> fa((size_t)h.na * h.na);
      for (int r = 0; r < h.na; ++r)
        for (int s2 = 0; s2 < h.na; ++s2) fa[r * h.na + s2] = h.h_fock[(h.nc + r) * h.nmo + h.nc + s2];
      if (!fa.empty())
        HIPCHECK(hipMemcpyAsync(fact.p, fa.data(), fa.size() * sizeof(double), hipMemcpyHostToDevice, h.s));
    }
    if (h.na > 0) {
      apply_onebody(h, fact.p, 0, h.ci_raw.p, nst, h.sec0, W.p);
      apply_onebody(h, fact.p, 1, h.ci_raw.p, nst, h.sec0, W2.p);
      HIPCHECK(vec_axpy((int64_t)nst * h.ndet, 1.0, W2.p, W.p, h.s));
      HIPCHECK(gemm_f64(true, nst, nst, h.ndet, 1.0, h.ci_raw.p, h.ndet, 0, W.p, h.ndet, 0, 0.0,
                        Fr.p, nst, 0, 1, h.s));
    } else {
      Fr.zero(h.s);
    }
    h.fref.resize(nst * nst);
    d2h(h, h.fref.data(), Fr.p, nst * nst * sizeof(double), h.s);
    DBuf wv(nst), Ud(nst * nst);
    h.U.assign(nst * nst, 0.0);
    h.e0.assign(nst, 0.0);
    if (dims->xms) {
      HIPCHECK(small_eigh(nst, Fr.p, wv.p, Ud.p, h.s));
      d2h(h, h.U.data(), Ud.p, nst * nst * sizeof(double), h.s);
      d2h(h, h.e0.data(), wv.p, nst * sizeof(double), h.s);
    } else {
      for (int k = 0; k < nst; ++k) {
        h.U[k * nst + k] = 1.0;
        h.e0[k] = h.fref[k * nst + k];
      }
      HIPCHECK(hipMemcpyAsync(Ud.p, h.U.data(), nst * nst * sizeof(double), hipMemcpyHostToDevice, h.s));
    }
    // rotated CI: ci[M] = sum_N U[N][M] ci_raw[N]  ->  C = U^T ci_raw
    {
      DBuf Ut(nst * nst);
      const int64_t dims2[2] = {nst, nst};
      const int64_t str2[2] = {1, nst};
      Ut.zero(h.s);
      HIPCHECK(permute_axpy(2, dims2, str2, 1.0, Ud.p, Ut.p, h.s));
      HIPCHECK(gemm_f64(false, nst, h.ndet, nst, 1.0, Ut.p, nst, 0, h.ci_raw.p, h.ndet, 0, 0.0,
                        h.ci.p, h.ndet, 0, 1, h.s));
      // H^ref = U^T diag(eref) U
      DBuf Er(nst * nst), T1(nst * nst), Hr(nst * nst);
      std::vector<double> ed(nst * nst, 0.0);
      for (int k = 0; k < nst; ++k) ed[k * nst + k] = h.eref[k];
      HIPCHECK(hipMemcpyAsync(Er.p, ed.data(), nst * nst * sizeof(double), hipMemcpyHostToDevice, h.s));
      HIPCHECK(gemm_f64(false, nst, nst, nst, 1.0, Er.p, nst, 0, Ud.p, nst, 0, 0.0, T1.p, nst, 0, 1, h.s));
      HIPCHECK(gemm_f64(false, nst, nst, nst, 1.0, Ut.p, nst, 0, T1.p, nst, 0, 0.0, Hr.p, nst, 0, 1, h.s));
      h.href.resize(nst * nst);
      d2h(h, h.href.data(), Hr.p, nst * nst * sizeof(double), h.s);
    }
    h.vcache.clear();
    progress(h, "XMS rotation");
    // ---- blocks, orthonormal bases, sources ------------------------------
    setup_blocks(h);
    setup_sources(h);
    setup_couplings(h);
    if (dims->precision == CASPT2_MIXED) setup_mixed(h);
    h.eri.clear();
    host_sync(h);
    *out = hp.release();
    return CASPT2_OK;
  })
}

int caspt2_create_many(int32_t n, const caspt2_dims* dims, const caspt2_inputs* inputs, int inputs_on_device,
                       void* const* streams, int32_t nthreads, caspt2_handle** out, int32_t* status) {
  if (n < 1 || nthreads < 1 || !dims || !inputs || !streams || !out || !status) return CASPT2_E_ARG;
  for (int k = 0; k < n; ++k) {
    out[k] = nullptr;
    status[k] = CASPT2_E_STATE;
  }
  ABI_GUARD({
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return CASPT2_E_DEVICE;
    std::atomic<int> next(0);
    std::vector<std::string> msg(n);
    auto worker = [&]() {
      if (hipSetDevice(dev) != hipSuccess) return;   // a new thread starts on device 0
      try {
        for (int k; (k = next.fetch_add(1)) < n;) {
          status[k] = caspt2_create(&dims[k], &inputs[k], inputs_on_device, streams[k], &out[k]);
          if (status[k] != CASPT2_OK) msg[k] = g_last_error;
        }
      } catch (...) {   // a message that cannot be copied: the status stays
      }
    };
    std::vector<std::thread> pool;
    const int nt = std::min(nthreads, n);
    try {
      for (int t = 0; t < nt; ++t) pool.emplace_back(worker);
    } catch (const std::exception& ex) {   // fewer threads than asked: the started ones take every problem
      if (pool.empty()) {
        g_last_error = ex.what();
        return CASPT2_E_DEVICE;
      }
    }
    for (auto& t : pool) t.join();
    for (int k = 0; k < n; ++k)
      if (status[k] != CASPT2_OK) {
        g_last_error = msg[k].empty() ? "problem " + std::to_string(k) + " not created" : msg[k];
        return status[k];
      }
    return CASPT2_OK;
  })
}

int caspt2_destroy(caspt2_handle* h) {
  if (h) {
    for (auto& r : h->prof_events) {
      (void)hipEventDestroy(r.a);
      (void)hipEventDestroy(r.b);
    }
    for (int l = 0; l < 2; ++l) {
      if (h->slane[l]) {
        (void)hipStreamSynchronize(h->slane[l]);
        (void)hipStreamDestroy(h->slane[l]);
      }
      if (h->slane_done[l]) (void)hipEventDestroy(h->slane_done[l]);
    }
    if (h->sfork) (void)hipEventDestroy(h->sfork);
  }
  delete h;
  return CASPT2_OK;
}

int caspt2_set_precision(caspt2_handle* h, int32_t precision) {
  if (!h || (precision != CASPT2_FP64 && precision != CASPT2_MIXED)) return CASPT2_E_ARG;
  ABI_GUARD({
    if (precision == CASPT2_MIXED) {
      setup_mixed(*h);
      host_sync(*h);
    }
    h->d.precision = precision;
    return CASPT2_OK;
  })
}

int caspt2_set_streams(caspt2_handle* h, int32_t n) {
  if (!h || n < 1 || n > 2) return CASPT2_E_ARG;
  h->residual_streams = n;
  return CASPT2_OK;
}

int caspt2_autotune(caspt2_handle* h, const char* cache_path, int32_t force) {
  if (!h) return CASPT2_E_ARG;
  ABI_GUARD({
    autotune(*h, cache_path, force != 0);
    host_sync(*h);
    return CASPT2_OK;
  })
}

int caspt2_tune_entry(const caspt2_handle* h, int32_t k, int32_t* choice, double* rule_ms, double* tuned_ms) {
  if (!h || k < 0 || k >= (int32_t)h->sets[0].size()) return CASPT2_E_ARG;
  const Entry& e = h->sets[0][k];
  if (choice) {
    choice[0] = e.tune.splitk;
    choice[1] = e.tune.order;
    choice[2] = (int32_t)e.tune.grid;
    choice[3] = e.tune.tile;
    choice[4] = e.tune.kb;
    choice[5] = e.tune.occ;
    choice[6] = e.tune.plain;
    choice[7] = e.tune.breg;
  }
  if (rule_ms) *rule_ms = e.tune_rule_ms;
  if (tuned_ms) *tuned_ms = e.tune_best_ms;
  return CASPT2_OK;
}

int caspt2_profile(caspt2_handle* h, int32_t enable) {
  if (!h) return CASPT2_E_ARG;
  ABI_GUARD({
    HIPCHECK(hipStreamSynchronize(h->s));
    for (auto& r : h->prof_events) {
      (void)hipEventDestroy(r.a);
      (void)hipEventDestroy(r.b);
    }
    h->prof_events.clear();
    h->prof_on = enable != 0;
    return CASPT2_OK;
  })
}

int caspt2_profile_entry(caspt2_handle* h, int32_t k, double* avg_ms, int64_t* launches,
                         double* bytes_per_launch) {
  if (!h || k < 0 || k > (int32_t)h->sets[0].size() + 3) return CASPT2_E_ARG;
  ABI_GUARD({
    HIPCHECK(hipStreamSynchronize(h->s));
    double tot = 0.0, bytes = 0.0;
    int64_t n = 0;
    for (auto& r : h->prof_events) {
      if (r.entry != k) continue;
      float ms = 0.f;
      HIPCHECK(hipEventElapsedTime(&ms, r.a, r.b));
      tot += ms;
      bytes += r.bytes;
      ++n;
    }
    if (avg_ms) *avg_ms = n ? tot / n : 0.0;
    if (launches) *launches = n;
    if (bytes_per_launch) *bytes_per_launch = n ? bytes / n : 0.0;
    return CASPT2_OK;
  })
}

int caspt2_profile_stage(caspt2_handle* h, int32_t k, char* name, int32_t name_len, double* ms_per_residual,
                         int64_t* residuals) {
  if (!h || k < 0) return CASPT2_E_ARG;
  if (k >= (int32_t)h->prof_stage.size()) return CASPT2_E_ARG;
  ABI_GUARD({
    HIPCHECK(hipStreamSynchronize(h->s));
    double tot = 0.0;
    int64_t n = 0, nres = 0;
    for (auto& r : h->prof_events) {
      if (r.entry == (int)h->sets[0].size()) ++nres;   // one per residual with couplings
      if (r.entry != 1000 + k) continue;
      float ms = 0.f;
      HIPCHECK(hipEventElapsedTime(&ms, r.a, r.b));
      tot += ms;
      ++n;
    }
    if (name && name_len > 0) {
      std::snprintf(name, (size_t)name_len, "%s", h->prof_stage[k].c_str());
    }
    if (ms_per_residual) *ms_per_residual = nres ? tot / nres : 0.0;
    if (residuals) *residuals = nres;
    return CASPT2_OK;
  })
}

int64_t caspt2_vector_length(const caspt2_handle* h) { return h ? h->length : -1; }

int caspt2_layout(const caspt2_handle* h, int32_t k, int64_t* offset, int64_t* rows, int64_t* nalpha) {
  if (!h || k < 0 || k >= (int32_t)h->sets[0].size()) return CASPT2_E_ARG;
  const auto& e = h->sets[0][k];
  if (offset) *offset = e.offset;
  if (rows) *rows = e.nrow;
  if (nalpha) *nalpha = e.nalpha;
  return CASPT2_OK;
}

int caspt2_residual(caspt2_handle* h, int32_t L, int32_t with_source, const double* x, double* sigma) {
  if (!h || L < 0 || L >= h->nst || !x || !sigma) return CASPT2_E_ARG;
  ABI_GUARD({
    residual(*h, L, x, sigma, with_source != 0);
    host_sync(*h);
    return CASPT2_OK;
  })
}

int caspt2_residual_all(caspt2_handle* h, int32_t with_source, const double* x, double* sigma) {
  if (!h || !x || !sigma) return CASPT2_E_ARG;
  ABI_GUARD({
    H& hh = *h;
    bool coupled = false;
    for (auto& cs : hh.couple) coupled = coupled || !cs.empty();
    if (hh.residual_streams < 2) {
      for (int L = 0; L < hh.nst; ++L)
        residual(hh, L, x + (int64_t)L * hh.length, sigma + (int64_t)L * hh.length, with_source != 0);
      host_sync(hh);
      return CASPT2_OK;
    }
    // states alternate between two streams; the second runs its entries in
    // reverse order, so MFMA-bound GEMMs of one state overlap the HBM-bound
    // streaming kernels of another, and with couplings the latency-bound
    // coupling kernels of two states overlap (each stream with its own work
    // set).  Results are identical to the one-stream order (each state's
    // launches and workspaces are its stream's own).  (Measured: splitting instead by kind -- all streaming entries on
    // one stream, all GEMM entries on the other -- is no faster at the full
    // size and slower at the mid size.)
    if (!hh.sfork) {
      HIPCHECK(hipEventCreateWithFlags(&hh.sfork, hipEventDisableTiming));
      for (int l = 0; l < 2; ++l) {
        HIPCHECK(hipStreamCreateWithFlags(&hh.slane[l], hipStreamNonBlocking));
        HIPCHECK(hipEventCreateWithFlags(&hh.slane_done[l], hipEventDisableTiming));
      }
    }
    if (hh.splitk_ws2.n != hh.splitk_ws.n) hh.splitk_ws2.alloc(hh.splitk_ws.n);
    if (coupled && hh.nst > 1) ensure_work_set2(hh);   // the second stream's coupling tensors
    const hipStream_t keep = hh.s;
    HIPCHECK(hipEventRecord(hh.sfork, keep));
    for (int l = 0; l < 2; ++l) HIPCHECK(hipStreamWaitEvent(hh.slane[l], hh.sfork, 0));
    try {
      for (int L = 0; L < hh.nst; ++L) {
        const int l = L & 1;
        hh.s = hh.slane[l];
        hh.ws_cur = l ? &hh.splitk_ws2 : &hh.splitk_ws;
        hh.wset = l;
        residual(hh, L, x + (int64_t)L * hh.length, sigma + (int64_t)L * hh.length, with_source != 0, l == 1);
      }
    } catch (...) {
      hh.s = keep;
      hh.ws_cur = nullptr;
      hh.wset = 0;
      throw;
    }
    hh.s = keep;
    hh.ws_cur = nullptr;
    hh.wset = 0;
    for (int l = 0; l < 2; ++l) {
      HIPCHECK(hipEventRecord(hh.slane_done[l], hh.slane[l]));
      HIPCHECK(hipStreamWaitEvent(keep, hh.slane_done[l], 0));
    }
    host_sync(hh);
    return CASPT2_OK;
  })
}

int caspt2_residual_all_many(int32_t n, caspt2_handle* const* handles, int32_t with_source, const double* const* x,
                             double* const* sigma, int32_t nthreads, int32_t* status) {
  if (n < 1 || nthreads < 1 || !handles || !x || !sigma || !status) return CASPT2_E_ARG;
  for (int k = 0; k < n; ++k) {
    if (!handles[k]) return CASPT2_E_ARG;
    for (int j = 0; j < k; ++j)
      if (handles[j] == handles[k]) return CASPT2_E_ARG;
    status[k] = CASPT2_E_STATE;
  }
  ABI_GUARD({
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return CASPT2_E_DEVICE;
    std::atomic<int> next(0);
    std::vector<std::string> msg(n);
    auto worker = [&]() {
      if (hipSetDevice(dev) != hipSuccess) return;
      try {
        for (int k; (k = next.fetch_add(1)) < n;) {
          status[k] = caspt2_residual_all(handles[k], with_source, x[k], sigma[k]);
          if (status[k] != CASPT2_OK) msg[k] = g_last_error;
        }
      } catch (...) {   // a message that cannot be copied: the status stays
      }
    };
    std::vector<std::thread> pool;
    const int nt = std::min(nthreads, n);
    try {
      for (int t = 0; t < nt; ++t) pool.emplace_back(worker);
    } catch (const std::exception& ex) {
      if (pool.empty()) {
        g_last_error = ex.what();
        return CASPT2_E_DEVICE;
      }
    }
    for (auto& t : pool) t.join();
    for (int k = 0; k < n; ++k)
      if (status[k] != CASPT2_OK) {
        g_last_error = msg[k].empty() ? "problem " + std::to_string(k) + " not evaluated" : msg[k];
        return status[k];
      }
    return CASPT2_OK;
  })
}

int caspt2_solve_amplitudes(caspt2_handle* h, double tol, int32_t maxiter, const double* T0,
                            caspt2_info* info) {
  if (!h || !(tol > 0.0) || maxiter < 0) return CASPT2_E_ARG;
  ABI_GUARD({
    H& hh = *h;
    hh.T.clear();
    hh.Tt.clear();
    hh.have_T = hh.have_heff = hh.have_lam = false;
    const int status = grouped_solve(hh, 0, 0, tol, maxiter, hh.T, hh.Tt, hh.tinfo, T0);
    if (status == CASPT2_E_INDEFINITE) return status;
    host_sync(hh);
    hh.have_T = true;
    if (info)
      for (int L = 0; L < hh.nst; ++L) info[L] = hh.tinfo[L];
    return status;
  })
}

int caspt2_get_amplitudes(caspt2_handle* h, int32_t L, double* T) {
  if (!h || L < 0 || L >= h->nst || !T) return CASPT2_E_ARG;
  if (!h->have_T) return CASPT2_E_STATE;
  ABI_GUARD({
    HIPCHECK(hipMemcpyAsync(T, h->T[L].p, h->length * sizeof(double), hipMemcpyDeviceToDevice, h->s));
    host_sync(*h);
    return CASPT2_OK;
  })
}

int caspt2_get_xms(const caspt2_handle* h, double* U, double* e0) {
  if (!h) return CASPT2_E_ARG;
  if (U) std::memcpy(U, h->U.data(), h->nst * h->nst * sizeof(double));
  if (e0) std::memcpy(e0, h->e0.data(), h->nst * sizeof(double));
  return CASPT2_OK;
}

int xms_rotate(int32_t nact, int32_t nst, const double* f_act, const double* rdm1, double* U, double* e0) {
  if (nact < 0 || nst <= 0 || nst > 16 || (nact > 0 && (!f_act || !rdm1)) || !U || !e0) return CASPT2_E_ARG;
  const int64_t nf = (int64_t)nact * nact, ng = (int64_t)nst * nst * nf;
  for (int64_t k = 0; k < nf; ++k)
    if (!std::isfinite(f_act[k])) return CASPT2_E_ARG;
  for (int64_t k = 0; k < ng; ++k)
    if (!std::isfinite(rdm1[k])) return CASPT2_E_ARG;
  ABI_GUARD({
    DBuf fd(nf), gd(ng), Fr((int64_t)nst * nst), wv(nst), Ud((int64_t)nst * nst);
    PinBuf<double> hp;
    hp.ensure((int64_t)nst * nst + nst);
    if (nf > 0) {
      HIPCHECK(hipMemcpy(fd.p, f_act, nf * sizeof(double), hipMemcpyHostToDevice));
      HIPCHECK(hipMemcpy(gd.p, rdm1, ng * sizeof(double), hipMemcpyHostToDevice));
    }
    HIPCHECK(xms_fref(nact, nst, fd.p, gd.p, Fr.p, nullptr));
    HIPCHECK(small_eigh(nst, Fr.p, wv.p, Ud.p, nullptr));
    HIPCHECK(hipMemcpy(hp.p, Ud.p, (size_t)nst * nst * sizeof(double), hipMemcpyDeviceToHost));
    HIPCHECK(hipMemcpy(hp.p + (int64_t)nst * nst, wv.p, nst * sizeof(double), hipMemcpyDeviceToHost));
    std::memcpy(U, hp.p, (size_t)nst * nst * sizeof(double));
    std::memcpy(e0, hp.p + (int64_t)nst * nst, nst * sizeof(double));
    return CASPT2_OK;
  })
}

int64_t caspt2_density2_length(const caspt2_handle* h) {
  if (!h) return -1;
  int64_t n = 0;
  for (const auto& k : d2_classes(*h)) n += k.size;
  return n;
}

int caspt2_density2_layout(const caspt2_handle* h, int32_t k, int64_t* offset, int32_t* spaces) {
  if (!h) return CASPT2_E_ARG;
  const auto cl = d2_classes(*h);
  if (k < 0 || k >= (int32_t)cl.size()) return CASPT2_E_ARG;
  if (offset) *offset = cl[k].offset;
  if (spaces)
    for (int a = 0; a < 4; ++a) spaces[a] = cl[k].sp[a] == CLO ? 0 : cl[k].sp[a] == ACT ? 1 : 2;
  return CASPT2_OK;
}

int caspt2_densities(caspt2_handle* h, double* d1, double* D1, double* dbar2, double* d2, double* NL) {
  if (!h) return CASPT2_E_ARG;
  if (!h->have_lam || !h->have_heff || h->lam_target < 0) return CASPT2_E_STATE;
  ABI_GUARD({
    H& hh = *h;
    DBuf dd1, dD1, dgf, dd2, dNL;
    compute_densities(hh, dd1, dD1, dgf, dd2, dNL);
    const size_t nn = (size_t)hh.nmo * hh.nmo;
    if (d1) d2h(hh, d1, dd1.p, nn * sizeof(double), hh.s);
    if (dbar2) d2h(hh, dbar2, dgf.p, nn * sizeof(double), hh.s);
    if (d2) d2h(hh, d2, dd2.p, nn * sizeof(double), hh.s);
    if (NL) d2h(hh, NL, dNL.p, hh.nst * sizeof(double), hh.s);
    if (D1 && dD1.n > 0)
      HIPCHECK(hipMemcpyAsync(D1, dD1.p, dD1.n * sizeof(double), hipMemcpyDeviceToDevice, hh.s));
    host_sync(hh);
    return CASPT2_OK;
  })
}

int xms_heff(caspt2_handle* h, double* heff, double* e_ms, double* R) {
  if (!h) return CASPT2_E_ARG;
  if (!h->have_T) return CASPT2_E_STATE;
  ABI_GUARD({
    H& hh = *h;
    const int nst = hh.nst;
    compute_heff(hh);
    if (heff) std::memcpy(heff, hh.heff.data(), nst * nst * sizeof(double));
    if (e_ms) std::memcpy(e_ms, hh.ems.data(), nst * sizeof(double));
    if (R) std::memcpy(R, hh.R.data(), nst * nst * sizeof(double));
    return CASPT2_OK;
  })
}

int caspt2_solve_lambda(caspt2_handle* h, int32_t P, double tol, int32_t maxiter, const double* lam0,
                        caspt2_info* info) {
  if (!h || P < 0 || P >= h->nst || !(tol > 0.0) || maxiter < 0) return CASPT2_E_ARG;
  if (!h->have_heff) return CASPT2_E_STATE;
  ABI_GUARD({
    H& hh = *h;
    const int nst = hh.nst;
    hh.lam.clear();
    hh.lamt.clear();
    hh.have_lam = false;
    const int status = grouped_solve(hh, 1, P, tol, maxiter, hh.lam, hh.lamt, hh.linfo, lam0);
    hh.lam_target = P;
    if (status == CASPT2_E_INDEFINITE) return status;
    host_sync(hh);
    hh.have_lam = true;
    if (info)
      for (int L = 0; L < nst; ++L) info[L] = hh.linfo[L];
    return status;
  })
}

int caspt2_batch_solve(caspt2_handle* const* handles, int32_t n, const int32_t* targets, double tol,
                       int32_t maxiter, caspt2_info* amp_info, caspt2_info* lambda_info) {
  if (!handles || n <= 0 || !targets || !(tol > 0.0) || maxiter < 0) return CASPT2_E_ARG;
  for (int i = 0; i < n; ++i) {
    if (!handles[i] || targets[i] < 0 || targets[i] >= handles[i]->nst) return CASPT2_E_ARG;
    if (handles[i]->d.precision != handles[0]->d.precision) return CASPT2_E_ARG;
    for (int j = 0; j < i; ++j)
      if (handles[j] == handles[i]) return CASPT2_E_ARG;
  }
  ABI_GUARD({
    int cap = 0;
    std::vector<int64_t> off(n + 1, 0);
    for (int i = 0; i < n; ++i) {
      cap += 2 * handles[i]->nst;
      off[i + 1] = off[i] + handles[i]->nst;
    }
    // four operator lanes (the hardware queues of a process)
    PcgEngine eng(cap, std::min(n, 4), handles[0]->d.precision == CASPT2_MIXED);
    // phase per problem: 0 amplitudes running, 1 lambda running, 2 done, 3 failed
    std::vector<int> phase(n, 0), result(n, CASPT2_OK);
    std::vector<std::vector<int>> amp(n), lam(n);
    for (int i = 0; i < n; ++i) {
      H& h = *handles[i];
      h.T.clear();
      h.Tt.clear();
      h.lam.clear();
      h.lamt.clear();
      h.tinfo.clear();
      h.linfo.clear();
      h.have_T = h.have_heff = h.have_lam = false;
      for (int L = 0; L < h.nst; ++L) {
        DBuf b(olen(h, set_of(h, L)));
        amplitude_rhs(h, L, b.p);
        host_sync(h);
        amp[i].push_back(eng.add(h, L, 0, b.p, tol, maxiter).id);
      }
    }
    std::vector<int> all;
    for (auto& v : amp) all.insert(all.end(), v.begin(), v.end());
    eng.start(all);
    auto done = [&](const std::vector<int>& ids) {
      for (int id : ids) {
        const int st = eng.sys[id]->status;
        if (st == PCG_RUNNING || st == PCG_IDLE) return false;
      }
      return true;
    };
    auto collect = [&](int i, const std::vector<int>& ids, std::vector<caspt2_info>& infos) {
      int rc = CASPT2_OK;
      infos.assign(handles[i]->nst, caspt2_info{});
      for (int id : ids) {
        PcgSystem& S = *eng.sys[id];
        eng.finish(S);
        infos[S.L] = S.info;
        rc = merge_status(rc, status_code(S.status));
      }
      return rc;
    };
    // interleaving: a problem whose amplitude systems have all stopped gets
    // H_eff and its lambda systems at once, while others still iterate
    eng.run([&](PcgEngine& e) {
      for (int i = 0; i < n; ++i) {
        H& h = *handles[i];
        if (phase[i] == 0 && done(amp[i])) {
          result[i] = collect(i, amp[i], h.tinfo);
          if (result[i] != CASPT2_OK) {
            phase[i] = 3;
            continue;
          }
          h.T.resize(h.nst);
          h.Tt.resize(h.nst);
          for (int id : amp[i]) {
            store_solution(*e.sys[id], h.T, h.Tt);
            e.retire(*e.sys[id]);
          }
          h.have_T = true;
          compute_heff(h);
          for (int L = 0; L < h.nst; ++L) {
            DBuf b(olen(h, set_of(h, L)));
            lambda_rhs(h, L, targets[i], b.p);
            lam[i].push_back(e.add(h, L, 1, b.p, tol, maxiter).id);
          }
          e.start(lam[i]);
          phase[i] = 1;
        }
        if (phase[i] == 1 && done(lam[i])) {
          result[i] = collect(i, lam[i], h.linfo);
          h.lam.resize(h.nst);
          h.lamt.resize(h.nst);
          for (int id : lam[i]) {
            store_solution(*e.sys[id], h.lam, h.lamt);
            e.retire(*e.sys[id]);
          }
          h.have_lam = result[i] == CASPT2_OK;
          h.lam_target = targets[i];
          phase[i] = result[i] == CASPT2_OK ? 2 : 3;
        }
      }
    });
    int status = CASPT2_OK;
    for (int i = 0; i < n; ++i) {
      H& h = *handles[i];
      if (amp_info && !h.tinfo.empty())
        for (int L = 0; L < h.nst; ++L) amp_info[off[i] + L] = h.tinfo[L];
      if (lambda_info && (int)h.linfo.size() == h.nst)
        for (int L = 0; L < h.nst; ++L) lambda_info[off[i] + L] = h.linfo[L];
      status = merge_status(status, result[i]);
    }
    return status;
  })
}

int caspt2_get_lambda(caspt2_handle* h, int32_t L, double* lambda) {
  if (!h || L < 0 || L >= h->nst || !lambda) return CASPT2_E_ARG;
  if (!h->have_lam) return CASPT2_E_STATE;
  ABI_GUARD({
    HIPCHECK(hipMemcpyAsync(lambda, h->lam[L].p, h->length * sizeof(double), hipMemcpyDeviceToDevice,
                            h->s));
    host_sync(*h);
    return CASPT2_OK;
  })
}

}  // extern "C"

#include "../../include/caspt2_debug.h"

extern "C" {

int caspt2_debug_ccvv_passes(int32_t on) {
  const int prev = g_ccvv_passes ? 1 : 0;
  g_ccvv_passes = on != 0;
  return prev;
}

int caspt2_debug_ccvv_passes_used(const caspt2_handle* h, int32_t set) {
  if (!h || set < 0 || set >= (int32_t)h->couple.size()) return CASPT2_E_ARG;
  int r = 0;
  if (set < (int32_t)h->ccvv_fused.size() && h->ccvv_fused[set]) r |= 1;
  if (set < (int32_t)h->ccvv_down_fused.size() && h->ccvv_down_fused[set]) r |= 2;
  if (set < (int32_t)h->cavv_fused.size() && h->cavv_fused[set]) r |= 4;
  return r;
}

int caspt2_debug_gemm(int32_t b_is_nk, int64_t M, int64_t N, int64_t K, const double* A,
                      const double* B, double* C) {
  ABI_GUARD({
    HIPCHECK(gemm_f64(b_is_nk != 0, M, N, K, 1.0, A, K, 0, B, b_is_nk ? K : N, 0, 0.0, C, N, 0, 1,
                      nullptr));
    HIPCHECK(hipStreamSynchronize(nullptr));
    return CASPT2_OK;
  })
}

int caspt2_debug_gemm_f32(int32_t b_is_nk, int64_t M, int64_t N, int64_t K, const float* A,
                          const float* B, float* C) {
  ABI_GUARD({
    HIPCHECK(gemm_f32(b_is_nk != 0, M, N, K, 1.f, A, K, 0, B, b_is_nk ? K : N, 0, 0.f, C, N, 0, 1,
                      nullptr));
    HIPCHECK(hipStreamSynchronize(nullptr));
    return CASPT2_OK;
  })
}

int caspt2_debug_residual_f32(caspt2_handle* h, int32_t L, const float* x, float* sigma) {
  if (!h || L < 0 || L >= h->nst || !x || !sigma) return CASPT2_E_ARG;
  if (!h->have_mixed) return CASPT2_E_STATE;
  ABI_GUARD({
    residual<float>(*h, L, x, sigma, false);
    host_sync(*h);
    return CASPT2_OK;
  })
}

int caspt2_set_verbose(caspt2_handle* h, int32_t level) {
  if (!h || level < 0) return CASPT2_E_ARG;
  h->verbose_level = level;
  h->verbose = level > 0;
  return CASPT2_OK;
}

int caspt2_debug_entry(const caspt2_handle* h, int32_t set, int32_t k, int32_t which, double* out) {
  if (!h || set < 0 || set >= (int32_t)h->sets.size() || k < 0 ||
      k >= (int32_t)h->sets[set].size() || !out)
    return CASPT2_E_ARG;
  ABI_GUARD({
    const auto& e = h->sets[set][k];
    const double* src = nullptr;
    int64_t n = 0;
    switch (which) {
      case 0: src = e.S.p; n = e.S.n; break;
      case 1: src = e.F.p; n = e.F.n; break;
      case 2: src = e.eps.p; n = e.eps.n; break;
      case 3: out[0] = (double)e.nkeep; return CASPT2_OK;
      case 4: src = e.X.p; n = e.X.n; break;
      case 5: src = e.mu.p; n = e.mu.n; break;
      default: return CASPT2_E_ARG;
    }
    if (n > 0) HIPCHECK(hipMemcpy(out, src, n * sizeof(double), hipMemcpyDeviceToHost));
    return CASPT2_OK;
  })
}

int caspt2_debug_source(const caspt2_handle* h, int32_t set, int32_t N, double* out) {
  if (!h || set < 0 || set >= (int32_t)h->src.size() || N < 0 || N >= h->nst || !out)
    return CASPT2_E_ARG;
  ABI_GUARD({
    HIPCHECK(hipMemcpy(out, h->src[set][N].p, h->length * sizeof(double), hipMemcpyDeviceToDevice));
    return CASPT2_OK;
  })
}

int caspt2_debug_eigh(int32_t n, double* A, double* w, double* V) {
  return caspt2_debug_eigh_method(n, A, w, V, 0, nullptr);
}

int caspt2_debug_eigh_method(int32_t n, double* A, double* w, double* V, int32_t method, int32_t* sweeps_out) {
  return caspt2_debug_eigh_abs(n, A, w, V, method, 0.0, sweeps_out);
}

int caspt2_debug_eigh_abs(int32_t n, double* A, double* w, double* V, int32_t method, double abs_tol,
                          int32_t* sweeps_out) {
  if (n <= 0 || !A || !w || !V || method < 0 || method > 5 || !(abs_tol >= 0.0)) return CASPT2_E_ARG;
  if ((method == 1 && n > 64) || (method == 2 && n > 512)) return CASPT2_E_ARG;
  ABI_GUARD({
    double* ws = nullptr;
    const size_t nws = (size_t)jacobi_ws_doubles(n);
    HIPCHECK(hipMalloc(&ws, (nws + (size_t)n * n) * sizeof(double)));
    PinBuf<double> hp;
    hp.ensure(std::max(n, 8));
    int sweeps = 0;
    // method 4: the whole-device form with one launch per step (second
    // buffer); method 0 picks the form by size as the library's set-up does
    const bool second = method == 4;
    hipError_t e = jacobi_eigh(n, A, V, ws, 60, 1e-15, nullptr, &sweeps, method == 4 ? 3 : method,
                               second ? ws + nws : nullptr, hp.p, abs_tol);
    if (sweeps_out) *sweeps_out = sweeps;
    // eigenvalues: the diagonal, one strided copy
    if (e == hipSuccess)
      e = hipMemcpy2D(hp.p, sizeof(double), A, (size_t)(n + 1) * sizeof(double), sizeof(double), (size_t)n,
                      hipMemcpyDeviceToHost);
    (void)hipFree(ws);
    HIPCHECK(e);
    std::memcpy(w, hp.p, (size_t)n * sizeof(double));
    return CASPT2_OK;
  })
}

}  // extern "C"
