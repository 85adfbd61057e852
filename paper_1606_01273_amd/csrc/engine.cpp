// Host-side bookkeeping: blocks of Eq. 8, Wick pairings of external strings,
// active-space determinant tables.  See engine.hpp.
#include "engine.hpp"

#include <algorithm>
#include <cstdlib>
#include <functional>
#include <set>
#include <stdexcept>

namespace caspt2 {

OpString E(const std::string& p, char sp, const std::string& q, char sq, const std::string& spin) {
  return {Op{'c', p, sp, spin}, Op{'a', q, sq, spin}};
}

OpString dagger(const OpString& o) {
  OpString r;
  for (auto it = o.rbegin(); it != o.rend(); ++it)
    r.push_back(Op{it->kind == 'c' ? 'a' : 'c', it->label, it->space, it->spin});
  return r;
}

OpString suffixed(const OpString& o, const std::string& suf) {
  OpString r;
  for (const auto& x : o) r.push_back(Op{x.kind, x.label + suf, x.space, x.spin + suf});
  return r;
}

static OpString cat(OpString a, const OpString& b) {
  a.insert(a.end(), b.begin(), b.end());
  return a;
}

const std::vector<Block>& blocks() {
  static const std::vector<Block> B = [] {
    const std::string s = "s1", t = "s2";
    std::vector<Block> v;
    v.push_back({"ccvv", {{"i", CLO}, {"j", CLO}, {"a", VIR}, {"b", VIR}}, {},
                 {cat(E("a", VIR, "i", CLO, s), E("b", VIR, "j", CLO, t))}, {{0, 1}, {2, 3}}});
    v.push_back({"cavv", {{"i", CLO}, {"a", VIR}, {"b", VIR}}, {"r"},
                 {cat(E("a", VIR, "r", ACT, s), E("b", VIR, "i", CLO, t))}, {{1, 2}}});
    v.push_back({"aavv", {{"a", VIR}, {"b", VIR}}, {"r", "s"},
                 {cat(E("a", VIR, "r", ACT, s), E("b", VIR, "s", ACT, t))}, {{0, 1}}});
    v.push_back({"ccav", {{"i", CLO}, {"j", CLO}, {"a", VIR}}, {"r"},
                 {cat(E("a", VIR, "i", CLO, s), E("r", ACT, "j", CLO, t))}, {{0, 1}}});
    v.push_back({"ccaa", {{"i", CLO}, {"j", CLO}}, {"r", "s"},
                 {cat(E("r", ACT, "i", CLO, s), E("s", ACT, "j", CLO, t))}, {{0, 1}}});
    v.push_back({"aaav", {{"a", VIR}}, {"r", "s", "t"},
                 {cat(E("a", VIR, "r", ACT, s), E("s", ACT, "t", ACT, t))}, {}});
    v.push_back({"caaa", {{"i", CLO}}, {"r", "s", "t"},
                 {cat(E("r", ACT, "i", CLO, s), E("s", ACT, "t", ACT, t))}, {}});
    v.push_back({"caav", {{"i", CLO}, {"a", VIR}}, {"r", "s"},
                 {cat(E("a", VIR, "i", CLO, s), E("r", ACT, "s", ACT, t)),
                  cat(E("a", VIR, "r", ACT, s), E("s", ACT, "i", CLO, t))}, {}});
    return v;
  }();
  return B;
}

std::vector<std::vector<int>> characters(const Block& b) {
  if (b.name == "ccvv") return {{1, 1}, {-1, -1}};
  if (!b.swaps.empty()) return {{1}, {-1}};
  return {{}};
}

// ---------------------------------------------------------------------------
// Wick pairings on the closed-shell core with empty virtuals
// ---------------------------------------------------------------------------

// <core| ops |core> on concrete orbitals: spin orbital 2*orb+spin; closed
// concrete orbitals 0..nclo-1 are doubly occupied.
static double ext_value(const std::vector<Op>& ops, const std::map<std::string, int>& orb,
                        const std::map<std::string, int>& spins, int nclo) {
  uint64_t ref = 0;
  for (int k = 0; k < nclo; ++k) ref |= (uint64_t)3 << (2 * k);
  uint64_t det = ref;
  double coeff = 1.0;
  for (auto it = ops.rbegin(); it != ops.rend(); ++it) {
    const int so = 2 * orb.at(it->label) + spins.at(it->spin);
    const bool occ = (det >> so) & 1;
    const int below = __builtin_popcountll(det & ((uint64_t(1) << so) - 1));
    if (it->kind == 'a') {
      if (!occ) return 0.0;
      det &= ~(uint64_t(1) << so);
    } else {
      if (occ) return 0.0;
      det |= uint64_t(1) << so;
    }
    if (below & 1) coeff = -coeff;
  }
  return det == ref ? coeff : 0.0;
}

std::vector<Pairing> matrix_element(const OpString& bra, const OpString& op, const OpString& ket) {
  OpString Y = cat(cat(dagger(bra), op), ket);
  // stable partition: external operators to the left; sign = (-1)^inversions
  std::vector<Op> ext, actv;
  int inv = 0;
  for (size_t k = 0; k < Y.size(); ++k) {
    if (Y[k].space == ACT) {
      for (size_t e = k + 1; e < Y.size(); ++e)
        if (Y[e].space != ACT) ++inv;
    }
  }
  const double psign = (inv & 1) ? -1.0 : 1.0;
  for (const auto& o : Y) (o.space == ACT ? actv : ext).push_back(o);
  std::vector<std::string> va, vc, cc, ca;
  for (const auto& o : ext) {
    if (o.space == VIR) (o.kind == 'a' ? va : vc).push_back(o.label);
    else (o.kind == 'c' ? cc : ca).push_back(o.label);
  }
  std::vector<Pairing> out;
  if (va.size() != vc.size() || cc.size() != ca.size()) return out;
  // spin variables in order of appearance
  std::vector<std::string> svars;
  for (const auto& o : Y)
    if (std::find(svars.begin(), svars.end(), o.spin) == svars.end()) svars.push_back(o.spin);
  std::vector<size_t> pv(vc.size()), pc(ca.size());
  for (size_t k = 0; k < pv.size(); ++k) pv[k] = k;
  for (size_t k = 0; k < pc.size(); ++k) pc[k] = k;
  do {
    std::vector<size_t> pcc = pc;
    do {
      Pairing P;
      std::map<std::string, int> orb;
      const int nclo = (int)cc.size();
      for (size_t k = 0; k < cc.size(); ++k) {
        P.pairs.push_back({cc[k], ca[pcc[k]]});
        orb[cc[k]] = orb[ca[pcc[k]]] = (int)k;
      }
      for (size_t k = 0; k < va.size(); ++k) {
        P.pairs.push_back({va[k], vc[pv[k]]});
        orb[va[k]] = orb[vc[pv[k]]] = nclo + (int)k;
      }
      const size_t ns = svars.size();
      for (uint32_t m = 0; m < (1u << ns); ++m) {
        std::map<std::string, int> spins;
        for (size_t k = 0; k < ns; ++k) spins[svars[k]] = (m >> k) & 1;
        const double v = ext_value(ext, orb, spins, nclo);
        if (v == 0.0) continue;
        WickEntry w;
        w.coeff = psign * v;
        for (const auto& o : bra)
          if (o.space == ACT) w.bra.push_back({o.kind, o.label, spins[o.spin]});
        for (const auto& o : op)
          if (o.space == ACT) w.mid.push_back({o.kind, o.label, spins[o.spin]});
        for (const auto& o : ket)
          if (o.space == ACT) w.ket.push_back({o.kind, o.label, spins[o.spin]});
        P.entries.push_back(w);
      }
      if (!P.entries.empty()) out.push_back(P);
    } while (std::next_permutation(pcc.begin(), pcc.end()));
  } while (std::next_permutation(pv.begin(), pv.end()));
  return out;
}

// ---------------------------------------------------------------------------
// active space
// ---------------------------------------------------------------------------

std::vector<int64_t> ActiveSpace::strings(int n) const {
  std::vector<int64_t> v;
  if (n < 0 || n > na) return v;
  for (int64_t s = 0; s < (int64_t(1) << na); ++s)
    if (__builtin_popcountll(s) == n) v.push_back(s);
  return v;
}

int64_t ActiveSpace::nstr(int n) const {
  if (n < 0 || n > na) return 0;
  int64_t c = 1;
  for (int k = 0; k < n; ++k) c = c * (na - k) / (k + 1);
  return c;
}

Sector ActiveSpace::target(char kind, int spin, Sector from) const {
  const int d = kind == 'a' ? -1 : 1;
  return spin == 0 ? Sector{from.na_el + d, from.nb_el} : Sector{from.na_el, from.nb_el + d};
}

void ActiveSpace::gather_table(char kind, int spin, Sector from, std::vector<int32_t>& src,
                               std::vector<double>& sign) const {
  const Sector to = target(kind, spin, from);
  const int64_t dto = dim(to);
  src.assign((size_t)na * dto, -1);
  sign.assign((size_t)na * dto, 0.0);
  if (!valid(to) || !valid(from)) return;
  const int nself = spin == 0 ? from.na_el : from.nb_el;
  const auto sfrom = strings(nself);
  const auto sto = strings(spin == 0 ? to.na_el : to.nb_el);
  std::map<int64_t, int64_t> idx_from;
  for (size_t k = 0; k < sfrom.size(); ++k) idx_from[sfrom[k]] = (int64_t)k;
  const int64_t nA_to = nstr(to.na_el), nB_to = nstr(to.nb_el);
  const int64_t nB_from = nstr(from.nb_el);
  for (int r = 0; r < na; ++r) {
    for (size_t kt = 0; kt < sto.size(); ++kt) {
      const int64_t t = sto[kt];
      const bool occ_t = (t >> r) & 1;
      // a_r: source has r occupied, target not; a+_r: the reverse
      if (kind == 'a' ? occ_t : !occ_t) continue;
      const int64_t s = t ^ (int64_t(1) << r);
      const int64_t ks = idx_from.at(s);
      const int below = __builtin_popcountll(s & ((int64_t(1) << r) - 1));
      double sg = (below & 1) ? -1.0 : 1.0;
      if (spin == 1 && (from.na_el & 1)) sg = -sg;  // pass the alpha creators
      if (spin == 0) {
        for (int64_t ib = 0; ib < nB_to; ++ib) {
          const int64_t tdet = (int64_t)kt * nB_to + ib;
          src[(size_t)r * dto + tdet] = (int32_t)(ks * nB_from + ib);
          sign[(size_t)r * dto + tdet] = sg;
        }
      } else {
        for (int64_t ia = 0; ia < nA_to; ++ia) {
          const int64_t tdet = ia * nB_to + (int64_t)kt;
          src[(size_t)r * dto + tdet] = (int32_t)(ia * nB_from + ks);
          sign[(size_t)r * dto + tdet] = sg;
        }
      }
    }
  }
}

// ---------------------------------------------------------------------------
// coupling terms of a block with itself
// ---------------------------------------------------------------------------

// A down term of a block with itself whose one summed label takes the place
// of bra slot sb, the other ket slots being fed one to one by the remaining
// bra slots, and whose Fock element is f(bra slot sb, summed label): it
// applies f along slot sb of the ket tensor read with its slots permuted,
// perm[l] being the bra slot that feeds ket slot l (sb for the summed one).
bool slot_form(const int* ks, int fx, int fy, int nslot, int* sb_out, int* perm) {
  int sb;
  if (fx >= 0 && fy == -1) sb = fx;
  else if (fy >= 0 && fx == -1) sb = fy;
  else return false;
  if (sb >= nslot) return false;
  bool fed[4] = {false, false, false, false};
  int nsum = 0;
  for (int l = 0; l < nslot; ++l) {
    const int v = ks[l];
    if (v == -1) {
      ++nsum;
      perm[l] = sb;
    } else if (v >= 0 && v < nslot && v != sb && !fed[v]) {
      fed[v] = true;
      perm[l] = v;
    } else {
      return false;
    }
  }
  for (int l = nslot; l < 4; ++l) perm[l] = l;
  *sb_out = sb;
  return nsum == 1;
}

// the slot-permuted tensor equals x itself: the identity, or for ccvv the
// joint exchange (i, a) <-> (j, b)
bool perm_trivial(int block, const int* perm, int nslot) {
  bool id = true;
  for (int l = 0; l < nslot; ++l) id = id && perm[l] == l;
  if (id) return true;
  return block == CCVV && nslot == 4 && perm[0] == 1 && perm[1] == 0 && perm[2] == 3 && perm[3] == 2;
}

// Images of a coupling term that act identically: the ccvv ket read through
// the joint exchange (i, a) <-> (j, b) of its slots (a symmetry of x), and
// the ccvv bra written through it (the packed result is the same: the
// exchange has character +1 in both ccvv entries).  Among them the form that
// a slot GEMM can run without a permuted copy of x and with f along an inner
// slot is preferred, then the lexicographically smallest (ks, fx, fy).
void canonical_term(bool up, int bra, int ket, int nslot_b, int nslot_k, int nsum, int ny, int* ks, int* fx,
                    int* fy) {
  auto pi = [](int v) { return v >= 0 && v < 4 ? (v ^ 1) : v; };
  const bool kswap = !up && ket == CCVV && nslot_k == 4;
  const bool bswap = bra == CCVV && nslot_b == 4;
  auto score = [&](const int* c) {
    int sb, perm[4];
    if (up || bra != ket || nsum != 1 || ny != 1 || !slot_form(c, c[4], c[5], nslot_k, &sb, perm)) return 4;
    return (perm_trivial(ket, perm, nslot_k) ? 0 : 2) + (sb == nslot_b - 1 ? 1 : 0);
  };
  int best[6] = {ks[0], ks[1], ks[2], ks[3], *fx, *fy};
  int best_score = score(best);
  for (int m = 1; m < 4; ++m) {
    if (((m & 1) && !kswap) || ((m & 2) && !bswap)) continue;
    int c[6] = {ks[0], ks[1], ks[2], ks[3], *fx, *fy};
    if (m & 1) {
      std::swap(c[0], c[1]);
      std::swap(c[2], c[3]);
    }
    if (m & 2) {
      for (int l = 0; l < nslot_k; ++l) c[l] = pi(c[l]);
      c[4] = pi(c[4]);
      c[5] = pi(c[5]);
    }
    const int sc = score(c);
    if (sc < best_score || (sc == best_score && std::lexicographical_compare(c, c + 6, best, best + 6))) {
      std::copy(c, c + 6, best);
      best_score = sc;
    }
  }
  std::copy(best, best + 4, ks);
  *fx = best[4];
  *fy = best[5];
}

}  // namespace caspt2
