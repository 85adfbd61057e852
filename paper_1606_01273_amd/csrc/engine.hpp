// Host-side bookkeeping for the internally contracted CASPT2 hot path:
// block definitions (Eq. 8), the external/active factorisation of operator
// strings and the Wick pairings of their external part, and the determinant
// sector tables used by the GPU gather kernels.  No floating-point work on
// the problem data happens here; every contraction runs in HIP kernels.
#pragma once
#include <array>
#include <cstdint>
#include <map>
#include <string>
#include <vector>

namespace caspt2 {

enum Space : char { CLO = 'c', ACT = 'a', VIR = 'v' };

struct Op {
  char kind;          // 'c' creator, 'a' annihilator
  std::string label;  // orbital label
  char space;         // CLO, ACT, VIR
  std::string spin;   // spin variable
};

using OpString = std::vector<Op>;

// E_pq = sum_s a+_{p s} a_{q s}
OpString E(const std::string& p, char sp, const std::string& q, char sq, const std::string& spin);
OpString dagger(const OpString& o);
OpString suffixed(const OpString& o, const std::string& suf);

struct Block {
  std::string name;
  std::vector<std::pair<std::string, char>> ext;  // slots in storage order
  std::vector<std::string> act;                   // active labels, storage order
  std::vector<OpString> types;                    // operator strings
  std::vector<std::pair<int, int>> swaps;         // exchangeable slot pairs
};

const std::vector<Block>& blocks();
enum BlockId { CCVV = 0, CAVV, AAVV, CCAV, CCAA, AAAV, CAAA, CAAV, NBLOCK };

// characters allowed for a block (entries of the packed layout)
std::vector<std::vector<int>> characters(const Block& b);

// An active operator with its spin fixed.
struct ActOp {
  char kind;
  std::string label;
  int spin;
};
using ActString = std::vector<ActOp>;

struct WickEntry {
  double coeff;       // sign of the ext/active split times the pairing value
  ActString bra;      // active string of the bra function (as in the function)
  ActString mid;      // active part of the operator
  ActString ket;      // active string of the ket function
};

struct Pairing {
  std::vector<std::pair<std::string, std::string>> pairs;  // identified labels
  std::vector<WickEntry> entries;
};

// sum over spins of <core,M| bra^+ op ket |core,N>, grouped by Wick pairing
// of the closed and virtual operators.
std::vector<Pairing> matrix_element(const OpString& bra, const OpString& op, const OpString& ket);

// A down coupling term of a block with itself (ket slot sources ks: a bra
// slot >= 0 or summed label -1 - s; Fock indices fx, fy likewise) whose one
// summed label takes the place of one bra slot sb, the other ket slots being
// fed one to one by the remaining bra slots, and whose Fock element is
// f(bra slot sb, summed label): f applied along slot sb of the ket tensor
// read with its slots permuted, perm[l] the bra slot feeding ket slot l (sb
// for the summed one).  False for any other term.
bool slot_form(const int* ks, int fx, int fy, int nslot, int* sb_out, int* perm);
// the slot-permuted tensor equals x itself: the identity map, or for ccvv
// the joint exchange (i, a) <-> (j, b)
bool perm_trivial(int block, const int* perm, int nslot);
// Canonical form of a coupling term (ket slot sources ks[4], Fock indices
// fx, fy; rewritten in place) among the images that give the same packed
// contribution: the ccvv ket read through its joint slot exchange, the ccvv
// bra written through it.  Prefers the form a slot GEMM runs without a
// permuted copy and with f along an inner slot, then the smallest.
void canonical_term(bool up, int bra, int ket, int nslot_b, int nslot_k, int nsum, int ny, int* ks, int* fx,
                    int* fy);

// ---------------------------------------------------------------------------
// determinant sectors of the active space
// ---------------------------------------------------------------------------
struct Sector {
  int na_el, nb_el;
  bool operator<(const Sector& o) const {
    return na_el != o.na_el ? na_el < o.na_el : nb_el < o.nb_el;
  }
  bool operator==(const Sector& o) const { return na_el == o.na_el && nb_el == o.nb_el; }
};

struct ActiveSpace {
  int na;
  explicit ActiveSpace(int na_) : na(na_) {}
  std::vector<int64_t> strings(int n) const;     // ascending bit masks
  int64_t nstr(int n) const;
  int64_t dim(Sector s) const { return nstr(s.na_el) * nstr(s.nb_el); }
  bool valid(Sector s) const {
    return s.na_el >= 0 && s.nb_el >= 0 && s.na_el <= na && s.nb_el <= na;
  }
  // Gather table of a_{r spin} (kind 'a') or a+_{r spin} ('c') from sector
  // `from` into the target sector, for every r: src[r*dim_to + t] is the
  // source determinant of target t (or -1), sign[r*dim_to + t] its sign.
  Sector target(char kind, int spin, Sector from) const;
  void gather_table(char kind, int spin, Sector from, std::vector<int32_t>& src,
                    std::vector<double>& sign) const;
};

}  // namespace caspt2
