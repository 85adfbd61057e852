// Checks of the classification of within-block coupling terms (a Fock
// element of one orbital space applied along one slot of a block's
// amplitudes); exits non-zero with a message on the first failure.
#include <cstdio>
#include <cstdlib>

#include "engine.hpp"

using namespace caspt2;

static int fails = 0;
static void expect(bool ok, const char* what) {
  if (!ok) {
    std::fprintf(stderr, "FAIL: %s\n", what);
    ++fails;
  }
}

static bool same(const int* a, const int* b, int n) {
  for (int l = 0; l < n; ++l)
    if (a[l] != b[l]) return false;
  return true;
}

int main() {
  int sb = -9, perm[4];
  // ccvv: sum over the virtual of slot 2, the other slots fed in place
  {
    const int ks[4] = {0, 1, -1, 3};
    expect(slot_form(ks, 2, -1, 4, &sb, perm), "ccvv identity map is a slot form");
    const int want[4] = {0, 1, 2, 3};
    expect(sb == 2 && same(perm, want, 4), "ccvv identity map: slot 2, identity permutation");
    expect(perm_trivial(CCVV, perm, 4), "identity permutation is trivial");
  }
  // the same with f's indices in the other order
  {
    const int ks[4] = {0, 1, -1, 3};
    expect(slot_form(ks, -1, 2, 4, &sb, perm) && sb == 2, "f(z, e) order gives the same slot");
  }
  // ccvv: ket slot 2 fed by bra slot 3, summed label on ket slot 3 (the
  // virtual pair read exchanged)
  {
    const int ks[4] = {0, 1, 3, -1};
    expect(slot_form(ks, 2, -1, 4, &sb, perm), "exchanged virtual pair is a slot form");
    const int want[4] = {0, 1, 3, 2};
    expect(sb == 2 && same(perm, want, 4), "exchanged virtual pair: permutation (0 1 3 2)");
    expect(!perm_trivial(CCVV, perm, 4), "virtual-pair exchange alone is not a symmetry of ccvv");
  }
  // the joint exchange of ccvv is a symmetry, the closed-pair exchange of
  // ccav is not
  {
    const int j[4] = {1, 0, 3, 2};
    expect(perm_trivial(CCVV, j, 4), "joint exchange is trivial for ccvv");
    expect(!perm_trivial(CCAV, j, 3), "closed-pair exchange is not trivial for ccav");
    const int c[4] = {0, 2, 1, 3};
    expect(!perm_trivial(CAVV, c, 3), "virtual exchange is not trivial for cavv");
  }
  // not slot forms: two summed labels, an active Fock index, a bra slot
  // feeding two ket slots, f on a slot that also feeds the ket
  {
    const int two[4] = {0, 1, -1, -2};
    expect(!slot_form(two, 2, -1, 4, &sb, perm), "two summed labels");
    const int one[4] = {0, 1, -1, 3};
    expect(!slot_form(one, -10, -1, 4, &sb, perm), "active Fock index");
    const int dup[4] = {0, 0, -1, 3};
    expect(!slot_form(dup, 2, -1, 4, &sb, perm), "bra slot feeding two ket slots");
    const int fed[4] = {0, 1, 2, -1};
    expect(!slot_form(fed, 2, -1, 4, &sb, perm), "f row on a slot that feeds the ket");
    expect(!slot_form(one, 2, 3, 4, &sb, perm), "both Fock indices on bra slots");
  }
  // a one-slot block (aaav: the virtual)
  {
    const int ks[4] = {-1, 0, 0, 0};
    expect(slot_form(ks, 0, -1, 1, &sb, perm) && sb == 0 && perm[0] == 0, "one-slot block");
  }
  // canonical forms of the eight Wick pairings of <ccvv| f_vv E |ccvv> (closed
  // labels paired straight or crossed; x paired with the bra's a or b, y with
  // the ket's a or b): they act as two distinct terms, f along the bra's
  // first virtual slot with the ket read in place or with its virtual pair
  // exchanged
  {
    const int in[8][5] = {{0, 1, 3, -1, 2}, {0, 1, -1, 3, 2}, {0, 1, 2, -1, 3}, {0, 1, -1, 2, 3},
                          {1, 0, 3, -1, 2}, {1, 0, -1, 3, 2}, {1, 0, 2, -1, 3}, {1, 0, -1, 2, 3}};
    const int want_in_place[6] = {0, 1, -1, 3, 2, -1}, want_exchanged[6] = {0, 1, 3, -1, 2, -1};
    int n_in_place = 0, n_exchanged = 0;
    for (const auto& t : in) {
      int ks[4] = {t[0], t[1], t[2], t[3]}, fx = t[4], fy = -1;
      canonical_term(false, CCVV, CCVV, 4, 4, 1, 1, ks, &fx, &fy);
      const int got[6] = {ks[0], ks[1], ks[2], ks[3], fx, fy};
      if (same(got, want_in_place, 6)) ++n_in_place;
      else if (same(got, want_exchanged, 6)) ++n_exchanged;
      else expect(false, "ccvv virtual pairing canonicalises to one of the two forms");
    }
    expect(n_in_place == 4 && n_exchanged == 4, "four pairings per ccvv form");
    // the in-place form runs as a slot GEMM without a copy, on inner slot 2
    int ks[4] = {0, 1, -1, 3};
    expect(slot_form(ks, 2, -1, 4, &sb, perm) && sb == 2 && perm_trivial(CCVV, perm, 4), "in-place form");
  }
  // a term between different blocks keeps its form when nothing applies
  {
    int ks[4] = {2, 0, 1, 0}, fx = -1, fy = -10;
    canonical_term(false, CAVV, CCAV, 3, 3, 1, 8, ks, &fx, &fy);
    const int got[6] = {ks[0], ks[1], ks[2], ks[3], fx, fy}, want[6] = {2, 0, 1, 0, -1, -10};
    expect(same(got, want, 6), "no symmetry: unchanged");
  }
  if (fails) return EXIT_FAILURE;
  std::printf("ok\n");
  return 0;
}
