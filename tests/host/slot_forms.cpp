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
  if (fails) return EXIT_FAILURE;
  std::printf("ok\n");
  return 0;
}
