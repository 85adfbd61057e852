// Prints the Wick pairings of <bra| E_xy |ket> (and of the plain overlap)
// that the library's host engine finds for every pair of excitation blocks,
// operator types and orbital classes of x and y, one canonical line per
// spin assignment, for comparison with the oracle's own enumeration.
#include <algorithm>
#include <cstdio>
#include <string>
#include <vector>

#include "engine.hpp"

using namespace caspt2;

static std::string act(const ActString& s) {
  std::string out;
  for (const auto& o : s) out += std::string(1, o.kind) + ":" + o.label + ":" + std::to_string(o.spin) + ";";
  return out;
}

int main() {
  const auto& BL = blocks();
  const char classes[3] = {CLO, ACT, VIR};
  for (size_t bb = 0; bb < BL.size(); ++bb)
    for (size_t kb = 0; kb < BL.size(); ++kb)
      for (int cx = -1; cx < 3; ++cx)
        for (int cy = 0; cy < 3; ++cy) {
          if (cx < 0 && cy > 0) continue;   // cx = -1: the overlap, once
          const OpString op = cx < 0 ? OpString{} : E("x_o", classes[cx], "y_o", classes[cy], "so");
          const std::string tag = cx < 0 ? "S" : std::string(1, classes[cx]) + classes[cy];
          for (size_t tb = 0; tb < BL[bb].types.size(); ++tb)
            for (size_t tk = 0; tk < BL[kb].types.size(); ++tk) {
              auto ps = matrix_element(suffixed(BL[bb].types[tb], "_b"), op, suffixed(BL[kb].types[tk], "_k"));
              for (const auto& P : ps) {
                std::vector<std::string> pr;
                for (const auto& q : P.pairs) {
                  std::string a = q.first, b = q.second;
                  if (b < a) std::swap(a, b);
                  pr.push_back(a + "=" + b);
                }
                std::sort(pr.begin(), pr.end());
                std::string pk;
                for (const auto& x : pr) pk += x + ",";
                for (const auto& w : P.entries)
                  std::printf("%s %s %s %zu %zu|%s|%.12g|%s|%s|%s\n", BL[bb].name.c_str(), BL[kb].name.c_str(),
                              tag.c_str(), tb, tk, pk.c_str(), w.coeff, act(w.bra).c_str(), act(w.mid).c_str(),
                              act(w.ket).c_str());
              }
            }
        }
  return 0;
}
