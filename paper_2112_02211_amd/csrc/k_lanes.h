// Lane tables that spread a wavefront's 16-byte LDS accesses over the banks.
//
// A kernel that gives each lane one grid line of a leaf and walks the lines'
// entries at a common stride reads, at each step, one 16-byte entry per lane
// at (first index of the lane's line) + step * stride.  With 64 four-byte
// banks, 16 entries of 16 B whose indices differ mod 16 touch disjoint banks
// (and 8 whose indices differ mod 8 cover 32 of them), which is what the bank
// conflict counters rewarded when measured.  The table assigns the lines of each axis pass
// to the slots of up to two wavefronts (slot = 64 * wavefront + lane) so that
// each group of 16 slots takes lines of as many different residues mod 16 as
// remain, the most plentiful residues first, in residue order (so each half
// group of 8 also differs mod 8).  Evaluated at compile time.
#pragma once

namespace hps {

// word s: in byte ax the line that slot s takes in axis pass ax (0, 1, 2);
// slots past the last line hold the number of lines
struct LaneTable {
  unsigned int w[128];
};

// nl lines per pass (at most 128); base(ax, line) is the LDS index, in 16-byte
// entries, of the line's first entry in pass ax
template <class Base>
constexpr LaneTable bank_spread_lanes(int nl, Base base) {
  LaneTable t{};
  for (int s = 0; s < 128; ++s) t.w[s] = 0;
  for (int ax = 0; ax < 3; ++ax) {
    int res[128] = {};
    int cnt[16] = {};
    bool used[128] = {};
    for (int l = 0; l < nl; ++l) {
      res[l] = base(ax, l) % 16;
      ++cnt[res[l]];
    }
    int slot = 0;
    while (slot < nl) {
      const int g = nl - slot < 16 ? nl - slot : 16;
      int took[16] = {};
      for (int k = 0; k < g; ++k) {
        int best = -1;
        for (int r = 0; r < 16; ++r) {
          if (cnt[r] == 0) continue;
          if (best < 0 || took[r] < took[best] || (took[r] == took[best] && cnt[r] > cnt[best])) best = r;
        }
        ++took[best];
        --cnt[best];
      }
      for (int r = 0; r < 16; ++r)
        for (int k = 0; k < took[r]; ++k) {
          int l = 0;
          while (used[l] || res[l] != r) ++l;
          used[l] = true;
          t.w[slot++] |= (unsigned)l << (8 * ax);
        }
    }
    for (int s = nl; s < 128; ++s) t.w[s] |= (unsigned)nl << (8 * ax);
  }
  return t;
}

}  // namespace hps
