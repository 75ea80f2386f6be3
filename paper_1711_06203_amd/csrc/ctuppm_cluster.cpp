// Berger & Rigoutsos (1991) clustering of tagged cells into boxes (host code).
//
// The paper's grids are adaptive: cells are tagged for refinement and boxes
// are built around them (section 2, section 3).  Here the tags of a level's
// index space are first coarsened by the blocking factor (a block is tagged
// if any of its cells is), the blocks are clustered, and the clusters are
// refined back, so every box is aligned to the blocking factor and boxes never
// overlap.  A cluster is accepted when its fraction of tagged blocks reaches
// the efficiency and no edge exceeds the maximum; otherwise it is cut: at an
// interior hole of a signature (the tagged-block count per plane), else at the
// strongest sign change of a signature's second difference, else across the
// middle of its longest edge.
#include <algorithm>
#include <cstdint>
#include <vector>

#include "ctuppm.h"

namespace {

struct Blocks {
  int n[3];
  std::vector<uint8_t> t;
  bool at(int i, int j, int k) const { return t[(size_t(k) * n[1] + j) * n[0] + i] != 0; }
};

struct Rect {
  int lo[3], hi[3];
  long long vol() const {
    long long v = 1;
    for (int d = 0; d < 3; ++d) v *= hi[d] - lo[d] + 1;
    return v;
  }
};

// Tagged blocks per plane of r along d.
std::vector<long long> signature(const Blocks& B, const Rect& r, int d) {
  std::vector<long long> s(r.hi[d] - r.lo[d] + 1, 0);
  for (int k = r.lo[2]; k <= r.hi[2]; ++k)
    for (int j = r.lo[1]; j <= r.hi[1]; ++j)
      for (int i = r.lo[0]; i <= r.hi[0]; ++i)
        if (B.at(i, j, k)) {
          const int x[3] = {i, j, k};
          s[x[d] - r.lo[d]] += 1;
        }
  return s;
}

// Bounding box of the tagged blocks inside r; false if none.
bool shrink(const Blocks& B, Rect& r, long long& ntag) {
  Rect b{{r.hi[0] + 1, r.hi[1] + 1, r.hi[2] + 1}, {r.lo[0] - 1, r.lo[1] - 1, r.lo[2] - 1}};
  ntag = 0;
  for (int k = r.lo[2]; k <= r.hi[2]; ++k)
    for (int j = r.lo[1]; j <= r.hi[1]; ++j)
      for (int i = r.lo[0]; i <= r.hi[0]; ++i)
        if (B.at(i, j, k)) {
          const int x[3] = {i, j, k};
          ++ntag;
          for (int d = 0; d < 3; ++d) {
            b.lo[d] = std::min(b.lo[d], x[d]);
            b.hi[d] = std::max(b.hi[d], x[d]);
          }
        }
  if (ntag == 0) return false;
  r = b;
  return true;
}

// Cut position along a direction (first plane of the upper part), or -1.
void choose_cut(const Blocks& B, const Rect& r, int& dir, int& at) {
  // 1. an interior hole of a signature, closest to the middle
  dir = -1;
  at = -1;
  int best = 1 << 30;
  for (int d = 0; d < 3; ++d) {
    const std::vector<long long> s = signature(B, r, d);
    const int len = int(s.size());
    for (int p = 1; p < len - 1; ++p)
      if (s[p] == 0) {
        const int dist = std::abs(2 * p - len);
        if (dist < best) {
          best = dist;
          dir = d;
          at = r.lo[d] + p;  // the hole goes to the upper part, which shrinks
        }
      }
  }
  if (dir >= 0) return;
  // 2. the strongest sign change of the second difference (an inflection)
  long long strength = 0;
  for (int d = 0; d < 3; ++d) {
    const std::vector<long long> s = signature(B, r, d);
    const int len = int(s.size());
    if (len < 4) continue;
    std::vector<long long> lap(len, 0);
    for (int p = 1; p < len - 1; ++p) lap[p] = s[p + 1] - 2 * s[p] + s[p - 1];
    for (int p = 2; p < len - 1; ++p)
      if ((lap[p - 1] < 0 && lap[p] > 0) || (lap[p - 1] > 0 && lap[p] < 0)) {
        const long long st = std::llabs(lap[p] - lap[p - 1]);
        if (st > strength) {
          strength = st;
          dir = d;
          at = r.lo[d] + p;
        }
      }
  }
  if (dir >= 0) return;
  // 3. the middle of the longest edge
  int len = 0;
  for (int d = 0; d < 3; ++d)
    if (r.hi[d] - r.lo[d] + 1 > len) {
      len = r.hi[d] - r.lo[d] + 1;
      dir = d;
    }
  at = len >= 2 ? r.lo[dir] + len / 2 : -1;
}

void cluster(const Blocks& B, Rect r, double eff, int max_edge, std::vector<Rect>& out, int depth) {
  long long ntag = 0;
  if (!shrink(B, r, ntag)) return;
  bool small = true;
  for (int d = 0; d < 3; ++d) small = small && (r.hi[d] - r.lo[d] + 1 <= max_edge);
  const double e = double(ntag) / double(r.vol());
  if ((e >= eff && small) || depth > 64) {
    out.push_back(r);
    return;
  }
  int dir, at;
  choose_cut(B, r, dir, at);
  if (dir < 0 || at < 0) {  // a single block cannot be cut
    out.push_back(r);
    return;
  }
  Rect a = r, b = r;
  a.hi[dir] = at - 1;
  b.lo[dir] = at;
  cluster(B, a, eff, max_edge, out, depth + 1);
  cluster(B, b, eff, max_edge, out, depth + 1);
}

}  // namespace

extern "C" int ctuppm_cluster(const unsigned char* tags, const int n[3], int blocking, double efficiency,
                              int max_edge, ctuppm_box* boxes, int capacity, int* nboxes) {
  if (!tags || !n || !boxes || !nboxes || blocking < 1 || max_edge < blocking || capacity < 0 ||
      !(efficiency > 0.0 && efficiency <= 1.0))
    return CTUPPM_EINVAL;
  for (int d = 0; d < 3; ++d)
    if (n[d] < 1) return CTUPPM_EINVAL;
  Blocks B;
  for (int d = 0; d < 3; ++d) B.n[d] = (n[d] + blocking - 1) / blocking;
  B.t.assign(size_t(B.n[0]) * B.n[1] * B.n[2], 0);
  for (int k = 0; k < n[2]; ++k)
    for (int j = 0; j < n[1]; ++j)
      for (int i = 0; i < n[0]; ++i)
        if (tags[(size_t(k) * n[1] + j) * n[0] + i])
          B.t[(size_t(k / blocking) * B.n[1] + j / blocking) * B.n[0] + i / blocking] = 1;
  std::vector<Rect> out;
  const Rect all{{0, 0, 0}, {B.n[0] - 1, B.n[1] - 1, B.n[2] - 1}};
  cluster(B, all, efficiency, max_edge / blocking, out, 0);
  *nboxes = int(out.size());
  if (int(out.size()) > capacity) return CTUPPM_ENOMEM;
  for (size_t q = 0; q < out.size(); ++q)
    for (int d = 0; d < 3; ++d) {
      boxes[q].lo[d] = out[q].lo[d] * blocking;
      boxes[q].hi[d] = std::min(n[d] - 1, (out[q].hi[d] + 1) * blocking - 1);
    }
  return CTUPPM_OK;
}
