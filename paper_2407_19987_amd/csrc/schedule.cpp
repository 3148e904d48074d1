// Work schedule of the blocked annealer (host only): each block's chunk
// lists dealt to the streaming waves of a work-group in whole rounds of
// kBlockRing slots.
//
// A wave's slots for a block are its early part (leading field chunks that
// read no bit of the block before it in the sweep), padded to whole rounds,
// then its late part (the other field chunks, then whole pair tiles), padded
// to whole rounds.  Every slot loads a tile, padding slots the zero tile, so
// the padding costs as much load bandwidth as a chunk: the rounds are dealt
// so that the block needs as few as possible.
//
//  * Early part: ceil(ne / D) rounds, spread evenly over the waves as
//    contiguous chunk ranges; only the range holding the last early chunk is
//    partial.
//  * Late part: ceil(late chunks / D) rounds, each given to the wave with the
//    fewest late rounds so far, then the fewest rounds in all.  Pair tiles go whole to the
//    wave with the most free slots (a tile that fits nowhere gets the rounds
//    it needs there); the late field chunks then fill the free slots in wave
//    order.
#include <algorithm>
#include <cstdint>
#include <numeric>
#include <vector>

#include "hobo_internal.h"

namespace hobo {

void build_block_schedule(const std::vector<BlockMeta>& blocks, int ns, bool masked, std::vector<uint32_t>* words,
                          std::vector<uint32_t>* hdr) {
  constexpr int D = kBlockRing;
  words->clear();
  hdr->clear();
  auto chunk_word = [](uint32_t c, bool close, int tgt) {
    return (c + 1u) | ((close ? 1u : 0u) << 20) | ((uint32_t)tgt << 22);
  };
  for (const BlockMeta& m : blocks) {
    const int ne = masked ? 0 : (int)m.nearly;
    const int nl = (int)m.nchunks[0] - ne;
    const int npt = (int)m.npt;
    // early rounds and chunk ranges
    const int re = (ne + D - 1) / D;
    std::vector<int> e0((size_t)ns), e1((size_t)ns), rounds((size_t)ns);
    for (int v = 0; v < ns; ++v) {
      const int a = re * v / ns, b = re * (v + 1) / ns;
      e0[(size_t)v] = std::min(ne, D * a);
      e1[(size_t)v] = std::min(ne, D * b);
      rounds[(size_t)v] = b - a;
    }
    // late rounds: each to the wave with the fewest late rounds so far, then
    // the fewest rounds in all (the late part runs after the decisions, so
    // its longest share is on every block's path)
    int late = nl;
    for (int t = 0; t < npt; ++t) late += (int)m.nchunks[1 + t];
    std::vector<int> lr((size_t)ns, 0);
    for (int k = 0; k < (late + D - 1) / D; ++k) {
      int best = 0;
      for (int v = 1; v < ns; ++v) {
        const int lv = lr[(size_t)v], lb = lr[(size_t)best];
        if (lv < lb || (lv == lb && rounds[(size_t)v] < rounds[(size_t)best])) best = v;
      }
      ++lr[(size_t)best];
    }
    // pair tiles, largest first, whole to the wave with the most free slots
    std::vector<int> used((size_t)ns, 0);
    std::vector<std::vector<int>> tiles_of((size_t)ns);
    std::vector<int> tord((size_t)npt);
    std::iota(tord.begin(), tord.end(), 0);
    std::stable_sort(tord.begin(), tord.end(), [&](int x, int y) { return m.nchunks[1 + x] > m.nchunks[1 + y]; });
    for (int t : tord) {
      const int sz = (int)m.nchunks[1 + t];
      if (sz == 0) continue;
      int best = 0;
      for (int v = 1; v < ns; ++v)
        if (D * lr[(size_t)v] - used[(size_t)v] > D * lr[(size_t)best] - used[(size_t)best]) best = v;
      while (D * lr[(size_t)best] - used[(size_t)best] < sz) ++lr[(size_t)best];
      used[(size_t)best] += sz;
      tiles_of[(size_t)best].push_back(t);
    }
    // late field chunks fill the free slots in wave order (they always fit:
    // the late rounds hold every late chunk, and a pair tile that did not fit
    // only added rounds)
    std::vector<int> l0((size_t)ns, 0), l1((size_t)ns, 0);
    int next = 0;
    for (int v = 0; v < ns; ++v) {
      const int take = std::min(nl - next, D * lr[(size_t)v] - used[(size_t)v]);
      l0[(size_t)v] = next;
      l1[(size_t)v] = next + take;
      next += take;
    }
    const uint32_t c0 = m.chunk0[0];
    for (int v = 0; v < ns; ++v) {
      const size_t base = words->size();
      const bool has_late_fields = l1[(size_t)v] > l0[(size_t)v];
      // the wave's last field chunk closes its field list
      const int64_t last = has_late_fields ? (int64_t)c0 + ne + l1[(size_t)v] - 1
                                           : (e1[(size_t)v] > e0[(size_t)v] ? (int64_t)c0 + e1[(size_t)v] - 1 : -1);
      for (int c = e0[(size_t)v]; c < e1[(size_t)v]; ++c)
        words->push_back(chunk_word(c0 + (uint32_t)c, (int64_t)(c0 + (uint32_t)c) == last, 0));
      while ((words->size() - base) % D) words->push_back(kSlotPad);
      const int pe = (int)(words->size() - base);
      for (int c = l0[(size_t)v]; c < l1[(size_t)v]; ++c) {
        const uint32_t cc = c0 + (uint32_t)(ne + c);
        words->push_back(chunk_word(cc, (int64_t)cc == last, 0));
      }
      for (int t : tiles_of[(size_t)v])
        for (uint32_t c = 0; c < m.nchunks[1 + t]; ++c)
          words->push_back(chunk_word(m.chunk0[1 + t] + c, c + 1 == m.nchunks[1 + t], 1 + t));
      while ((words->size() - base) % D) words->push_back(kSlotPad);
      if (words->size() == base)
        for (int d = 0; d < D; ++d) words->push_back(kSlotPad);
      hdr->push_back((uint32_t)base);
      hdr->push_back(((uint32_t)pe << 16) | (uint32_t)(words->size() - base));
    }
  }
}

}  // namespace hobo
