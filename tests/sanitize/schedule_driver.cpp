// Host-side check of the blocked annealer's work schedule
// (build_block_schedule) on seeded random block layouts: every chunk of a
// block's lists is dealt exactly once; each wave's part holds early field
// chunks, then late field chunks, then whole pair tiles in order, padded to
// whole rounds; the close flags sit on each wave's last field chunk and on
// each pair tile's last chunk; the block needs no more rounds than its early
// and late chunks fill (plus the rounds of a pair tile that fit nowhere, and
// one per wave that has nothing).  Built with g++ (no device
// code).
#include <cstdint>
#include <cstdio>
#include <random>
#include <vector>

#include "hobo_internal.h"

using hobo::BlockMeta;
using hobo::kBlockRing;

int main() {
  std::mt19937_64 rng(11);
  int failures = 0;
  auto fail = [&](int trial, const char* what) {
    if (failures < 20) std::printf("trial %d: %s\n", trial, what);
    ++failures;
  };
  const int D = kBlockRing;
  for (int trial = 0; trial < 3000; ++trial) {
    const int ns = 1 + (int)(rng() % 14);
    const bool masked = rng() % 4 == 0;
    const int nblocks = 1 + (int)(rng() % 4);
    std::vector<BlockMeta> blocks((size_t)nblocks);
    uint32_t next = 0;
    for (auto& m : blocks) {
      m = BlockMeta{};
      const int nf = (int)(rng() % 300);
      m.chunk0[0] = next;
      m.nchunks[0] = (uint32_t)nf;
      m.nearly = nf ? (uint32_t)(rng() % (nf + 1)) : 0u;
      next += (uint32_t)nf;
      m.npt = (uint32_t)(rng() % (hobo::kPairTiles + 1));
      for (uint32_t t = 0; t < m.npt; ++t) {
        m.chunk0[1 + t] = next;
        m.nchunks[1 + t] = (uint32_t)(rng() % 12);  // may be empty
        next += m.nchunks[1 + t];
      }
      m.nbits = 16;
    }
    std::vector<uint32_t> words, hdr;
    hobo::build_block_schedule(blocks, ns, masked, &words, &hdr);
    if (hdr.size() != (size_t)(2 * nblocks * ns)) {
      fail(trial, "header size");
      continue;
    }
    for (int q = 0; q < nblocks; ++q) {
      const BlockMeta& m = blocks[(size_t)q];
      const uint32_t ne = masked ? 0u : m.nearly;
      std::vector<int> seen(next + 1, 0);
      int rounds = 0;
      int wave_nothing = 0;
      for (int v = 0; v < ns; ++v) {
        const uint32_t off = hdr[(size_t)(2 * (q * ns + v))], cnt = hdr[(size_t)(2 * (q * ns + v)) + 1];
        const int pe = (int)(cnt >> 16), all = (int)(cnt & 0xFFFFu);
        if (all % D || pe % D || pe > all || all < D || off + (size_t)all > words.size()) {
          fail(trial, "part sizes");
          continue;
        }
        rounds += all / D;
        int phase = 0;  // 0 early fields, 1 late fields, 2 pair tiles
        int last_field = -1, cur_tile = -1;
        uint32_t expect_next_in_tile = 0;
        bool any = false, field_closed = false;
        for (int k = 0; k < all; ++k) {
          const uint32_t w = words[off + (size_t)k];
          const uint32_t kind = (w >> 20) & 3u, tix = w & 0xFFFFFu, tgt = w >> 22;
          if (kind == 2u) {
            // padding only at the end of a part
            const int part_end = k < pe ? pe : all;
            for (int k2 = k; k2 < part_end; ++k2)
              if (((words[off + (size_t)k2] >> 20) & 3u) != 2u) fail(trial, "padding inside a part");
            continue;
          }
          if (kind == 3u || tix == 0u) {
            fail(trial, "bad slot word");
            continue;
          }
          any = true;
          const uint32_t c = tix - 1u;
          if (c >= next) {
            fail(trial, "chunk out of range");
            continue;
          }
          ++seen[c];
          const bool close = kind == 1u;
          if (tgt == 0) {
            if (c < m.chunk0[0] || c >= m.chunk0[0] + m.nchunks[0]) fail(trial, "field slot holds another list");
            const bool early = c < m.chunk0[0] + ne;
            if (k < pe && !early) fail(trial, "late chunk in the early part");
            if (k >= pe && early) fail(trial, "early chunk in the late part");
            if (phase == 2) fail(trial, "field chunk after a pair tile");
            phase = k < pe ? 0 : 1;
            if (last_field >= 0 && (int)c != last_field + 1 && !(k >= pe && last_field < (int)(m.chunk0[0] + ne)))
              fail(trial, "field chunks not contiguous");
            if (field_closed) fail(trial, "field chunk after the close");
            last_field = (int)c;
            field_closed = close;
          } else {
            const uint32_t t = tgt - 1u;
            if (t >= m.npt || c < m.chunk0[1 + t] || c >= m.chunk0[1 + t] + m.nchunks[1 + t])
              fail(trial, "pair slot holds another list");
            if (k < pe) fail(trial, "pair tile in the early part");
            if (phase == 1 || phase == 0) phase = 2;
            if ((int)t != cur_tile) {
              if (c != m.chunk0[1 + t]) fail(trial, "pair tile does not start at its first chunk");
              cur_tile = (int)t;
            } else if (c != expect_next_in_tile) {
              fail(trial, "pair tile chunks out of order");
            }
            expect_next_in_tile = c + 1;
            if (close != (c + 1 == m.chunk0[1 + t] + m.nchunks[1 + t])) fail(trial, "pair close flag");
          }
        }
        if (last_field >= 0 && !field_closed) fail(trial, "wave's fields never closed");
        if (!any) ++wave_nothing;
      }
      uint32_t first = m.chunk0[0];
      uint32_t end = m.npt ? m.chunk0[m.npt] + m.nchunks[m.npt] : m.chunk0[0] + m.nchunks[0];
      for (uint32_t c = first; c < end; ++c)
        if (seen[c] != 1) fail(trial, "chunk not dealt exactly once");
      // round budget
      uint32_t late = m.nchunks[0] - ne;
      for (uint32_t t = 0; t < m.npt; ++t) late += m.nchunks[1 + t];
      int bound = (int)((ne + D - 1) / D + (late + D - 1) / D) + wave_nothing;
      for (uint32_t t = 0; t < m.npt; ++t) bound += (int)((m.nchunks[1 + t] + D - 1) / D);
      if (rounds > bound) fail(trial, "more rounds than the chunks need");
    }
  }
  std::printf("schedule driver: %d failures\n", failures);
  return failures ? 1 : 0;
}
