// Host-side check of the batched split (tq_batched.h batch_split): for every
// query count up to 1024, every query tile of the two engines, grids from 8 to
// 2048 workgroups and databases of 1 to 156 250 tiles, the split must stay
// inside the buffers sized from it (batch_max_lists, batch_max_parts), cover
// every tile, keep the part count a multiple of the XCD count, take at most
// kMaxRounds rounds of the grid unless the query tiles alone need more (the
// 8-part floor), and never use fewer parts than one round of the grid holds.
// The same for the sample split of the matrix engine (see below).
// Prints "OK <cases>" or the first violation.
#include <cstdio>

#include "tq_batched.h"

int main() {
  const int qtiles[] = {2, 4, 8, 16, 64, 128, 256};
  const int grids[] = {8, 16, 24, 256, 512, 768, 1024, 2048};
  const long long spans[] = {1, 7, 8, 9, 100, 1000, 15625, 78125, 156250};
  long long cases = 0;
  for (int qt : qtiles)
    for (int grid : grids)
      for (long long span : spans)
        for (int nq = 1; nq <= 1024; ++nq) {
          for (long long lo : {0LL, 3LL}) {
            tqi::BatchParams b;
            tqi::batch_split(b, nq, qt, grid, lo, lo + span);
            ++cases;
            const long long parts = b.parts, tpp = b.tiles_per_part;
            const long long nqt = (nq + qt - 1) / qt;
            const long long rounds = (nqt * parts + grid - 1) / grid;
            // the parts one round of the grid holds (a multiple of 8), capped by the tiles
            const long long cap = (span + tqi::kXcds - 1) / tqi::kXcds * tqi::kXcds;
            long long one = grid / (tqi::kXcds * nqt) * tqi::kXcds;
            if (one > cap) one = cap;
            const char *bad = nullptr;
            if (b.nqt != nqt) bad = "query tile count";
            else if (parts < tqi::kXcds || parts % tqi::kXcds) bad = "part count not a positive multiple of 8";
            else if (parts > tqi::batch_max_parts(grid)) bad = "more parts than the merge bound";
            else if (static_cast<size_t>(nq) * parts > tqi::batch_max_lists(qt, grid, nq))
              bad = "more lists than the buffers";
            else if (tpp < 1 || tpp * parts < span) bad = "tiles not covered";
            else if ((tpp - 1) * parts >= span && span >= parts) bad = "parts longer than needed";
            else if (rounds > tqi::kMaxRounds && parts != tqi::kXcds) bad = "more rounds than allowed";
            else if (one >= tqi::kXcds && parts < one) bad = "fewer parts than one round of the grid holds";
            else if (b.tile_lo != lo || b.tile_hi != lo + span) bad = "tile range";
            if (bad) {
              std::printf("FAIL %s: nq=%d qtile=%d grid=%d tiles=%lld parts=%lld tpp=%lld\n", bad, nq, qt, grid, span,
                          parts, tpp);
              return 1;
            }
          }
        }
  // The matrix engine's sample pass (every 16th tile, k > 16): its split of
  // the sample tiles fits the same list buffers as the full scan's, every
  // sample tile is a database tile of the range, and its lists (8 or 16 keys,
  // fewer than k) hold at least 2k keys per query when they are 8 long.
  for (int qt : {64, 128, 256})
    for (int grid : grids)
      for (long long span : spans)
        for (int nq = 1; nq <= 1024; ++nq)
          for (int k : {17, 64, 100, 128}) {
            const long long lo = 3;
            const int stride = 16;
            tqi::BatchParams b, sb;
            tqi::batch_split(b, nq, qt, grid, lo, lo + span);
            tqi::sample_split(sb, b, qt, grid, stride);
            ++cases;
            const long long stiles = (span + stride - 1) / stride;
            const int lk = tqi::sample_list_len(sb.parts, k);
            const char *bad = nullptr;
            if (sb.nq != nq || sb.tile_lo != 0 || sb.tile_hi != stiles) bad = "sample range";
            else if (lo + (stiles - 1) * stride >= lo + span) bad = "sample tile past the range";
            else if (sb.tiles_per_part * sb.parts < stiles) bad = "sample tiles not covered";
            else if (static_cast<size_t>(nq) * sb.parts > tqi::batch_max_lists(qt, grid, nq))
              bad = "more sample lists than the buffers";
            else if (!(lk == 8 || lk == 16) || lk >= k) bad = "sample list length";
            else if (lk == 8 && sb.parts * 8LL < 2LL * k) bad = "8-key sample lists hold fewer than 2k keys";
            else if (sb.bound || sb.running || sb.ids || sb.scores || sb.slots) bad = "sample split keeps outputs";
            if (bad) {
              std::printf("FAIL %s: nq=%d qtile=%d grid=%d tiles=%lld k=%d parts=%d\n", bad, nq, qt, grid, span, k,
                          sb.parts);
              return 1;
            }
          }
  std::printf("OK %lld\n", cases);
  return 0;
}
