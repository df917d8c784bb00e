// Host-only check of the sweep's tile bookkeeping (paper_1808_07284_amd/csrc/emd_tiling.h):
// the padded layout, the tile tables over the XCDs, the split into chains and the
// narrowing rule, on random batches.  Built with the address and undefined-behaviour
// sanitizers by tests/test_sanitizers.py; exits non-zero on the first violated rule.
#include <cstdio>
#include <cstdlib>
#include <random>
#include <set>
#include <vector>

#include "emd_tiling.h"

using namespace emd;

#define CHECK(cond)                                                                     \
    do {                                                                                \
        if (!(cond)) {                                                                  \
            std::fprintf(stderr, "violated: %s (line %d, case %d)\n", #cond, __LINE__, ncase); \
            std::exit(1);                                                               \
        }                                                                               \
    } while (0)

int main()
{
    int ncase = 0;
    long tiles_seen = 0;
    for (int seed = 1; seed <= 300; ++seed, ++ncase) {
        std::mt19937_64 rng(seed);
        auto uni = [&](int lo, int hi) { return std::uniform_int_distribution<int>(lo, hi)(rng); };
        const int n = uni(1, 70);
        const int span = 56 * (uni(0, 1) ? 4 : 2);
        std::vector<tiling::GatherIn> gin(n);
        int64_t off = 0;
        for (auto& g : gin) {
            g.nr = uni(0, 9) == 0 ? 1 : uni(1, 600);
            g.nt = uni(0, 9) == 0 ? 1 : uni(1, 4000);
            g.dx = 1.0 / std::max(g.nr - 1, 1);
            g.dt = 1.0 / std::max(g.nt - 1, 1);
            g.offset = off;
            off += (int64_t)g.nr * g.nt;
            g.rows = uni(0, 3) == 0 ? uni(1, 40) : 16;
        }
        const tiling::Layout L = tiling::plan_layout(gin, span, 0.0, 1e5);
        CHECK((int)L.meta.size() == n);
        int64_t prev_end = 0;
        int32_t base = 0;
        for (int g = 0; g < n; ++g) {
            const GatherMeta& m = L.meta[g];
            CHECK(m.ld >= m.nt && m.ld % 32 == 0);
            CHECK(m.poff % 64 == 0 && m.poff >= prev_end);
            prev_end = m.poff + (int64_t)m.nr * m.ld;
            CHECK(m.tile_base == base);
            CHECK(L.ntt[g] == (m.nt + span - 1) / span && L.nst[g] == (m.nr + m.rows - 1) / m.rows);
            CHECK(m.ntiles == L.ntt[g] * L.nst[g]);
            CHECK(m.alpha1 > 0.0);
            base += m.ntiles;
        }
        CHECK(L.slots == base && L.padded_len >= prev_end);

        // the full table: every tile once, in eight equal runs of whole blocks
        std::vector<char> all(n, 1);
        const std::vector<Tile> full = tiling::layout_tiles(L, span, all);
        CHECK(full.size() % (tiling::kXcd * tiling::kWavesPerBlock) == 0);
        const size_t run = full.size() / tiling::kXcd;
        std::vector<int> hits(L.slots, 0);
        std::vector<Tile> by_slot(L.slots);
        for (size_t x = 0; x < (size_t)tiling::kXcd; ++x) {
            bool padding = false;
            int last_g = -1, last_strip = -1;
            for (size_t k = x * run; k < (x + 1) * run; ++k) {
                const Tile& t = full[k];
                if (t.g < 0) {
                    padding = true;
                    continue;
                }
                CHECK(!padding);  // real entries first, padding after
                CHECK(t.g < n);
                const GatherMeta& m = L.meta[t.g];
                CHECK(t.r0 >= 0 && t.r0 < m.nr && t.r0 % m.rows == 0);
                CHECK(t.c0 >= 0 && t.c0 < m.nt && t.c0 % span == 0);
                CHECK(t.slot == m.tile_base + (t.r0 / m.rows) * L.ntt[t.g] + t.c0 / span);
                // gather-major, strip by strip
                CHECK(t.g > last_g || (t.g == last_g && t.r0 / m.rows >= last_strip));
                last_strip = t.g == last_g ? std::max(last_strip, t.r0 / m.rows) : t.r0 / m.rows;
                last_g = t.g;
                ++hits[t.slot];
                by_slot[t.slot] = t;
                ++tiles_seen;
            }
        }
        for (int s = 0; s < L.slots; ++s) CHECK(hits[s] == 1);

        // a narrowed table: the selected gathers' tiles, unchanged
        std::vector<char> sel(n);
        for (auto& c : sel) c = (char)uni(0, 1);
        const std::vector<Tile> part = tiling::layout_tiles(L, span, sel);
        CHECK(part.size() % (tiling::kXcd * tiling::kWavesPerBlock) == 0);
        std::set<int> seen;
        for (const Tile& t : part) {
            if (t.g < 0) continue;
            CHECK(sel[t.g]);
            const Tile& f = by_slot[t.slot];
            CHECK(f.g == t.g && f.r0 == t.r0 && f.c0 == t.c0);
            CHECK(seen.insert(t.slot).second);
        }
        int64_t want = 0;
        for (int g = 0; g < n; ++g)
            if (sel[g]) want += L.meta[g].ntiles;
        CHECK((int64_t)seen.size() == want);

        // chains: a partition of the selected gathers with balanced cells
        std::vector<int64_t> cells(n);
        int64_t biggest = 0, nsel = 0;
        for (int g = 0; g < n; ++g) {
            cells[g] = (int64_t)gin[g].nr * gin[g].nt;
            if (sel[g]) {
                biggest = std::max(biggest, cells[g]);
                ++nsel;
            }
        }
        for (int nc = 1; nc <= 4; ++nc) {
            const auto chains = tiling::split_chains(cells, sel, nc);
            CHECK((int64_t)chains.size() == std::max<int64_t>(1, std::min<int64_t>(nsel, nc)));
            std::vector<int64_t> load(chains.size(), 0);
            for (int g = 0; g < n; ++g) {
                int owners = 0;
                for (size_t k = 0; k < chains.size(); ++k)
                    if (chains[k][g]) {
                        ++owners;
                        load[k] += cells[g];
                    }
                CHECK(owners == (sel[g] ? 1 : 0));
            }
            const auto mm = std::minmax_element(load.begin(), load.end());
            CHECK(*mm.second - *mm.first <= biggest);
        }

        // the chain count: two chains from kChainMinTiles real tiles on
        const int64_t nt_sel = want;
        CHECK(tiling::chain_count(nt_sel, 2) == (nt_sel >= tiling::kChainMinTiles ? 2 : 1));
        CHECK(tiling::chain_count(tiling::kChainMinTiles - 1, 2) == 1 && tiling::chain_count(tiling::kChainMinTiles, 2) == 2);

        // the narrowing rule
        const int64_t table = uni(1, 1 << 20);
        const int64_t live = uni(0, (int)table);
        CHECK(tiling::narrow_now(live, table) == (live > 0 && live * 16 <= table * 15));
    }
    std::printf("ok: %d batches, %ld tiles\n", ncase, tiles_seen);
    return 0;
}
