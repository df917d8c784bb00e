// emd_tiling.h -- host-only bookkeeping of the sweep's tile tables: the padded
// layout and tiles of each gather, the table order over the XCDs, the split of the
// running gathers into chains of launches, and when the tables narrow.  Plain C++
// with no HIP types, so that it can also be built and checked on its own (under the
// address and undefined-behaviour sanitizers).
#pragma once

#include <algorithm>
#include <cmath>
#include <cstdint>
#include <vector>

namespace emd {

// A sweep wave owns OUT_LANES * V consecutive time samples in lanes 1..OUT_LANES;
// lanes 0 and OUT_LANES + 1 carry the time-axis halo, the remaining lanes idle.
// 56 lanes x 16 bytes = 896 bytes = 7 whole 128-byte cache lines, so the stores of
// a row never leave a partially written line behind (a partial line costs a fill
// read and a whole-line write-back).
constexpr int OUT_LANES = 56;
constexpr int HALO_LANE_R = OUT_LANES + 1;

struct GatherMeta {
    int32_t nr, nt, ld, ntiles;  // grid, padded pitch, sweep tiles of the gather
    int32_t tile_base;           // first partial-sum slot (tiles own consecutive slots)
    int32_t rows;                // receiver rows per tile (one strip)
    int64_t poff;                // element offset in the padded workspace fields
    int64_t uoff;                // element offset in the caller's batch buffers
    double dx, dt;               // EMD grid spacings
    double cm;                   // cell measure (dx if nr > 1, times dt if nt > 1)
    double alpha1;               // initial step (delta lambda)^(-1/2) or user's
};

struct Tile {
    int32_t g;      // gather (-1: empty padding entry)
    int32_t r0, c0; // first output row, first output sample
    int32_t slot;   // partial-sum slot (a gather's slots are contiguous)
};

namespace tiling {

constexpr int kXcd = 8;
constexpr int kWavesPerBlock = 4;

inline int64_t round_up(int64_t v, int64_t m) { return (v + m - 1) / m * m; }

// One gather as the layout sees it.
struct GatherIn {
    int32_t nr, nt;
    double dx, dt;
    int64_t offset;  // in the caller's batch buffers
    int32_t rows;    // tile height
};

// The padded layout and tiling of a batch.
struct Layout {
    std::vector<GatherMeta> meta;
    std::vector<int> ntt, nst;  // time tiles and row strips per gather
    int32_t slots = 0;          // real tiles (partial-sum slots)
    int64_t padded_len = 0;     // elements of one padded field
};

// Gather g at padded offset poff (rows of ld = nt rounded up to 32 elements, so each
// row starts on a 128-byte line and each wave's 896-byte window is seven whole
// lines), cut into strips of `rows` receivers by time tiles of span = 56 V samples;
// its tiles own slots [tile_base, tile_base + ntiles).  alpha1 <= 0 selects
// (delta lambda)^(-1/2), lambda = 4/dx^2 + 4/dt^2 (an axis of length one drops its
// term).
inline Layout plan_layout(const std::vector<GatherIn>& gin, int span, double alpha1, double delta)
{
    Layout L;
    const int n = (int)gin.size();
    L.meta.resize(n);
    L.ntt.resize(n);
    L.nst.resize(n);
    int64_t poff = 0;
    int32_t slots = 0;
    for (int g = 0; g < n; ++g) {
        const GatherIn& d = gin[g];
        GatherMeta& m = L.meta[g];
        m.nr = d.nr;
        m.nt = d.nt;
        m.ld = (int32_t)round_up(d.nt, 32);
        m.poff = poff;
        m.uoff = d.offset;
        m.dx = d.dx;
        m.dt = d.dt;
        m.cm = (d.nr > 1 ? d.dx : 1.0) * (d.nt > 1 ? d.dt : 1.0);
        double lam = 0.0;
        if (d.nr > 1) lam += 4.0 / (d.dx * d.dx);
        if (d.nt > 1) lam += 4.0 / (d.dt * d.dt);
        m.alpha1 = alpha1 > 0.0 ? alpha1 : (lam > 0.0 ? 1.0 / std::sqrt(delta * lam) : 1.0);
        L.ntt[g] = (d.nt + span - 1) / span;
        m.rows = d.rows;
        L.nst[g] = (d.nr + m.rows - 1) / m.rows;
        m.tile_base = slots;
        m.ntiles = L.ntt[g] * L.nst[g];
        slots += m.ntiles;
        poff += round_up((int64_t)d.nr * m.ld, 64);
    }
    L.slots = slots;
    L.padded_len = poff;
    return L;
}

// Tile table of the selected gathers (sel[g] != 0).  Their strips, gather-major, are
// cut into kXcd runs of about equal cells, one per XCD (the kernel maps block b, which
// the hardware dispatches to XCD b % 8, to logical block (b % 8) * per + b / 8), and
// inside a run the tiles go gather by gather, strip by strip: neighbouring strips
// start together and march in opposite directions, so the rows they share are read at
// about the same moment, the second time from that XCD's L2.  Runs are padded with
// empty entries (g = -1) to a common length that is a multiple of the block size.
inline std::vector<Tile> layout_tiles(const Layout& L, int span, const std::vector<char>& sel)
{
    struct Strip {
        int g, st;
        int64_t cells;
    };
    std::vector<Strip> strips;
    int64_t total = 0;
    for (int g = 0; g < (int)L.meta.size(); ++g) {
        if (!sel[g]) continue;
        for (int st = 0; st < L.nst[g]; ++st) {
            const GatherMeta& m = L.meta[g];
            const int64_t c = (int64_t)std::min(m.rows, m.nr - st * m.rows) * m.nt;
            strips.push_back(Strip{g, st, c});
            total += c;
        }
    }
    std::vector<std::vector<Tile>> runs(kXcd);
    size_t s0 = 0;
    int64_t acc = 0;
    for (int x = 0; x < kXcd; ++x) {
        const int64_t goal = total * (x + 1) / kXcd;
        size_t s1 = s0;
        while (s1 < strips.size() && (x == kXcd - 1 || acc + strips[s1].cells / 2 < goal)) acc += strips[s1++].cells;
        for (size_t s = s0; s < s1; ++s) {
            const int g = strips[s].g, st = strips[s].st;
            const GatherMeta& m = L.meta[g];
            for (int tt = 0; tt < L.ntt[g]; ++tt)
                runs[x].push_back(Tile{g, st * m.rows, tt * span, m.tile_base + st * L.ntt[g] + tt});
        }
        s0 = s1;
    }
    size_t run_len = 0;
    for (auto& r : runs) run_len = std::max(run_len, r.size());
    run_len = (size_t)round_up((int64_t)std::max<size_t>(run_len, 1), kWavesPerBlock);
    std::vector<Tile> tiles;
    tiles.reserve(run_len * kXcd);
    for (auto& r : runs) {
        tiles.insert(tiles.end(), r.begin(), r.end());
        tiles.resize(tiles.size() + (run_len - r.size()), Tile{-1, 0, 0, 0});
    }
    return tiles;
}

// Split the selected gathers into up to nchains groups of about equal cells
// (largest first, each to the lighter group).  Returns one selection per group.
inline std::vector<std::vector<char>> split_chains(const std::vector<int64_t>& cells, const std::vector<char>& sel,
                                                   int nchains)
{
    const int n = (int)cells.size();
    std::vector<int> order;
    for (int g = 0; g < n; ++g)
        if (sel[g]) order.push_back(g);
    std::stable_sort(order.begin(), order.end(), [&](int x, int y) { return cells[x] > cells[y]; });
    const int nc = std::max(1, std::min((int)order.size(), nchains));
    std::vector<std::vector<char>> part(nc, std::vector<char>(n, 0));
    std::vector<int64_t> load(nc, 0);
    for (int g : order) {
        int k = 0;
        for (int j = 1; j < nc; ++j)
            if (load[j] < load[k]) k = j;
        part[k][g] = 1;
        load[k] += cells[g];
    }
    return part;
}

// Chains of launches for a table of `tiles` real tiles: up to max_chains once a launch
// is long enough for one chain's draining waves to overlap the other's next sweep;
// below kChainMinTiles a launch lasts about one wave's march whatever its size, two
// such launches barely overlap, and one chain over all of them is faster.
constexpr int64_t kChainMinTiles = 2048;
inline int chain_count(int64_t tiles, int max_chains) { return tiles >= kChainMinTiles ? max_chains : 1; }

// Finished gathers leave the sweep's tables once the running ones hold at most 15/16
// of the cells the tables cover (tiles keep their shape and slots, so no result
// changes; only the launch gets smaller).
inline bool narrow_now(int64_t live, int64_t table_cells) { return live > 0 && live * 16 <= table_cells * 15; }

}  // namespace tiling
}  // namespace emd
