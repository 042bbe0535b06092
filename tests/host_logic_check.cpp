// Invariants of the library's host-side logic (paper_1602_05650_amd/csrc/host_logic.hpp),
// built by test_host_logic_cpu.py with the address and undefined-behaviour sanitizers.
//   partition: the launch grid is n_tblocks x n_chunks, every source tile lies in exactly
//     one chunk, every target in exactly one target block, and the carved scratch holds
//     n_chunks x 3 x n_t partials within the bytes the workspace is sized for;
//   allocator: random alloc/release sequences against a byte map (no overlap, ranges
//     inside the capacity, free ranges merged, everything free again at the end).
#include <stdio.h>
#include <stdlib.h>

#include <random>
#include <vector>

#include "host_logic.hpp"

using namespace stokes;

static int failures = 0;
#define CHECK(c, ...)                                      \
    do {                                                   \
        if (!(c)) {                                        \
            ++failures;                                    \
            if (failures < 20) {                           \
                fprintf(stderr, "FAIL %s:%d: %s: ", __FILE__, __LINE__, #c); \
                fprintf(stderr, __VA_ARGS__);              \
                fprintf(stderr, "\n");                     \
            }                                              \
        }                                                  \
    } while (0)

static void check_partition(int64_t n_t, int64_t n_s, int R, int64_t tb, int min_small) {
    const Partition P = make_partition(n_t, n_s, R, tb, min_small);
    const int64_t n_tiles = (n_s + TILE - 1) / TILE;
    CHECK(P.n_tiles == n_tiles, "n_t %lld n_s %lld", (long long)n_t, (long long)n_s);
    CHECK((int64_t)P.n_tblocks * 4 * 64 * R >= n_t, "targets not covered");
    CHECK(n_t == 0 || (int64_t)(P.n_tblocks - 1) * 4 * 64 * R < n_t, "empty target block");
    if (n_t == 0 || n_s == 0) {
        CHECK(P.n_chunks == 0, "empty problem has chunks");
        return;
    }
    CHECK(P.n_chunks >= 1 && P.tiles_per_chunk >= 1, "no chunk");
    // tiles [c tpc, min((c+1) tpc, n_tiles)) for chunk c: a partition of the tiles
    CHECK((int64_t)P.n_chunks * P.tiles_per_chunk >= n_tiles, "tiles beyond the last chunk");
    CHECK((int64_t)(P.n_chunks - 1) * P.tiles_per_chunk < n_tiles, "empty chunk");
    CHECK(P.grid() == (int64_t)P.n_tblocks * P.n_chunks && P.grid() <= INT32_MAX, "grid");
    // the last workgroup's chunk index is within the partial rows
    const int64_t last = P.grid() - 1;
    CHECK(last / P.n_tblocks == P.n_chunks - 1, "workgroup chunk index");
    for (size_t s32b : {(size_t)0, (size_t)32, (size_t)48}) {
        const SumLayout L = sum_layout(n_s, n_t, 7, 80, 64, s32b, P.n_chunks);
        const size_t offs[] = {L.tiles, L.s64, L.s32, L.near_t, L.excl, L.fbounds, L.partial, L.counters, L.flag};
        for (size_t i = 0; i < sizeof(offs) / sizeof(offs[0]); ++i) CHECK(offs[i] % 256 == 0, "alignment");
        for (size_t i = 1; i < sizeof(offs) / sizeof(offs[0]); ++i) CHECK(offs[i] >= offs[i - 1], "order");
        CHECK(L.counters - L.partial >= (size_t)P.n_chunks * 3 * n_t * 8, "partial rows do not fit");
        CHECK(L.s64 - L.tiles >= (size_t)n_tiles * 80 && L.near_t - L.s32 >= (size_t)n_s * s32b, "packs");
        CHECK(L.end <= L.bytes, "layout beyond the workspace size");
    }
}

static void check_allocator(unsigned seed) {
    std::mt19937_64 rng(seed);
    const size_t cap = (size_t)(1 + rng() % 64) << 16;
    RangeAllocator A;
    A.reset(cap + (rng() % 255));
    CHECK(A.capacity() == cap, "capacity rounding");
    std::vector<unsigned char> owner(cap / 256, 0);
    std::vector<std::pair<size_t, size_t>> live;   // (offset, bytes)
    for (int step = 0; step < 4000; ++step) {
        if (live.empty() || rng() % 3 != 0) {
            const size_t want = rng() % 5 == 0 ? 0 : 1 + rng() % (cap / 8);
            const size_t off = A.alloc(want);
            if (off == SIZE_MAX) {
                // first fit fails only if no free range is large enough
                const size_t need = std::max<size_t>(256, (want + 255) & ~size_t(255));
                for (auto& f : A.free_ranges()) CHECK(f.second < need, "fit refused");
                continue;
            }
            const size_t len = std::max<size_t>(256, (want + 255) & ~size_t(255));
            CHECK(off % 256 == 0 && off + len <= cap, "range outside the arena");
            for (size_t b = off / 256; b < (off + len) / 256 && b < owner.size(); ++b) {
                CHECK(owner[b] == 0, "overlap at block %zu", b);
                owner[b] = 1;
            }
            live.push_back({off, len});
        } else {
            const size_t i = rng() % live.size();
            CHECK(A.release(live[i].first), "release of a live range");
            for (size_t b = live[i].first / 256; b < (live[i].first + live[i].second) / 256; ++b) owner[b] = 0;
            live.erase(live.begin() + i);
            CHECK(!A.release(cap + 256), "release of an unknown offset");
        }
        // free ranges: disjoint, merged (no two adjacent), and with the used ones tile the arena
        size_t prev_end = SIZE_MAX, total = 0;
        for (auto& f : A.free_ranges()) {
            CHECK(prev_end != f.first, "adjacent free ranges not merged");
            prev_end = f.first + f.second;
            total += f.second;
        }
        for (auto& u : A.used_ranges()) total += u.second;
        CHECK(total == cap, "free + used != capacity");
    }
    for (auto& l : live) A.release(l.first);
    CHECK(A.free_ranges().size() == 1 && A.free_ranges().begin()->second == cap, "not all free at the end");
}

int main() {
    const int64_t sizes[] = {0, 1, 2, 31, 32, 33, 63, 64, 65, 255, 256, 257, 1000, 4095, 4096, 4097,
                             32768, 38912, 131072, 262144, 548864, 1 << 21};
    int n = 0;
    for (int64_t nt : sizes)
        for (int64_t ns : sizes)
            for (int R : {1, 2, 4})
                for (int64_t tb : {(int64_t)1, (int64_t)4096, TARGET_BLOCKS, (int64_t)1 << 20})
                    for (int ms : {1, MIN_TILES_PER_CHUNK}) {
                        check_partition(nt, ns, R, tb, ms);
                        ++n;
                    }
    for (unsigned seed = 0; seed < 40; ++seed) check_allocator(seed);
    printf("%d partitions, 40 allocator sequences, %d failures\n", n, failures);
    return failures ? 1 : 0;
}
