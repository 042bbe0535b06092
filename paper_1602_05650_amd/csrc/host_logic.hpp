// Host-side arithmetic of libstokes.so that does not touch the GPU: the work
// partition of a sum, the carving of workspaces into aligned slices and the
// first-fit allocator of the serving arena.  Plain C++ (no HIP headers), so the
// CPU tests compile it on its own, with the address and undefined-behaviour
// sanitizers, and check its invariants.
#pragma once

#include <stddef.h>
#include <stdint.h>

#include <algorithm>
#include <iterator>
#include <map>

namespace stokes {

// ---- geometry of the kernel sums -----------------------------------------
constexpr int TILE = 32;      // sources per tile (one 32-node fiber in the benchmark geometries)
constexpr int BLOCK = 256;    // 4 waves per block
// Targets per lane (register blocking) of each pair kernel, and the number of
// blocks a launch aims for (many small work items keep all 256 CUs busy to
// the end; measured on gfx950: R = 1 with ~64k blocks is fastest for both
// precisions, because occupancy matters more here than reuse of the SGPR
// source operands).
constexpr int R_SL64 = 1, R_SL32 = 1, R_DL64 = 1, R_DL32 = 1;
constexpr int64_t TARGET_BLOCKS = 65536;
// Serving slots share the GPU with other requests, so each uses fewer chunks
// (less partial-sum memory per request).
constexpr int64_t TARGET_BLOCKS_SLOT = 4096;
constexpr int MIN_TILES_PER_CHUNK = 8;
// The double layer's (a pair costs more than a single-layer pair, so shorter chunks).
constexpr int MIN_TILES_PER_CHUNK_DL = 4;
constexpr int64_t SMALL_GRID = 8192;

// Bump allocator over a workspace buffer (256-byte aligned slices).
struct Carve {
    char* base;
    size_t off = 0;
    explicit Carve(void* b) : base(static_cast<char*>(b)) {}
    template <class T>
    T* take(size_t n) {
        off = (off + 255) & ~size_t(255);
        T* p = reinterpret_cast<T*>(base + off);
        off += n * sizeof(T);
        return p;
    }
    static size_t round(size_t b) { return (b + 255) & ~size_t(255); }
};

// Work partition of one sum: targets in waves of 64*R, sources in chunks of
// whole tiles.  Depends only on the problem sizes (bitwise reproducibility).
// A launch has n_tblocks * n_chunks workgroups, and chunk k writes partial
// row k of n_chunks: both follow from this one struct.
struct Partition {
    int R;
    int64_t n_t;
    int32_t n_tiles;
    int32_t tiles_per_chunk;
    int32_t n_chunks;
    int32_t n_tblocks;
    int64_t grid() const { return (int64_t)n_tblocks * n_chunks; }
};

// min_tiles_small: least source tiles per chunk when there are fewer than 64
// target blocks (a problem too small to fill the chip with target blocks alone);
// min_tiles_large: the same with 64 target blocks or more.
inline Partition make_partition(int64_t n_t, int64_t n_s, int R, int64_t target_blocks = TARGET_BLOCKS,
                                int min_tiles_small = 1, int min_tiles_large = MIN_TILES_PER_CHUNK) {
    Partition p{};
    p.R = R;
    p.n_t = n_t;
    p.n_tiles = (int32_t)((n_s + TILE - 1) / TILE);
    const int64_t waves = (n_t + 64 * R - 1) / (64 * R);
    p.n_tblocks = (int32_t)((waves + 3) / 4);
    if (p.n_tiles == 0 || n_t == 0) {
        p.tiles_per_chunk = 1;
        p.n_chunks = 0;
        return p;
    }
    // few target blocks (a small problem): aim at SMALL_GRID workgroups, enough to fill
    // the chip, rather than target_blocks, which would cut the sources into one-tile
    // chunks and write a partial row per tile
    if (p.n_tblocks < 64) target_blocks = std::min<int64_t>(target_blocks, SMALL_GRID);
    int64_t ch = (target_blocks + p.n_tblocks - 1) / p.n_tblocks;
    // few target blocks (a small, latency-bound problem): shorter chunks
    const int64_t min_tiles = p.n_tblocks >= 64 ? min_tiles_large : min_tiles_small;
    ch = std::min<int64_t>(ch, std::max<int64_t>(1, p.n_tiles / min_tiles));
    ch = std::max<int64_t>(1, std::min<int64_t>(ch, p.n_tiles));
    p.tiles_per_chunk = (int32_t)((p.n_tiles + ch - 1) / ch);
    p.n_chunks = (p.n_tiles + p.tiles_per_chunk - 1) / p.tiles_per_chunk;
    return p;
}

// Byte offsets of the scratch of one direct sum, in carve order: tiles, FP64
// source pack, FP32 source pack, near thresholds, exclusion ranges, fiber bounds,
// chunk partials (n_chunks x 3 x n_t doubles), counters, flag.  `bytes` bounds
// the end of the last slice (every slice 256-aligned).
struct SumLayout {
    size_t tiles, s64, s32, near_t, excl, fbounds, partial, counters, flag, end, bytes;
};
inline SumLayout sum_layout(int64_t n_s, int64_t n_t, int32_t n_fib, size_t tile_b, size_t s64b,
                            size_t s32b, int32_t n_chunks) {
    const int64_t n_tiles = (n_s + TILE - 1) / TILE;
    SumLayout L{};
    Carve c(nullptr);
    auto at = [&](size_t n, size_t elem) {
        c.off = (c.off + 255) & ~size_t(255);
        const size_t o = c.off;
        c.off += n * elem;
        return o;
    };
    L.tiles = at(n_tiles, tile_b);
    L.s64 = at(n_s, s64b);
    L.s32 = at(s32b ? n_s : 0, s32b);
    L.near_t = at(n_s, sizeof(float));
    L.excl = at(n_t, 8);
    L.fbounds = at((size_t)std::max<int32_t>(n_fib, 1), 8);
    L.partial = at((size_t)n_chunks * 3 * n_t, sizeof(double));
    L.counters = at(4, 8);
    L.flag = at(4, 4);
    L.end = c.off;
    L.bytes = L.end + 256;
    return L;
}

// First-fit allocator of byte ranges [0, capacity), offsets 256-aligned; adjacent
// free ranges are merged on release.  The serving arena places requests with it.
class RangeAllocator {
public:
    void reset(size_t capacity) {
        size_ = capacity & ~size_t(255);
        free_.clear();
        used_.clear();
        if (size_) free_[0] = size_;
    }
    // Offset of a free range of at least `bytes`, or SIZE_MAX.
    size_t alloc(size_t bytes) {
        bytes = (bytes + 255) & ~size_t(255);
        if (bytes == 0) bytes = 256;
        for (auto it = free_.begin(); it != free_.end(); ++it) {
            if (it->second >= bytes) {
                const size_t off = it->first, len = it->second;
                free_.erase(it);
                if (len > bytes) free_[off + bytes] = len - bytes;
                used_[off] = bytes;
                return off;
            }
        }
        return SIZE_MAX;
    }
    // Releases the range that alloc returned at `off`; false if there is none.
    bool release(size_t off) {
        auto u = used_.find(off);
        if (u == used_.end()) return false;
        size_t len = u->second;
        used_.erase(u);
        auto nx = free_.lower_bound(off);   // first free range after the released one
        if (nx != free_.end() && nx->first == off + len) {
            len += nx->second;
            nx = free_.erase(nx);
        }
        if (nx != free_.begin()) {
            auto pv = std::prev(nx);
            if (pv->first + pv->second == off) {
                pv->second += len;
                return true;
            }
        }
        free_[off] = len;
        return true;
    }
    // Would alloc(bytes) succeed now?
    bool fits(size_t bytes) const {
        bytes = std::max<size_t>(256, (bytes + 255) & ~size_t(255));
        for (const auto& f : free_)
            if (f.second >= bytes) return true;
        return false;
    }
    size_t capacity() const { return size_; }
    const std::map<size_t, size_t>& free_ranges() const { return free_; }
    const std::map<size_t, size_t>& used_ranges() const { return used_; }

private:
    size_t size_ = 0;
    std::map<size_t, size_t> free_, used_;
};

}  // namespace stokes
