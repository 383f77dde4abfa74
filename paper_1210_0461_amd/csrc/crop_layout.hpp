// LDS layout of a staged chunk of transactions, shared by the device code
// (crop_enum.hpp) and the host's launch checks.  Plain C++: it also builds
// with a host compiler, so its alignment and bounds can be tested without a
// GPU.
#pragma once
#include <stddef.h>
#include <stdint.h>

#ifndef __HIPCC__
#ifndef __host__
#define __host__
#endif
#ifndef __device__
#define __device__
#endif
#endif

namespace crop {

// Word offsets of a chunk image placed after `lead` 32-bit words: xh (two
// words per entry, 8-byte aligned for its 64-bit LDS loads), then w and perm
// (u16 each, each padded to an even count of u16 so the next array starts on
// a word), then the 64 bucket words that take 32-bit LDS atomics.
struct TxLayout {
    size_t xh, w, perm, bucket, end;
};

__host__ __device__ inline TxLayout tx_layout(uint32_t lead, uint32_t max_items)
{
    TxLayout t;
    const size_t half = ((size_t)max_items + 1) / 2;  // words of one padded u16 array
    t.xh = ((size_t)lead + 1) & ~(size_t)1;
    t.w = t.xh + 2 * (size_t)max_items;
    t.perm = t.w + half;
    t.bucket = t.perm + half;
    t.end = t.bucket + 64;
    return t;
}

__host__ __device__ inline size_t tx_lds_words(uint32_t lead, uint32_t max_items)
{
    return tx_layout(lead, max_items).end;
}

// The properties the kernels rely on, checked on the host before a launch
// with `smem_bytes` of dynamic LDS: 64-bit alignment of xh, no overlap of
// the arrays (each at least as long as its entries need), and the whole
// image inside the dynamic allocation.
__host__ __device__ inline bool tx_layout_ok(uint32_t lead, uint32_t max_items, size_t smem_bytes)
{
    const TxLayout t = tx_layout(lead, max_items);
    if (t.xh % 2 != 0 || t.xh < lead) return false;
    if (t.w < t.xh + 2 * (size_t)max_items) return false;
    if (2 * (t.perm - t.w) < max_items || 2 * (t.bucket - t.perm) < max_items) return false;
    if (t.end != t.bucket + 64) return false;
    return 4 * t.end <= smem_bytes;
}

// LDS image of a chunk for windowed enumeration (an owner's share of the
// hash space), after `lead` 32-bit words: hist, the (rows << kb) + 1
// exclusive starts of every (row, h_b bucket); yh, (item, h_b) of each entry
// in (row, bucket) order, 8-byte aligned; row, the chunk row of each sorted
// entry (u16, padded to a whole word).
struct WinLayout {
    size_t hist, yh, row, rin, end;
};

__host__ __device__ inline WinLayout win_layout(uint32_t lead, uint32_t rows, uint32_t kb,
                                                uint32_t max_items)
{
    WinLayout t;
    t.hist = lead;
    const size_t nh = ((size_t)rows << kb) + 1;
    t.yh = (t.hist + nh + 1) & ~(size_t)1;
    t.row = t.yh + 2 * (size_t)max_items;
    t.rin = t.row + ((size_t)max_items + 1) / 2;
    t.end = t.rin + ((size_t)max_items + 1) / 2;
    return t;
}

__host__ __device__ inline bool win_layout_ok(uint32_t lead, uint32_t rows, uint32_t kb,
                                              uint32_t max_items, size_t smem_bytes)
{
    const WinLayout t = win_layout(lead, rows, kb, max_items);
    if (t.hist < lead || t.yh % 2 != 0) return false;
    if (t.yh < t.hist + ((size_t)rows << kb) + 1) return false;
    if (t.row < t.yh + 2 * (size_t)max_items) return false;
    if (2 * (t.rin - t.row) < max_items || 2 * (t.end - t.rin) < max_items) return false;
    if (rows > 65535 || max_items > 65535) return false;  // u16 rows and positions
    return 4 * t.end <= smem_bytes;
}

// LDS image of a sub-batch of the region route (k_sb_route): hist, the
// NB + 1 bin counters (then their exclusive starts) and a discard counter;
// ro and tp, the rows + 1
// item offsets and term prefixes of its transactions; xh, (item, h_b) of
// each of its items, 8-byte aligned; keys, its terms sorted by bin, 16-byte
// aligned (they leave LDS in 16-byte loads).  All offsets in 32-bit words.
struct SbLayout {
    uint32_t hist, ro, tp, xh, keys, end;
};

__host__ __device__ inline SbLayout sb_layout(uint32_t NB, uint32_t max_rows, uint32_t max_items,
                                              uint32_t max_terms, uint32_t key_bytes)
{
    SbLayout t;
    t.hist = 0;
    t.ro = NB + 2;
    t.tp = t.ro + max_rows + 1;
    t.xh = (t.tp + max_rows + 1 + 1) & ~1u;
    t.keys = (t.xh + 2 * max_items + 3) & ~3u;  // 16-byte loads of the sorted keys
    t.end = t.keys + max_terms * (key_bytes / 4);
    return t;
}

// What k_sb_route relies on, checked on the host before its launch with
// `smem_bytes` of dynamic LDS: the arrays in order without overlap, xh and
// 64-bit keys 8-byte aligned, the image inside the allocation, and at most
// 65,535 terms (bin ranks and region offsets are 16-bit) and 8,192 bins.
__host__ __device__ inline bool sb_layout_ok(uint32_t NB, uint32_t max_rows, uint32_t max_items,
                                             uint32_t max_terms, uint32_t key_bytes,
                                             size_t smem_bytes)
{
    if (key_bytes != 4 && key_bytes != 8) return false;
    if (NB == 0 || NB > 8192 || max_terms > 65535 || max_rows == 0) return false;
    const SbLayout t = sb_layout(NB, max_rows, max_items, max_terms, key_bytes);
    if (t.ro < t.hist + NB + 2 || t.tp < t.ro + max_rows + 1) return false;
    if (t.xh < t.tp + max_rows + 1 || t.xh % 2 != 0) return false;
    if (t.keys < t.xh + 2 * (size_t)max_items || t.keys % 4 != 0) return false;
    if (max_terms % (16 / key_bytes) != 0) return false;  // whole 16-byte stores
    if (t.end < t.keys + (size_t)max_terms * (key_bytes / 4)) return false;
    return 4 * (size_t)t.end <= smem_bytes;
}

}  // namespace crop
