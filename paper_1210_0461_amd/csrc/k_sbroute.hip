// Term routing by sorted sub-batch regions.
//
// Every term of the stream goes to its routing bin by the consistent hash
// (Section 5: h(x, y) = h_a(x) + h_b(y) mod 2^32; Section 6, Theorem 1:
// owners hold equal intervals of the hash space, and a bin is a finer
// interval inside one).  A sub-batch is a run of consecutive transactions
// with at most max_terms terms.  Its workgroup enumerates every pair x < y,
// takes each key's rank inside its bin with one LDS atomic, counting-sorts
// the keys by bin in LDS and writes them as one contiguous region of the
// routed array, together with a row of 16-bit bin starts inside the region.
// The region of sub-batch s begins at sb_term[s], the stream's term prefix
// with every region rounded up to whole 16-byte groups of keys, known from
// the offsets alone: no count pass and no count matrix are needed, and every
// HBM write is a 16-byte store of consecutive keys.
//
// Bin b is then one run per region.  k_sb_headers transposes the start rows
// (so a bin's starts are contiguous) and sums them over the sub-batches: the
// sum of the starts of bin b is the number of keys in bins below b, i.e. the
// offset of bin b's results in a bin-contiguous layout.  The exact
// aggregation reads each bin's runs where they are (k_aggregate_regions).
// The route takes packed 32-bit keys (fewer than 2^16 items); 64-bit keys
// stay on the chunk route.
#include "crop_device.hpp"
#include "crop_enum.hpp"
#include "crop_internal.hpp"
#include "crop_layout.hpp"

namespace crop {

namespace {

constexpr int kSbBS = 1024;  // threads of a route workgroup

// One sub-batch: rows [sb_row[s], sb_row[s+1]); its region of the routed
// array starts at sb_base[s], a multiple of four keys.  Thread t enumerates
// terms [t Q, t Q + Q) of the sub-batch in row-major order ((a, b) with
// a < b over the positions of a row), so a thread's terms are consecutive
// pairs of one or two rows; the LDS read of the next term's partner is
// issued before the current term is hashed and ranked.  DROP: an owned
// share, where most terms fall outside the run's bins and take no rank.
template <int BS, int Q, class KeyT, bool DROP>
__global__ void __launch_bounds__(BS)
k_sb_route(const uint32_t *__restrict__ off, const uint32_t *__restrict__ items, HashParams hp,
           const SbSeg *__restrict__ segs, const uint32_t *__restrict__ sub_seg, SbLayout lay,
           const uint32_t *__restrict__ sb_row, const uint32_t *__restrict__ sb_base,
           KeyT *__restrict__ routed, uint16_t *__restrict__ hdr)
{
    constexpr uint32_t KPQ = 16 / sizeof(KeyT);  // keys per 16-byte store
    extern __shared__ uint32_t smem[];
    __shared__ uint32_t s_tmp[BS / kWave + 1];
    uint32_t *hist = smem + lay.hist;
    uint32_t *ro = smem + lay.ro;
    uint32_t *tp = smem + lay.tp;
    uint2 *xh = reinterpret_cast<uint2 *>(smem + lay.xh);
    KeyT *sorted = reinterpret_cast<KeyT *>(smem + lay.keys);

    const uint32_t s = blockIdx.x;
    // the sub-batch's segment: its bins, and where its header row goes
    const SbSeg &sg = segs[sub_seg ? sub_seg[s] : 0u];
    const BinMap bm = sg.bm;
    const uint32_t NB = sg.NB;
    uint16_t *hrow = hdr + sg.hdr0 + (size_t)(s - sg.sub0) * sg.hs;
    const uint32_t r0 = sb_row[s], R = sb_row[s + 1] - r0;
    const uint32_t t0 = sb_base[s];
    const uint32_t p0 = off[r0];
    const uint32_t m = off[r0 + R] - p0;
    for (uint32_t i = threadIdx.x; i <= R; i += BS) ro[i] = off[r0 + i] - p0;
    for (uint32_t k = threadIdx.x; k < m; k += BS) {
        const uint32_t x = items[p0 + k];
        xh[k] = make_uint2(x, hash_b(hp, x));
    }
    for (uint32_t b = threadIdx.x; b < NB; b += BS) hist[b] = 0;
    __syncthreads();
    for (uint32_t i = threadIdx.x; i < R; i += BS) {
        const uint32_t L = ro[i + 1] - ro[i];
        tp[i] = L * (L - 1) / 2;
    }
    __syncthreads();
    lds_exclusive_scan<BS>(tp, R, s_tmp);
    const uint32_t nt = tp[R];

    // Each term takes its rank inside its bin with one LDS atomic, not waited
    // for until the placement: nothing in the loop needs its result.  A full
    // run issues it for every term (a term past the thread's count counts in
    // the discard counter hist[NB + 1]); an owned share only for its own
    // terms, since the discarded majority would queue on that one word.
    KeyT key[Q];
    uint32_t bins[Q], rank[Q];
    const uint32_t tb = threadIdx.x * Q;
    const uint32_t nv = tb < nt ? min((uint32_t)Q, nt - tb) : 0u;  // this thread's terms
    if (nv) {
        // the row of term tb: tp[row] <= tb < tp[row + 1]
        uint32_t lo = 0, hi = R;
        while (hi - lo > 1) {
            const uint32_t mid = (lo + hi) >> 1;
            if (tp[mid] <= tb) lo = mid;
            else hi = mid;
        }
        uint32_t row = lo, base = ro[row], L = ro[row + 1] - base;
        uint32_t k = tb - tp[row], a = 0;
        while (k >= L - 1 - a) {
            k -= L - 1 - a;
            ++a;
        }
        uint32_t b = a + 1 + k;
        // x: the first item of the current term, x1: the item after it (the
        // x of the next a), yh: the current term's partner and its h_b
        uint32_t x = xh[base + a].x, x1 = xh[base + a + 1].x;
        uint32_t ha = hash_a(hp, x);
        uint2 yh = xh[base + b];
#pragma unroll
        for (int u = 0; u < Q; ++u) {
            // the next term (a, b + 1), else (a + 1, a + 2), else the first
            // pair of the next row with two or more items (one exists: terms
            // remain); its partner's read is issued before this term's rank
            uint2 yn = yh;
            uint32_t nx = x, nha = ha;
            if ((uint32_t)u + 1 < nv) {
                if (++b == L) {
                    ++a;
                    b = a + 1;
                    if (b == L) {
                        do {
                            ++row;
                            base = ro[row];
                            L = ro[row + 1] - base;
                        } while (L < 2);
                        a = 0;
                        b = 1;
                        nx = xh[base].x;
                    } else {
                        nx = x1;
                    }
                    nha = hash_a(hp, nx);
                }
                yn = xh[base + b];
            }
            const uint32_t bin = bm.local(ha + yh.y);
            bins[u] = ((uint32_t)u < nv && bin < NB) ? bin : NB + 1;
            key[u] = pack_key<KeyT>(x, yh.x);
            if (DROP)
                rank[u] = bins[u] < NB ? atomicAdd(&hist[bins[u]], 1u) : 0u;
            else
                rank[u] = atomicAdd(&hist[bins[u]], 1u);
            yh = yn;
            x = nx;
            ha = nha;
            if (b == a + 1) x1 = yh.x;
        }
    } else {
#pragma unroll
        for (int u = 0; u < Q; ++u) {
            bins[u] = NB + 1;
            key[u] = 0;
            rank[u] = 0;
        }
    }
    __syncthreads();
    lds_exclusive_scan<BS>(hist, NB, s_tmp);  // hist[NB] = kept terms
    // every slot is read before any key is placed
    uint32_t pos[Q];
#pragma unroll
    for (int u = 0; u < Q; ++u) pos[u] = bins[u] < NB ? hist[bins[u]] + rank[u] : kEmpty32;
#pragma unroll
    for (int u = 0; u < Q; ++u)
        if (pos[u] != kEmpty32) sorted[pos[u]] = key[u];
    __syncthreads();
    // the region in 16-byte stores (its tail past the kept keys is padding)
    const uint32_t kept = hist[NB];
    const uint32_t nq = (kept + KPQ - 1) / KPQ;
    const uint4 *src = reinterpret_cast<const uint4 *>(sorted);
    uint4 *dst = reinterpret_cast<uint4 *>(routed + t0);
    constexpr uint32_t QPT = Q / KPQ;  // 16-byte groups per thread: BS QPT = the LDS keys
    uint4 v[QPT];
#pragma unroll
    for (uint32_t j = 0; j < QPT; ++j) v[j] = src[threadIdx.x + j * BS];
#pragma unroll
    for (uint32_t j = 0; j < QPT; ++j) {
        const uint32_t i = threadIdx.x + j * BS;
        if (i < nq) dst[i] = v[j];
    }
    for (uint32_t b = threadIdx.x; b <= NB; b += BS) hrow[b] = (uint16_t)hist[b];
}

// The segment of header tile (or bin) `t`: the last segment whose first
// tile (bin) is at most t.  field: tile0 or bin0.
template <class F>
__device__ inline uint32_t seg_of(const SbSeg *segs, uint32_t n_seg, uint32_t t, F first)
{
    uint32_t lo = 0, hi = n_seg;
    while (hi - lo > 1) {
        const uint32_t mid = (lo + hi) >> 1;
        if (first(segs[mid]) <= t) lo = mid;
        else hi = mid;
    }
    return lo;
}

// Tiles of 64 sub-batches x 64 bin starts of one segment (block b: tile
// b - tile0 of its segment, bin tiles first): hdrT[p][s] = hdr[s][p] for
// p <= NB, and tsum[t][p] = tile row t's sum of hdr[s][p] (k_sb_tile_scan
// adds them up).
__global__ void __launch_bounds__(256)
k_sb_headers(const uint16_t *__restrict__ hdr, const SbSeg *__restrict__ segs, uint32_t n_seg,
             uint16_t *__restrict__ hdrT, uint32_t *__restrict__ tsum)
{
    __shared__ uint16_t tile[64][66];
    __shared__ uint32_t part[4][64];
    const SbSeg sg = segs[seg_of(segs, n_seg, blockIdx.x, [](const SbSeg &x) { return x.tile0; })];
    const uint32_t local = blockIdx.x - sg.tile0;
    const uint32_t NB = sg.NB, n_sub = sg.n_sub;
    const uint32_t b0 = (local % sg.btiles) * 64, st = local / sg.btiles, s0 = st * 64;
    const uint16_t *h = hdr + sg.hdr0;
    uint16_t *hT = hdrT + sg.hdrT0;
    const uint32_t c = threadIdx.x & 63, q = threadIdx.x >> 6;
    uint32_t sum = 0;
    for (uint32_t r = q; r < 64; r += 4) {
        const uint32_t s = s0 + r, b = b0 + c;
        uint16_t v = 0;
        if (s < n_sub && b <= NB) v = h[(size_t)s * sg.hs + b];
        tile[r][c] = v;
        sum += v;
    }
    part[q][c] = sum;
    __syncthreads();
    if (q == 0 && b0 + c <= NB)
        tsum[sg.tsum0 + (size_t)st * (NB + 1) + b0 + c] =
            part[0][c] + part[1][c] + part[2][c] + part[3][c];
    for (uint32_t k = q; k < 64; k += 4) {
        const uint32_t b = b0 + k, s = s0 + c;
        if (b <= NB && s < n_sub) hT[(size_t)b * sg.hts + s] = tile[c][k];
    }
}

// bin_off[b] for b <= NBtot: its segment's kept keys before it (key0) plus
// the sum of its bin starts over the segment's header tiles; the sum of the
// starts of bin p over every sub-batch is the number of the segment's keys
// in bins below p.  bin_off[NBtot] is the last segment's end (its start
// column NB).
__global__ void __launch_bounds__(256)
k_sb_tile_scan(const uint32_t *__restrict__ tsum, const SbSeg *__restrict__ segs, uint32_t n_seg,
               uint32_t NBtot, uint32_t *__restrict__ bin_off)
{
    const uint32_t b = blockIdx.x * 256 + threadIdx.x;
    if (b > NBtot) return;
    const uint32_t g = b < NBtot ? seg_of(segs, n_seg, b, [](const SbSeg &x) { return x.bin0; })
                                 : n_seg - 1;
    const SbSeg sg = segs[g];
    const uint32_t p = b < NBtot ? b - sg.bin0 : sg.NB;
    const uint32_t n_tiles = (sg.n_sub + 63) / 64;
    const uint32_t *ts = tsum + sg.tsum0 + p;
    uint32_t run = 0;
    for (uint32_t t0 = 0; t0 < n_tiles; t0 += 8) {  // eight loads in flight
        uint32_t v[8];
#pragma unroll
        for (uint32_t k = 0; k < 8; ++k)
            v[k] = t0 + k < n_tiles ? ts[(size_t)(t0 + k) * (sg.NB + 1)] : 0u;
#pragma unroll
        for (uint32_t k = 0; k < 8; ++k) run += v[k];
    }
    bin_off[b] = sg.key0 + run;
}

}  // namespace

size_t sb_route_smem_bytes(uint32_t NB, uint32_t max_rows, uint32_t max_items,
                           uint32_t max_terms, uint32_t key_bytes)
{
    return 4 * (size_t)sb_layout(NB, max_rows, max_items, max_terms, key_bytes).end;
}

// Terms per route thread: the sub-batch holds kSbBS * Q terms at most.
uint32_t sb_threads() { return kSbBS; }

hipError_t launch_sb_route(const crop_ctx *c, hipStream_t s)
{
    const RoutePlan &pl = c->plan;
    const SbPlan &sp = c->sb;
    const uint32_t kb = c->in.wide_keys ? 8 : 4;
    const SbLayout lay = sb_layout(sp.NBmax, sp.max_rows, sp.max_items, sp.max_terms, kb);
    const size_t sm = 4 * (size_t)lay.end;
    if (!sb_layout_ok(sp.NBmax, sp.max_rows, sp.max_items, sp.max_terms, kb, sm))
        return hipErrorInvalidConfiguration;
    const uint32_t Q = sp.max_terms / kSbBS;
    if (Q * kSbBS != sp.max_terms) return hipErrorInvalidConfiguration;
    const uint32_t *row = c->sb_row.as<uint32_t>(), *term = c->sb_term.as<uint32_t>();
    const SbSeg *segs = c->sb_seg.as<SbSeg>();
    const uint32_t *sub_seg = sp.segs.size() > 1 ? c->sb_subseg.as<uint32_t>() : nullptr;
    uint16_t *hdr = c->sb_hdr.as<uint16_t>();
    const bool drop = pl.nu < pl.M;  // an owned share (one segment)
#define SB_LAUNCH(QQ, KT, DR)                                                                \
    hipLaunchKernelGGL((k_sb_route<kSbBS, QQ, KT, DR>), dim3(sp.n_sub), dim3(kSbBS), sm, s,   \
                       c->in.off, c->in.items, c->hp, segs, sub_seg, lay, row, term,          \
                       c->routed.as<KT>(), hdr)
    if (c->in.wide_keys) return hipErrorInvalidConfiguration;  // packed keys only
    if (Q == 16 && drop)
        SB_LAUNCH(16, uint32_t, true);
    else if (Q == 16)
        SB_LAUNCH(16, uint32_t, false);
    else if (Q == 24 && drop)
        SB_LAUNCH(24, uint32_t, true);
    else if (Q == 24)
        SB_LAUNCH(24, uint32_t, false);
    else
        return hipErrorInvalidConfiguration;
#undef SB_LAUNCH
    return hipGetLastError();
}

// bin_off of every bin of the run (pl.NB of them) and its end.
hipError_t launch_sb_headers(const crop_ctx *c, hipStream_t s)
{
    const RoutePlan &pl = c->plan;
    const SbPlan &sp = c->sb;
    uint32_t *bin_off = c->bin_off.as<uint32_t>();
    if (sp.n_sub == 0 || sp.segs.empty()) return launch_zero32(bin_off, pl.NB + 1, s);
    const uint32_t n_seg = (uint32_t)sp.segs.size();
    const SbSeg *segs = c->sb_seg.as<SbSeg>();
    if (sp.n_tiles)
        hipLaunchKernelGGL(k_sb_headers, dim3(sp.n_tiles), dim3(256), 0, s,
                           c->sb_hdr.as<uint16_t>(), segs, n_seg, c->sb_hdrT.as<uint16_t>(),
                           c->sb_tsum.as<uint32_t>());
    hipLaunchKernelGGL(k_sb_tile_scan, dim3((pl.NB + 1 + 255) / 256), dim3(256), 0, s,
                       c->sb_tsum.as<uint32_t>(), segs, n_seg, pl.NB, bin_off);
    return hipGetLastError();
}

}  // namespace crop
