// Reading a routing bin of the region route: bin b is one run in each
// sub-batch region (the region's keys are sorted by bin), so its keys are a
// concatenation of short runs scattered over the routed array.  With the
// non-empty runs listed in LDS (rb: routed position of a run's first key,
// rp: keys before it), sb_span maps 64 consecutive positions of the
// concatenation to routed positions, one per lane, so that a wavefront
// reads consecutive keys of a run with consecutive lanes.
#pragma once
#include "crop_device.hpp"

namespace crop {

// The run holding tile position c: the last r < nr with rp[r] <= c (c <
// rp[nr]).  Wavefront-uniform arguments: every lane reads the same words.
__device__ inline uint32_t sb_find_run(uint32_t c, uint32_t nr, const uint32_t *rp)
{
    uint32_t lo = 0, hi = nr;
    while (hi - lo > 1) {
        const uint32_t mid = (lo + hi) >> 1;
        if (rp[mid] <= c) lo = mid;
        else hi = mid;
    }
    return lo;
}

// Positions c + lane (lane = 0..63) of the tile: returns the routed position
// of this lane's key, valid when c + lane < rp[nr].  r0 is a run with
// rp[r0] <= c and rp[r0 + 1] >= c (the run of c, or of c - 1); on return it
// is the run of c + 63, ready for the span that starts at c + 64.  wflag is
// the wavefront's own 64 words, tag a value it has not yet written there
// (the run starts inside the span are marked, then counted with a ballot).
__device__ inline uint32_t sb_span(uint32_t c, uint32_t &r0, uint32_t nr, const uint32_t *rb,
                                   const uint32_t *rp, uint32_t *wflag, uint32_t tag)
{
    const uint32_t lane = lane_id();
    const uint32_t j = r0 + 1 + lane;
    if (j < nr) {
        const uint32_t d = rp[j] - c;  // rp[j] >= rp[r0 + 1] >= c
        if (d < (uint32_t)kWave) wflag[d] = tag;
    }
    // the marks of every lane are in LDS before any lane reads them back
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    const uint64_t m = __ballot(wflag[lane] == tag);
    const uint64_t upto = lane == kWave - 1 ? ~0ull : ((2ull << lane) - 1);
    uint32_t run = r0 + (uint32_t)__popcll(m & upto);
    r0 += (uint32_t)__popcll(m);
    run = run < nr ? run : nr - 1;  // lanes past the tile's end
    return rb[run] + (c + lane - rp[run]);
}

}  // namespace crop
