// Pieces shared by the two matrix-core forward kernels (fwd_mfma.hip: fp64 and
// fp32 operands; fwd_h16.hip: split 16-bit operands): the power-of-two scale
// helpers of the normalised half-precision form and the conflict-free phase
// plan of the end-of-block scatter into the output ring.
#pragma once

#include <stdint.h>

#include <hip/hip_runtime.h>

namespace sse {

// power of two s with m * s in [2^(t-1), 2^t) (1 for m = 0)
__device__ __forceinline__ double pow2_scale(double m, int t) {
    if (!(m > 0.0)) return 1.0;
    int e;
    frexp(m, &e);
    return ldexp(1.0, t - e);
}

// largest value over a full wave: butterflies inside each row of 16 lanes on
// the DPP network, then the four row results through scalar registers
__device__ __forceinline__ int wave_max(int v) {
    v = max(v, __builtin_amdgcn_update_dpp(v, v, 0xB1, 0xF, 0xF, false));   // quad_perm [1,0,3,2]
    v = max(v, __builtin_amdgcn_update_dpp(v, v, 0x4E, 0xF, 0xF, false));   // quad_perm [2,3,0,1]
    v = max(v, __builtin_amdgcn_update_dpp(v, v, 0x124, 0xF, 0xF, false));  // row_ror:4
    v = max(v, __builtin_amdgcn_update_dpp(v, v, 0x128, 0xF, 0xF, false));  // row_ror:8
    const int r0 = __builtin_amdgcn_readlane(v, 0), r1 = __builtin_amdgcn_readlane(v, 16);
    const int r2 = __builtin_amdgcn_readlane(v, 32), r3 = __builtin_amdgcn_readlane(v, 48);
    return max(max(r0, r1), max(r2, r3));
}

constexpr int ceil_log2(int x) {
    int e = 0;
    while ((1 << e) < x) ++e;
    return e;
}

// Phases of the end-of-block scatter into the output ring.  The GEMM rows are
// (k, w, re/im); a tile's contributions land on ring entries of the momenta k
// its rows carry, so tiles of different waves whose k sets are disjoint can add
// concurrently without touching the same entry; every entry then receives its
// additions in a fixed order and the fp64 sums are bitwise reproducible.
// Greedy first fit, own tiles before extra pairs.  C provides WAVES, OWN
// (waves that own a whole M-tile), XP (extra (M-tile, N-tile) pairs, one per
// wave), NT, MROWS and NWV (frequencies per momentum).
template <class C>
struct ScatterPlan {
    int own_phase[C::WAVES];
    int ext_phase[C::WAVES];
    int nphase;
    static constexpr uint32_t kmask(int mt) {
        uint32_t m = 0;
        for (int row = 16 * mt; row < 16 * mt + 16 && row < C::MROWS; ++row) m |= 1u << ((row >> 1) / C::NWV);
        return m;
    }
    constexpr ScatterPlan() : own_phase{}, ext_phase{}, nphase(0) {
        uint32_t used[2 * C::WAVES] = {};        // k set of each phase
        int owner[2 * C::WAVES][C::WAVES] = {};  // per phase: k set contributed by each wave
        for (int item = 0; item < 2 * C::WAVES; ++item) {
            const int w = item % C::WAVES;
            const bool ext = item >= C::WAVES;
            if (ext ? !(w < C::XP) : !(w < C::OWN)) {
                (ext ? ext_phase : own_phase)[w] = -1;
                continue;
            }
            const uint32_t m = kmask(ext ? C::WAVES + w / C::NT : w);
            int p = 0;
            for (;; ++p) {
                const uint32_t others = used[p] & ~(uint32_t)owner[p][w];
                if ((others & m) == 0) break;
            }
            used[p] |= m;
            owner[p][w] |= (int)m;
            (ext ? ext_phase : own_phase)[w] = p;
            if (p + 1 > nphase) nphase = p + 1;
        }
    }
};

}  // namespace sse
