// The spill between the two passes of a four-step transform: layout and
// the writer used by the last stage of a first pass.
#pragma once

#include "rsf_device.h"

namespace rsf {

// Spill layout: 8-column groups, float4 [template][k_a / 8][n_b][k_a % 8]:
// a group is one second-pass block, one contiguous run, and the eight
// consecutive k_a of a first-pass row fill one whole 128-byte line, which
// that row's workgroup writes alone.
constexpr int kGroupCols = kPassBCols;
static_assert(kGroupCols == 8, "the offsets below assume 8-column groups");

typedef float spill_v4 __attribute__((ext_vector_type(4)));

// Writer of the first pass's last stage: output k_a = j + r L1/R of the row
// transform, times the inter-pass twiddle W_N^{n_b k_a}, goes straight from
// registers to the spill.  The twiddle of butterfly j = tid + q NT is
// W^{n_b tid} (W^{n_b NT})^q, advanced once per call (calls come in q order),
// and steps by W^{n_b L1/R} along r.  The spill is written once and read once
// by the second pass.  When a launch's spill is larger than the last-level
// cache it cannot stay there until then, and the stores are non-temporal
// (NT), so that they do not displace cached lines; a smaller spill is stored
// normally and read back from the cache.
template <bool NT>
struct SpillSink {
    char* out;  // this template's spill (< 4 GiB, so byte offsets fit 32 bits)
    int LB, n_b, LR;
    float2 wq, w_step, w_lr;
    template <int R>
    __device__ __forceinline__ void put(int, int j, int, cp (&v)[R]) {
        // offsets and twiddles depend only on the thread and the plan; opaque
        // copies of j and w keep the compiler from hoisting all of them out
        // of the spindown loop (where they would be spilled)
        int jv = j;
        float2 w = wq;
        asm volatile("" : "+v"(jv), "+v"(w.x), "+v"(w.y));
#pragma unroll
        for (int r = 0; r < R; ++r) {
            const uint32_t k = (uint32_t)(jv + r * LR);
            const uint32_t off = (((k >> 3) * (uint32_t)LB + (uint32_t)n_b) * kGroupCols + (k & 7u)) * 16u;
            const cp u = cp_rot(v[r], w);
            if constexpr (NT)
                __builtin_nontemporal_store(spill_v4{u.x, u.y, u.z, u.w}, reinterpret_cast<spill_v4*>(out + off));
            else
                *reinterpret_cast<float4*>(out + off) = u;
            if (r + 1 < R) w = c_mul(w, w_lr);
        }
        wq = c_mul(wq, w_step);
    }
};

}  // namespace rsf
