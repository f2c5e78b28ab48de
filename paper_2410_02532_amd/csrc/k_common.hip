// k_common.hip -- the kernels that are not templates: the adaptive step's
// control decision, the per-round-trip energy reduction and the counter reset.
#include "ssfm_kernels.h"

namespace opo {

// Adaptive step, one wave per instance (lane 0 decides), see ssfm_kernels.h.
// The error ratio d = ||u_f - u_c|| / ||u_f|| is undefined (0/0) for an
// instance whose fields are zero everywhere: its attempt is kept and its step
// left as it is. Any other d that is not a number (a step that overflowed, or
// non-finite fields) rejects the attempt like a too-large error and halves dz;
// the attempt budget ends an instance that never recovers.
__global__ __launch_bounds__(kThreads) void adapt_control(AdaptState *ctl, int n_inst, int chunks,
                                                          const double *part, int mode, double z0, double length,
                                                          double dz0, double tol, int max_attempts)
{
    const int lane = threadIdx.x & 63;
    for (int ii = blockIdx.x * (kThreads / 64) + (threadIdx.x >> 6); ii < n_inst; ii += gridDim.x * (kThreads / 64)) {
        // error sums of the attempt: lane-strided partials, then a fixed shuffle tree
        double num = 0.0, den = 0.0;
        if (mode == 1)
            for (int c = lane; c < chunks; c += 64) {
                num += part[2 * (static_cast<long long>(ii) * chunks + c)];
                den += part[2 * (static_cast<long long>(ii) * chunks + c) + 1];
            }
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) {
            num += __shfl_down(num, o, 64);
            den += __shfl_down(den, o, 64);
        }
        if (lane != 0) continue;
        AdaptState st = ctl[ii];
        if (mode == 0) {
            st.z = z0;
            st.end = z0 + length;
            st.dz = dz0;
            st.tol = tol;
            st.max_attempts = max_attempts;
            st.status = 0;
            st.last = 0;
            st.pend = 0;
            st.accepted = 0;
            st.rejected = 0;
        } else if (st.status == 0) {
            const bool zero = num == 0.0 && den == 0.0;
            const double dd = sqrt(num / den);
            const double tol = st.tol;
            if (!zero && !(dd <= 2.0 * tol)) {
                st.dz *= 0.5;
                st.rejected += 1;
                st.pend = 0;
            } else {
                st.z = st.last ? st.end : st.z + st.dz;
                st.accepted += 1;
                st.pend = 1;
                if (dd > tol) st.dz /= kAdaptGrow;
                else if (dd < 0.5 * tol) st.dz *= kAdaptGrow;
            }
        } else {
            st.pend = 0;      // extrapolated by the begin of this attempt
        }
        if (st.status == 0) {
            if (!(st.z < st.end)) {
                st.status = 1;
            } else if (st.accepted + st.rejected >= st.max_attempts) {
                st.status = 2;
            } else {
                const double rest = st.end - st.z;
                st.last = rest <= st.dz * kAdaptSlack;
                if (st.last) st.dz = rest;
            }
        }
        ctl[ii] = st;
    }
}

__global__ __launch_bounds__(kThreads) void energy_reduce(const InstDesc *inst, int n_inst,
                                                          const double *partial, double *hist,
                                                          int *counter, int capacity)
{
    __shared__ int bad;
    if (counter[2] != 0) return;     // stopped by an earlier round trip of this call
    const int slot = counter[0];
    if (threadIdx.x == 0) bad = counter[3];
    __syncthreads();
    bool mine = false;
    for (int ii = threadIdx.x; ii < n_inst; ii += kThreads) {
        const InstDesc &d = inst[ii];
        double e[3] = {0.0, 0.0, 0.0};
        for (int t = 0; t < d.tiles_a; ++t)
            for (int x = 0; x < 3; ++x)
                e[x] += partial[(d.tile_a0 + t) * 3 + x];
        mine = mine || !(isfinite(e[0]) && isfinite(e[1]) && isfinite(e[2]));
        // written in any case: the host reads only the rows below counter[0]
        if (slot < capacity)
            for (int x = 0; x < 3; ++x)
                hist[(static_cast<long long>(slot) * n_inst + ii) * 3 + x] = e[x];
    }
    if (mine) bad = 1;               // benign race: every writer stores 1
    __syncthreads();
    if (threadIdx.x == 0) {
        if (bad) {
            counter[2] = 1;
        } else {
            counter[0] = slot + 1;
            counter[1] += 1;         // round trips completed
        }
    }
}

__global__ void set_counter(int *counter, int slot, int rt, int clear_flags)
{
    if (threadIdx.x == 0 && blockIdx.x == 0) {
        counter[0] = slot;
        if (rt >= 0) counter[1] = rt;
        if (clear_flags) {
            counter[2] = 0;
            counter[3] = 0;
        }
    }
}

__global__ __launch_bounds__(kThreads) void spectrum_prep(const InstDesc *inst, int i, InstDesc *desc,
                                                          int *counter, int *map, int map_len)
{
    if (threadIdx.x == 0) {
        InstDesc d = inst[i];
        d.off = 0;
        d.tile_a0 = 0;
        d.tile_b0 = 0;
        *desc = d;
    }
    if (threadIdx.x < 4) counter[threadIdx.x] = 0;
    for (int q = threadIdx.x; q < map_len; q += kThreads) map[q] = 0;
}

} // namespace opo
