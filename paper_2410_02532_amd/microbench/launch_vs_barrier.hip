// launch_vs_barrier.hip -- what a step boundary costs on the device: one kernel
// launch per step replayed from a hipGraph, against a persistent kernel whose
// G workgroups meet at a device-scope barrier between steps.
//
// Each step, every workgroup writes 12 KB and then reads the 12 KB its
// neighbour wrote in the same step (the shape of an exchange between the two
// passes of a four-step transform). The persistent variant separates the write
// and the read by a barrier: release fence at agent scope, one atomic arrival on
// a counter, a spin on that counter (bounded: after 2^22 polls the workgroup
// records a time-out and leaves the loop), acquire fence. The launch variant
// puts each step in its own kernel. Both check every value they read.
//
// Build and run (one GPU):
//   hipcc --offload-arch=gfx950 -O3 -Xclang -target-feature -Xclang -packed-fp32-ops \
//         -o launch_vs_barrier paper_2410_02532_amd/microbench/launch_vs_barrier.hip
//   ./launch_vs_barrier
#include <hip/hip_runtime.h>
#include <cstdio>

#define CK(x) do { hipError_t e_ = (x); if (e_ != hipSuccess) { \
    std::printf("HIP error %s at line %d\n", hipGetErrorString(e_), __LINE__); return 1; } } while (0)

constexpr int kThreadsMb = 256;
constexpr int kPer = 3072;          // floats exchanged per workgroup and step (12 KB)
constexpr int kSpinLimit = 1 << 22;

__device__ inline void exch_write(float *buf, int par, int r, int G, int it)
{
    float4 *p = reinterpret_cast<float4 *>(buf + static_cast<size_t>(par * G + r) * kPer);
    const float v = static_cast<float>(it * G + r);
    for (int k = 0; k < 3; ++k) p[threadIdx.x + kThreadsMb * k] = make_float4(v, v, v, v);
}

__device__ inline float exch_read(const float *buf, int par, int r, int G, int it, int *err)
{
    const int q = (r + 1) % G;
    const float4 *p = reinterpret_cast<const float4 *>(buf + static_cast<size_t>(par * G + q) * kPer);
    const float want = static_cast<float>(it * G + q);
    float s = 0.f;
    int bad = 0;
    for (int k = 0; k < 3; ++k) {
        const float4 a = p[threadIdx.x + kThreadsMb * k];
        s += a.x + a.w;
        bad += (a.x != want) | (a.w != want);
    }
    if (bad) atomicAdd(err + 1, bad);
    return s;
}

// all G workgroups reach it before any leaves; false after a time-out
__device__ inline bool group_barrier(int *ctr, int target, int *err)
{
    __shared__ int ok;
    __syncthreads();
    if (threadIdx.x == 0) {
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
        __hip_atomic_fetch_add(ctr, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        int n = 0;
        while (__hip_atomic_load(ctr, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < target && ++n < kSpinLimit)
            __builtin_amdgcn_s_sleep(1);
        ok = n < kSpinLimit;
        if (!ok) atomicAdd(err, 1);
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
    }
    __syncthreads();
    return ok;
}

// stride 1: workgroups 0..G-1; stride 8: every eighth of 8G workgroups (the
// workgroups are dealt to the eight XCDs in turn, so these share one XCD)
__global__ __launch_bounds__(kThreadsMb) void persistent_steps(float *buf, int *ctr, int *err, float *out, int G,
                                                               int steps, int stride)
{
    if (blockIdx.x % stride) return;
    const int r = blockIdx.x / stride;
    float acc = 0.f;
    for (int it = 0; it < steps; ++it) {
        exch_write(buf, it & 1, r, G, it);
        if (!group_barrier(ctr, G * (it + 1), err)) break;
        acc += exch_read(buf, it & 1, r, G, it, err);
    }
    out[r * kThreadsMb + threadIdx.x] = acc;
}

__global__ __launch_bounds__(kThreadsMb) void first_step(float *buf, int G) { exch_write(buf, 0, blockIdx.x, G, 0); }

__global__ __launch_bounds__(kThreadsMb) void next_step(float *buf, int *err, float *out, int G, int it)
{
    out[blockIdx.x * kThreadsMb + threadIdx.x] += exch_read(buf, (it - 1) & 1, blockIdx.x, G, it - 1, err);
    exch_write(buf, it & 1, blockIdx.x, G, it);
}

int main()
{
    const int gmax = 256, steps = 2000, graph_steps = 400;
    float *buf, *out;
    int *ctr, *err;
    CK(hipMalloc(&buf, sizeof(float) * 2 * gmax * kPer));
    CK(hipMalloc(&out, sizeof(float) * gmax * kThreadsMb));
    CK(hipMalloc(&ctr, 64));
    CK(hipMalloc(&err, 64));
    hipStream_t s;
    CK(hipStreamCreate(&s));
    hipEvent_t e0, e1;
    CK(hipEventCreate(&e0));
    CK(hipEventCreate(&e1));
    std::printf("| workgroups G | persistent, barrier (us/step) | persistent, one XCD (us/step) | graph, launch (us/step) |\n");
    std::printf("|---|---|---|---|\n");
    for (int G : {8, 16, 24, 32, 48, 64, 128, 256}) {
        float per[2] = {-1.f, -1.f};
        int fails = 0;
        for (int v = 0; v < 2; ++v) {
            const int stride = v == 0 ? 1 : 8;
            if (G * stride > gmax) continue;
            float best = 1e30f;
            int herr[2] = {0, 0};
            for (int rep = 0; rep < 3; ++rep) {
                CK(hipMemsetAsync(ctr, 0, 64, s));
                CK(hipMemsetAsync(err, 0, 64, s));
                CK(hipEventRecord(e0, s));
                hipLaunchKernelGGL(persistent_steps, dim3(G * stride), dim3(kThreadsMb), 0, s, buf, ctr, err, out, G,
                                   steps, stride);
                CK(hipGetLastError());
                CK(hipEventRecord(e1, s));
                CK(hipStreamSynchronize(s));
                float ms;
                CK(hipEventElapsedTime(&ms, e0, e1));
                best = ms < best ? ms : best;
                CK(hipMemcpy(herr, err, 8, hipMemcpyDeviceToHost));
                fails += herr[0] + herr[1];
            }
            per[v] = best * 1e3f / steps;
        }
        CK(hipMemsetAsync(err, 0, 64, s));
        hipGraph_t g;
        hipGraphExec_t ge;
        CK(hipStreamBeginCapture(s, hipStreamCaptureModeGlobal));
        hipLaunchKernelGGL(first_step, dim3(G), dim3(kThreadsMb), 0, s, buf, G);
        for (int it = 1; it < graph_steps; ++it)
            hipLaunchKernelGGL(next_step, dim3(G), dim3(kThreadsMb), 0, s, buf, err, out, G, it);
        CK(hipStreamEndCapture(s, &g));
        CK(hipGraphInstantiate(&ge, g, nullptr, nullptr, 0));
        float best = 1e30f;
        for (int rep = 0; rep < 3; ++rep) {
            CK(hipEventRecord(e0, s));
            CK(hipGraphLaunch(ge, s));
            CK(hipEventRecord(e1, s));
            CK(hipStreamSynchronize(s));
            float ms;
            CK(hipEventElapsedTime(&ms, e0, e1));
            best = ms < best ? ms : best;
        }
        int herr[2];
        CK(hipMemcpy(herr, err, 8, hipMemcpyDeviceToHost));
        fails += herr[1];
        CK(hipGraphExecDestroy(ge));
        CK(hipGraphDestroy(g));
        char one[32];
        if (per[1] < 0.f) std::snprintf(one, sizeof one, "-");
        else std::snprintf(one, sizeof one, "%.2f", per[1]);
        std::printf("| %d | %.2f | %s | %.2f |%s\n", G, per[0], one, best * 1e3f / graph_steps,
                    fails ? " (time-outs or wrong values)" : "");
        std::fflush(stdout);
        if (fails) return 1;
    }
    return 0;
}
