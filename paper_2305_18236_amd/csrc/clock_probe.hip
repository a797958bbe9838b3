// Shader-clock probe, for reporting the clock a measurement ran at beside
// its fraction of the spec peak (the spec peaks assume 2.4 GHz; under
// sustained matrix work the chip holds less).
//
// A few one-wave workgroups each read two counters, spin for a fixed span of
// the constant-rate wall clock (s_memrealtime, 100 MHz), and read them again:
// the shader-cycle counter (s_memtime) advances with the core clock, so
// cycles / wall time is the average core clock of that compute unit over the
// span.  Launched on the caller's stream behind its work, the probe starts
// as the last kernel ahead of it retires.
#include <mutex>

#include "kernels.h"

namespace mg {

constexpr int kClockProbeBlocks = 16;   // two per XCD under the round-robin dispatch

__device__ unsigned long long g_clock_probe[2 * kClockProbeBlocks];

__global__ __launch_bounds__(64) void clock_probe_kernel(unsigned long long wall_ticks)
{
    const unsigned long long w0 = __builtin_amdgcn_s_memrealtime();
    const unsigned long long c0 = __builtin_amdgcn_s_memtime();
    unsigned long long w1 = w0;
    while (w1 - w0 < wall_ticks) w1 = __builtin_amdgcn_s_memrealtime();
    const unsigned long long c1 = __builtin_amdgcn_s_memtime();
    if (threadIdx.x == 0) {
        g_clock_probe[2 * blockIdx.x] = c1 - c0;
        g_clock_probe[2 * blockIdx.x + 1] = w1 - w0;
    }
}

// Host side: launch, wait for the stream, read the counters back.  Calls are
// serialised (the result array is shared by every caller of the process).
hipError_t measure_sclk(hipStream_t stream, int64_t wall_ticks, double wall_hz, double* mhz)
{
    static std::mutex m;
    std::lock_guard<std::mutex> lock(m);
    hipLaunchKernelGGL(clock_probe_kernel, dim3(kClockProbeBlocks), dim3(64), 0, stream,
                       (unsigned long long)wall_ticks);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    unsigned long long h[2 * kClockProbeBlocks];
    e = hipMemcpyFromSymbolAsync(h, HIP_SYMBOL(g_clock_probe), sizeof(h), 0, hipMemcpyDeviceToHost, stream);
    if (e != hipSuccess) return e;
    e = hipStreamSynchronize(stream);
    if (e != hipSuccess) return e;
    double cycles = 0.0, ticks = 0.0;
    for (int b = 0; b < kClockProbeBlocks; ++b) {
        cycles += double(h[2 * b]);
        ticks += double(h[2 * b + 1]);
    }
    *mhz = ticks > 0.0 ? cycles / (ticks / wall_hz) / 1e6 : 0.0;
    return hipSuccess;
}

}  // namespace mg
