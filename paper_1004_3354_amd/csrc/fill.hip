// Device-side fill with the counter-based SplitMix64 generator (Steele, Lea and
// Flood 2014; constants of Vigna's public-domain reference): element i of stream
// `seed` is output i+1 of SplitMix64 started from state `seed`, so any element
// can be produced on its own, here and on the host, without storing a stream.
#include <cmath>

#include "ed_internal.h"

namespace ed {

__device__ __forceinline__ uint64_t splitmix_at(uint64_t seed, uint64_t i) {
    uint64_t z = seed + (i + 1ull) * 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

__global__ void k_fill(void *out, int64_t n, uint64_t seed, int dist, int is_f32) {
    const double inv53 = 1.0 / 9007199254740992.0;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        double v;
        if (dist == 0) {
            v = 2.0 * ((double)(splitmix_at(seed, (uint64_t)i) >> 11) * inv53) - 1.0;
        } else {
            const double u1 = ((double)(splitmix_at(seed, 2ull * (uint64_t)i) >> 11) + 1.0) * inv53;
            const double u2 = (double)(splitmix_at(seed, 2ull * (uint64_t)i + 1ull) >> 11) * inv53;
            v = sqrt(-2.0 * log(u1)) * cos(2.0 * 3.141592653589793 * u2);
        }
        if (is_f32) ((float *)out)[i] = (float)v;
        else ((double *)out)[i] = v;
    }
}

}  // namespace ed

using namespace ed;

extern "C" ed_status ed_fill_random(void *x, int64_t n, uint64_t seed, int dist, int precision, void *stream) {
    return guard([&] {
        if (n < 0 || (n > 0 && !x)) fail(ED_EINVAL, "ed_fill_random: bad vector");
        if (dist != 0 && dist != 1) fail(ED_EINVAL, "ed_fill_random: dist must be 0 or 1");
        if (precision != ED_FP64 && precision != ED_FP32) fail(ED_EINVAL, "ed_fill_random: bad precision");
        if (n == 0) return;
        k_fill<<<grid_for(n, 256, 1 << 16), 256, 0, (hipStream_t)stream>>>(x, n, seed, dist, precision == ED_FP32);
        ED_LAUNCH_CHECK();
    });
}
