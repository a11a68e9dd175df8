// synth.hip -- libsynth.so: the counter-based draws of synthetic/generate.py on the
// GPU, for workloads too large to draw on the host.  Random numbers only; no
// ladder arithmetic.  SplitMix64 (Steele, Lea, Flood, OOPSLA 2014) as a hash of
// counter = seed << 48 | stream << 40 | index; uniform = (z >> 11) * 2^-53;
// Gaussian = sqrt(-2 log1p(-u1)) cos(2 pi u2) with u2 from stream | 0x80.
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

namespace {

__device__ inline uint64_t splitmix64(uint64_t x) {
    uint64_t z = x + 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

__device__ inline double uniform(uint64_t seed, uint64_t stream, uint64_t index) {
    const uint64_t c = (seed << 48) | (stream << 40) | index;
    return (double)(splitmix64(c) >> 11) * 0x1.0p-53;
}

__device__ inline double gaussian(uint64_t seed, uint64_t stream, uint64_t index) {
    const double u1 = uniform(seed, stream, index);
    const double u2 = uniform(seed, stream | 0x80, index);
    return sqrt(-2.0 * log1p(-u1)) * cos(2.0 * M_PI * u2);
}

__global__ void L_block_kernel(uint64_t seed, int64_t N, int64_t n, int64_t p0, int64_t np, int64_t q0, int64_t nq,
                               double scale, double* __restrict__ out) {
    const int64_t total = np * nq * n;
    for (int64_t x = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; x < total; x += (int64_t)gridDim.x * blockDim.x) {
        const int64_t J = x % n, pq = x / n;
        const int64_t p = p0 + pq / nq, q = q0 + pq % nq;
        const int64_t lo = p < q ? p : q, hi = p < q ? q : p;
        out[x] = scale * gaussian(seed, 1, (uint64_t)((lo * N + hi) * n + J));
    }
}

__global__ void eps_kernel(uint64_t seed, int64_t o, int64_t v, double* __restrict__ eps) {
    const int64_t x = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (x < o) eps[x] = -1.5 + 1.2 * uniform(seed, 2, (uint64_t)x);
    else if (x < o + v) eps[x] = 0.1 + 2.9 * uniform(seed, 3, (uint64_t)(x - o));
}

// out = t + scale * xi with xi_ij^ab = xi_ji^ba (stream 4, index min*ov + max).
__global__ void add_noise_kernel(uint64_t seed, int64_t o, int64_t v, double scale, const double* __restrict__ t,
                                 double* __restrict__ out) {
    const int64_t total = o * o * v * v, ov = o * v;
    for (int64_t x = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; x < total; x += (int64_t)gridDim.x * blockDim.x) {
        const int64_t b = x % v, a = (x / v) % v, ij = x / (v * v);
        const int64_t j = ij % o, i = ij / o;
        const int64_t P1 = i * v + a, P2 = j * v + b;
        const int64_t lo = P1 < P2 ? P1 : P2, hi = P1 < P2 ? P2 : P1;
        out[x] = t[x] + scale * gaussian(seed, 4, (uint64_t)(lo * ov + hi));
    }
}

unsigned grid(int64_t total) {
    int64_t g = (total + 255) / 256;
    return (unsigned)(g > 65536 ? 65536 : (g < 1 ? 1 : g));
}

}  // namespace

extern "C" {

int synth_L_block(uint64_t seed, int64_t N, int64_t n, int64_t p0, int64_t np, int64_t q0, int64_t nq, double scale,
                  double* out, void* stream) {
    if (!out || N < 1 || n < 1 || np < 0 || nq < 0 || p0 < 0 || q0 < 0 || p0 + np > N || q0 + nq > N) return -1;
    if ((uint64_t)(N * N) * (uint64_t)n >= (1ull << 40) || seed >= (1u << 16)) return -1;
    hipLaunchKernelGGL(L_block_kernel, dim3(grid(np * nq * n)), dim3(256), 0, (hipStream_t)stream, seed, N, n, p0, np,
                       q0, nq, scale, out);
    return hipGetLastError() == hipSuccess ? 0 : -4;
}

int synth_eps(uint64_t seed, int64_t o, int64_t v, double* eps, void* stream) {
    if (!eps || o < 1 || v < 1 || seed >= (1u << 16)) return -1;
    hipLaunchKernelGGL(eps_kernel, dim3(grid(o + v)), dim3(256), 0, (hipStream_t)stream, seed, o, v, eps);
    return hipGetLastError() == hipSuccess ? 0 : -4;
}

int synth_add_noise(uint64_t seed, int64_t o, int64_t v, double scale, const double* t, double* out, void* stream) {
    if (!t || !out || o < 1 || v < 1 || seed >= (1u << 16)) return -1;
    if ((uint64_t)(o * v) * (uint64_t)(o * v) >= (1ull << 40)) return -1;
    hipLaunchKernelGGL(add_noise_kernel, dim3(grid(o * o * v * v)), dim3(256), 0, (hipStream_t)stream, seed, o, v,
                       scale, t, out);
    return hipGetLastError() == hipSuccess ? 0 : -4;
}

}  // extern "C"
