// Kernels launched only from api.hip: initial droplet fields, the health check, the solid
// mask and the streaming copy of the bandwidth measurement (gfx950).
#pragma once

#include "common.h"

namespace lbmk {

// SplitMix64 (Steele, Lea and Flood, OOPSLA 2014) used as a counter-based generator:
// the value for counter n under seed s is the output for state s + (n+1) * golden gamma;
// the uniform double in [0, 1) is the top 53 bits times 2^-53.
__device__ __forceinline__ double splitmix_uniform(uint64_t seed, uint64_t n) {
    uint64_t z = seed + (n + 1) * 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    z = z ^ (z >> 31);
    return (double)(z >> 11) * (1.0 / 9007199254740992.0);
}

// Droplet initial density and velocity fields (float64), see lbm_init_droplet.
__global__ __launch_bounds__(256) void k_droplet_fields(double* __restrict__ rho0, double* __restrict__ u0,
                                                        Grid g, double cx, double cy, double cz,
                                                        double R, double W, double rin, double rout,
                                                        double ux, double uy, double uz,
                                                        double amp, uint64_t seed) {
    const int x = blockIdx.x * blockDim.x + threadIdx.x;
    const int y = blockIdx.y * blockDim.y + threadIdx.y;
    const int z = blockIdx.z;
    if (x >= g.nx || y >= g.ny) return;
    const long long N = (long long)g.nx * g.ny * g.nz;
    const long long n = x + (long long)g.nx * (y + (long long)g.ny * z);
    const double dx = x - cx, dy = y - cy, dz = z - cz;
    const double r = sqrt(dx * dx + dy * dy + dz * dz);
    double rho = 0.5 * (rin + rout) - 0.5 * (rin - rout) * tanh(2.0 * (r - R) / W);
    double phi = (rho - rout) / (rin - rout);
    phi = phi < 0.0 ? 0.0 : (phi > 1.0 ? 1.0 : phi);
    if (amp != 0.0 && fabs(r - R) < W)
        rho = rho * (1.0 + amp * (2.0 * splitmix_uniform(seed, (uint64_t)n) - 1.0));
    rho0[n] = rho;
    u0[n] = ux * phi; u0[N + n] = uy * phi; u0[2 * N + n] = uz * phi;
}

// Health check of the stored state: per-block minimum of the node density and a
// non-finite flag over the fluid nodes (solid mask byte 0). The stored values of a fluid
// node are the populations it wrote in the last step (after an initialisation, values
// written into its slots), whose sum is its density; solid nodes hold no populations and
// are skipped. Reads only the populations and the mask, so it is valid after either step
// schedule. Writes partial[2 b] = min rho, partial[2 b + 1] = 1 if any sum is non-finite.
template <int Q, typename T>
__global__ __launch_bounds__(256) void k_health(const T* __restrict__ f,
                                                const uint8_t* __restrict__ solid,
                                                double* __restrict__ partial, Grid g, double rho_ref) {
    const int x = blockIdx.x * blockDim.x + threadIdx.x;
    const int y = blockIdx.y * blockDim.y + threadIdx.y;
    const int z = blockIdx.z;
    double mn = 1e300, bad = 0.0;
    if (x < g.nx && y < g.ny) {
        const int n = x + g.nx * (y + g.ny * z);
        if (!solid[n]) {
            double s = rho_ref;
            for (int i = 0; i < Q; ++i) s += (double)f[(long long)i * g.stride + n];
            if (!isfinite(s)) bad = 1.0; else mn = s;
        }
    }
    for (int off = 32; off > 0; off >>= 1) {
        mn = fmin(mn, __shfl_down(mn, off, 64));
        bad = fmax(bad, __shfl_down(bad, off, 64));
    }
    __shared__ double red[2][8];
    const int tid = threadIdx.x + blockDim.x * threadIdx.y;
    if ((tid & 63) == 0) { red[0][tid >> 6] = mn; red[1][tid >> 6] = bad; }
    __syncthreads();
    if (tid == 0) {
        const int nw = (blockDim.x * blockDim.y + 63) / 64;
        for (int w = 1; w < nw; ++w) { mn = fmin(mn, red[0][w]); bad = fmax(bad, red[1][w]); }
        mn = fmin(mn, red[0][0]); bad = fmax(bad, red[1][0]);
        const long long b = blockIdx.x + (long long)gridDim.x * (blockIdx.y + (long long)gridDim.y * blockIdx.z);
        partial[2 * b] = mn; partial[2 * b + 1] = bad;
    }
}

__global__ __launch_bounds__(256) void k_health_final(const double* __restrict__ partial,
                                                      long long nblocks, double* __restrict__ out) {
    __shared__ double red[2][256];
    double mn = 1e300, bad = 0.0;
    for (long long b = threadIdx.x; b < nblocks; b += blockDim.x) {
        mn = fmin(mn, partial[2 * b]);
        bad = fmax(bad, partial[2 * b + 1]);
    }
    red[0][threadIdx.x] = mn; red[1][threadIdx.x] = bad;
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s) {
            red[0][threadIdx.x] = fmin(red[0][threadIdx.x], red[0][threadIdx.x + s]);
            red[1][threadIdx.x] = fmax(red[1][threadIdx.x], red[1][threadIdx.x + s]);
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) { out[0] = red[0][0]; out[1] = red[1][0]; }
}

// Plain streaming copy (measurement aid: the attainable read + write HBM bandwidth that the
// step kernels are compared with): 16-byte elements, grid-stride, nontemporal hints.
typedef float lbm_f4 __attribute__((ext_vector_type(4)));
__global__ __launch_bounds__(256) void k_copy_stream(const lbm_f4* __restrict__ a,
                                                     lbm_f4* __restrict__ b, long long n) {
    const long long stride = (long long)gridDim.x * blockDim.x;
    for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride)
        __builtin_nontemporal_store(__builtin_nontemporal_load(a + i), b + i);
}

// Solid mask: wall layers on the faces set in g.walls and nodes whose centre lies in the
// x-aligned cylinder (y - cy)^2 + (z - cz)^2 <= r^2 (float64, as on the host).
__global__ __launch_bounds__(256) void k_build_solid(uint8_t* __restrict__ solid, Grid g, int cylinder,
                                                     double cy, double cz, double r) {
    const int x = blockIdx.x * blockDim.x + threadIdx.x;
    const int y = blockIdx.y * blockDim.y + threadIdx.y;
    const int z = blockIdx.z;
    if (x >= g.nx || y >= g.ny) return;
    const int c[3] = {x, y, z}, n[3] = {g.nx, g.ny, g.nz};
    bool s = false;
    for (int a = 0; a < 3; ++a) {
        if (((g.walls >> (2 * a)) & 1) && c[a] == 0) s = true;
        if (((g.walls >> (2 * a + 1)) & 1) && c[a] == n[a] - 1) s = true;
    }
    if (cylinder) {
        const double dy = y - cy, dz = z - cz;
        if (dy * dy + dz * dz <= r * r) s = true;
    }
    solid[x + (long long)g.nx * (y + (long long)g.ny * z)] = s ? 1 : 0;
}


}  // namespace lbmk
