// kernels_inject.hip - the seeded disk source of fepic_set_injector: a beam's particles
// enter through a disk on a wall every step (Sec. IV-B), drawn on the device from a
// counter-based generator, so that particle j of injection k of a species is the same
// whatever the launch shape.
//
// Generator: Philox4x32-10 (Salmon, Moraes, Dror and Shaw, SC 2011).  Particle j of
// injection k of species s takes the three blocks of counter (j, k mod 2^32, k div 2^32,
// 4 s + b), b = 0..2, under the key (seed mod 2^32, seed div 2^32): twelve words, read in
// pairs as six uniforms u_i = ((w_2i >> 5) 2^26 + (w_2i+1 >> 6) + 1/2) 2^-53 in (0, 1):
// disk radius R sqrt(u_0) and angle 2 pi u_1; three standard normals by Box-Muller from
// (u_2, u_3) and (u_4, u_5); v = v0 n + sigma N, stored as gamma v (Boris) or v (AB).
#include "fepic_internal.h"

namespace fepic {
namespace {

constexpr int kBlock = 256;

__device__ __forceinline__ void philox4x32_10(uint32_t c[4], uint32_t k0, uint32_t k1) {
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        if (r > 0) {
            k0 += 0x9E3779B9u;
            k1 += 0xBB67AE85u;
        }
        const uint32_t hi0 = __umulhi(0xD2511F53u, c[0]), lo0 = 0xD2511F53u * c[0];
        const uint32_t hi1 = __umulhi(0xCD9E8D57u, c[2]), lo1 = 0xCD9E8D57u * c[2];
        const uint32_t n0 = hi1 ^ c[1] ^ k0, n2 = hi0 ^ c[3] ^ k1;
        c[0] = n0;
        c[1] = lo1;
        c[2] = n2;
        c[3] = lo0;
    }
}

__global__ __launch_bounds__(kBlock) void k_inject_disk(InjectorSpec sp, int64_t k, double* __restrict__ x,
                                                        double* __restrict__ u) {
    const int64_t j = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (j >= sp.per_step) return;
    const uint32_t k0 = (uint32_t)(sp.seed & 0xFFFFFFFFull), k1 = (uint32_t)(sp.seed >> 32);
    uint32_t w[12];
#pragma unroll
    for (int b = 0; b < 3; ++b) {
        uint32_t c[4] = {(uint32_t)j, (uint32_t)((uint64_t)k & 0xFFFFFFFFull), (uint32_t)((uint64_t)k >> 32),
                         (uint32_t)(4 * sp.species + b)};
        philox4x32_10(c, k0, k1);
#pragma unroll
        for (int q = 0; q < 4; ++q) w[4 * b + q] = c[q];
    }
    double U[6];
#pragma unroll
    for (int i = 0; i < 6; ++i)
        U[i] = ((double)(w[2 * i] >> 5) * 67108864.0 + (double)(w[2 * i + 1] >> 6) + 0.5) * 0x1p-53;
    const double r = sp.radius * sqrt(U[0]);
    const double phi = 2.0 * M_PI * U[1];
    const double cp = cos(phi), sp_ = sin(phi);
    const double a = sqrt(-2.0 * log(U[2])), bb = sqrt(-2.0 * log(U[4]));
    const double N[3] = {a * cos(2.0 * M_PI * U[3]), a * sin(2.0 * M_PI * U[3]), bb * cos(2.0 * M_PI * U[5])};
    double v[3];
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        x[3 * j + d] = sp.c[d] + r * (cp * sp.e1[d] + sp_ * sp.e2[d]);
        v[d] = sp.v0 * sp.n[d] + sp.sigma * N[d];
    }
    double g = 1.0;
    if (sp.relativistic_u) g = 1.0 / sqrt(1.0 - (v[0] * v[0] + v[1] * v[1] + v[2] * v[2]) / (kC * kC));
#pragma unroll
    for (int d = 0; d < 3; ++d) u[3 * j + d] = g * v[d];
}

}  // namespace

void launch_inject_disk(hipStream_t s, const InjectorSpec& spec, int64_t k, double* x, double* u) {
    if (spec.per_step <= 0) return;
    hipLaunchKernelGGL(k_inject_disk, dim3(grid_1d(spec.per_step, kBlock)), dim3(kBlock), 0, s, spec, k, x, u);
}

}  // namespace fepic
