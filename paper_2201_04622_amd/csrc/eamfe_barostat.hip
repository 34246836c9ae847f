// Pieces of the stochastic cell-rescaling barostat (Bernetti and Bussi, J.
// Chem. Phys. 153, 114107, 2020), isotropic or per axis, that the coupling
// move of eamfe_barostat_step needs besides the virial: each replica's
// kinetic sums, the scaling of positions and velocities by each replica's
// factors, and the normal deviates that drive the box.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>

#include "eamfe_internal.h"

namespace eamfe {

// sum_i v_i,a^2 over each replica's atoms, per axis a (the kinetic part of the
// diagonal pressure, before the mass): one block per replica, a strided sum
// per thread, then a fixed tree; out[n_rep][3].
constexpr int kKinBlock = 256;

__global__ __launch_bounds__(kKinBlock) void k_kinetic(const double* v, const RepDesc* reps, int N, double* out)
{
    __shared__ double sh[3][kKinBlock];
    const RepDesc& R = reps[blockIdx.x];
    double s[3] = {0.0, 0.0, 0.0};
    for (int k = threadIdx.x; k < R.n; k += blockDim.x) {
        const int i = R.off + k;
        for (int c = 0; c < 3; ++c) s[c] += v[(size_t)c * N + i] * v[(size_t)c * N + i];
    }
    for (int c = 0; c < 3; ++c) sh[c][threadIdx.x] = s[c];
    __syncthreads();
    for (int h = kKinBlock / 2; h > 0; h >>= 1) {
        if ((int)threadIdx.x < h)
            for (int c = 0; c < 3; ++c) sh[c][threadIdx.x] += sh[c][threadIdx.x + h];
        __syncthreads();
    }
    if (threadIdx.x < 3) out[3 * blockIdx.x + threadIdx.x] = sh[threadIdx.x][0];
}

hipError_t launch_kinetic(const double* v, const RepDesc* reps, int n_rep, int N, double* out, hipStream_t s)
{
    if (n_rep <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_kinetic, dim3(n_rep), dim3(kKinBlock), 0, s, v, reps, N, out);
    return hipGetLastError();
}

// x_a <- mu_a x_a, v_a <- v_a / mu_a for the atoms of each replica (SoA
// [3][N] FP64; one thread per atom; mu[n_rep][3] on the device, one factor
// per axis)
__global__ void k_rescale(double* x, double* v, const int32_t* rep_of, const double* mu, int N)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= N) return;
    const int r = rep_of[i];
    for (int c = 0; c < 3; ++c) {
        const double m = mu[3 * r + c];   // the factor of axis c
        x[(size_t)c * N + i] *= m;
        v[(size_t)c * N + i] *= 1.0 / m;
    }
}

hipError_t launch_rescale(double* x, double* v, const int32_t* rep_of, const double* mu, int N, hipStream_t s)
{
    if (N <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_rescale, dim3((N + 255) / 256), dim3(256), 0, s, x, v, rep_of, mu, N);
    return hipGetLastError();
}

// Philox4x32-10 (Salmon, Moraes, Dror and Shaw, SC'11) on the host: ten
// rounds of two 32x32 -> 64-bit products with the published multipliers,
// the key bumped by the published Weyl constants between rounds.
static void philox4x32_10(uint32_t ctr[4], uint32_t k0, uint32_t k1)
{
    for (int round = 0; round < 10; ++round) {
        const uint64_t p0 = (uint64_t)0xD2511F53u * ctr[0];
        const uint64_t p1 = (uint64_t)0xCD9E8D57u * ctr[2];
        const uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
        const uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
        const uint32_t n0 = hi1 ^ ctr[1] ^ k0, n1 = lo1, n2 = hi0 ^ ctr[3] ^ k1, n3 = lo0;
        ctr[0] = n0;
        ctr[1] = n1;
        ctr[2] = n2;
        ctr[3] = n3;
        k0 += 0x9E3779B9u;
        k1 += 0xBB67AE85u;
    }
}

// The three Box--Muller deviates of the Philox block at counter (atom, step
// low word, stream, step high word) under key (seed low word, seed high
// word): z0, z1 from the uniforms (w + 1) 2^-32 of its first two words, z2
// from the last two.
void barostat_gauss3(uint64_t seed, uint32_t atom, int64_t step, uint32_t stream, double z[3])
{
    uint32_t c[4] = {atom, (uint32_t)((uint64_t)step & 0xffffffffu), stream, (uint32_t)((uint64_t)step >> 32)};
    philox4x32_10(c, (uint32_t)(seed & 0xffffffffu), (uint32_t)(seed >> 32));
    double u[4];
    for (int q = 0; q < 4; ++q) u[q] = ((double)c[q] + 1.0) * 2.3283064365386963e-10;
    const double r0 = std::sqrt(-2.0 * std::log(u[0])), r1 = std::sqrt(-2.0 * std::log(u[2]));
    z[0] = r0 * std::cos(2.0 * M_PI * u[1]);
    z[1] = r0 * std::sin(2.0 * M_PI * u[1]);
    z[2] = r1 * std::cos(2.0 * M_PI * u[3]);
}

}  // namespace eamfe
