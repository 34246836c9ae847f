// Pieces of the isotropic stochastic cell-rescaling barostat (Bernetti and
// Bussi, J. Chem. Phys. 153, 114107, 2020) that the coupling move of
// eamfe_barostat_step needs besides the pressure evaluation: the scaling of
// positions and velocities by each replica's factor, and the normal deviate
// that drives the volume.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>

namespace eamfe {

// x <- mu x, v <- v / mu for the atoms of each replica (SoA [3][N] FP64; one
// thread per atom; mu[n_rep] on the device)
__global__ void k_rescale(double* x, double* v, const int32_t* rep_of, const double* mu, int N)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= N) return;
    const double m = mu[rep_of[i]];
    const double im = 1.0 / m;
    for (int c = 0; c < 3; ++c) {
        x[(size_t)c * N + i] *= m;
        v[(size_t)c * N + i] *= im;
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

// The first Box--Muller deviate of the Philox block at counter (atom, step
// low word, stream, step high word) under key (seed low word, seed high
// word), from the uniforms (w + 1) 2^-32 of its first two words.
double barostat_gauss(uint64_t seed, uint32_t atom, int64_t step, uint32_t stream)
{
    uint32_t c[4] = {atom, (uint32_t)((uint64_t)step & 0xffffffffu), stream, (uint32_t)((uint64_t)step >> 32)};
    philox4x32_10(c, (uint32_t)(seed & 0xffffffffu), (uint32_t)(seed >> 32));
    const double u0 = ((double)c[0] + 1.0) * 2.3283064365386963e-10;
    const double u1 = ((double)c[1] + 1.0) * 2.3283064365386963e-10;
    return std::sqrt(-2.0 * std::log(u0)) * std::cos(2.0 * M_PI * u1);
}

}  // namespace eamfe
