// gfx950 kernels of the EAM switching engine.
//
// One MD iteration is two launches over a table of tiles (a tile = a run of
// atoms of one replica; every replica of the batch is in the same launch):
//
//   k_density : rho_i = sum_j rho(r_ij) over the Verlet row, F(rho_i), F'(rho_i),
//               and the thermostat noise of the step with its replica sum;
//   k_force   : pair + embedding forces, the Einstein spring, the lambda blend
//               (Eq. interp) or scale (Eq. H_rs), the closing B half-kick of the
//               previous step and B-A-O-A of the next one (BAOAB), per-replica
//               energy sums, dH/dl, and the work increment (Eq. w_irr).
//
// T lanes cooperate on one atom; lane t takes blocks of SB consecutive
// neighbour slots t, t+T, ...  In FP32 each block's partial sum is rounded
// to a 2^-32 grid and added as an exact integer held in a float64, so the
// per-atom sums do not depend on T or on the block size.  List rows have a
// fixed order (cells sorted by atom id) and per-replica reductions use a
// fixed tree and a "last block finishes" pass, so runs are bitwise
// reproducible.
#include "eamfe_internal.h"

namespace eamfe {

constexpr int SB = 4;           // neighbour slots per lane block
constexpr int kMaxBlock = 1024;

// --------------------------------------------------------------------------
// Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11) and Box-Muller
// --------------------------------------------------------------------------
__device__ __forceinline__ void philox4x32_10(uint32_t& c0, uint32_t& c1, uint32_t& c2, uint32_t& c3,
                                              uint32_t k0, uint32_t k1)
{
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        if (r) {
            k0 += 0x9E3779B9u;
            k1 += 0xBB67AE85u;
        }
        const uint32_t lo0 = 0xD2511F53u * c0, hi0 = __umulhi(0xD2511F53u, c0);
        const uint32_t lo1 = 0xCD9E8D57u * c2, hi1 = __umulhi(0xCD9E8D57u, c2);
        const uint32_t n0 = hi1 ^ c1 ^ k0;
        const uint32_t n2 = hi0 ^ c3 ^ k1;
        c0 = n0;
        c1 = lo1;
        c2 = n2;
        c3 = lo0;
    }
}

// Three N(0,1) deviates for (seed; atom, step, stream): counter words
// (atom, step low, stream, step high), uniforms u = (w + 1) 2^-32.
__device__ __forceinline__ void gauss3(uint64_t seed, uint32_t atom, int64_t step, uint32_t stream,
                                       double& z0, double& z1, double& z2)
{
    const uint64_t st = (uint64_t)step;
    uint32_t c0 = atom, c1 = (uint32_t)st, c2 = stream, c3 = (uint32_t)(st >> 32);
    philox4x32_10(c0, c1, c2, c3, (uint32_t)seed, (uint32_t)(seed >> 32));
    const double s = 2.3283064365386963e-10;
    const double twopi = 6.283185307179586476925286766559;
    const double u0 = ((double)c0 + 1.0) * s, u1 = ((double)c1 + 1.0) * s;
    const double u2 = ((double)c2 + 1.0) * s, u3 = ((double)c3 + 1.0) * s;
    const double r0 = sqrt(-2.0 * log(u0));
    const double r1 = sqrt(-2.0 * log(u2));
    z0 = r0 * cos(twopi * u1);
    z1 = r0 * sin(twopi * u1);
    z2 = r1 * cos(twopi * u3);
}

// --------------------------------------------------------------------------
// Table access
// --------------------------------------------------------------------------
template <typename real>
struct Tab;

template <>
struct Tab<float> {
    static __device__ __forceinline__ float4 ld4(const void* p, int m) { return ((const float4*)p)[m]; }
    static __device__ __forceinline__ void ld8(const void* p, int m, float4& u, float4& w)
    {
        const float4* q = (const float4*)p + 2 * m;
        u = q[0];
        w = q[1];
    }
};

template <>
struct Tab<double> {
    struct d4 {
        double x, y, z, w;
    };
    static __device__ __forceinline__ d4 ld4(const void* p, int m)
    {
        const double2* q = (const double2*)p + 2 * m;
        const double2 a = q[0], b = q[1];
        return d4{a.x, a.y, b.x, b.y};
    }
    static __device__ __forceinline__ void ld8(const void* p, int m, d4& u, d4& w)
    {
        const double2* q = (const double2*)p + 4 * m;
        const double2 a = q[0], b = q[1], c = q[2], d = q[3];
        u = d4{a.x, a.y, b.x, b.y};
        w = d4{c.x, c.y, d.x, d.y};
    }
};

// Accumulation of a lane block's partial sum into a float64 accumulator.
template <typename real>
struct Acc;
template <>
struct Acc<double> {
    static __device__ __forceinline__ double q(double p) { return p; }
    static __device__ __forceinline__ double fin(double a) { return a; }
};
template <>
struct Acc<float> {
    static __device__ __forceinline__ double q(float p) { return rint((double)p * kFixScale); }
    static __device__ __forceinline__ double fin(double a) { return a * kFixInv; }
};

// interval index and local coordinate on a uniform grid; m clamped to [0, n-2]
template <typename real>
__device__ __forceinline__ int interval(real x, real inv_h, int n, real& t)
{
    const real p = x * inv_h;
    int m = (int)p;   // truncation = floor for x >= 0; NaN converts to 0 on gfx9
    m = m < 0 ? 0 : (m > n - 2 ? n - 2 : m);
    t = p - (real)m;
    return m;
}

__device__ __forceinline__ void min_image(const RepDesc& R, double& dx, double& dy, double& dz)
{
    dx -= R.L[0] * rint(dx * R.invL[0]);
    dy -= R.L[1] * rint(dy * R.invL[1]);
    dz -= R.L[2] * rint(dz * R.invL[2]);
}

// --------------------------------------------------------------------------
// Deterministic block reductions
// --------------------------------------------------------------------------
template <int K>
__device__ __forceinline__ void block_sum(double (&v)[K], double* sh)
{
#pragma unroll
    for (int o = 32; o > 0; o >>= 1)
#pragma unroll
        for (int k = 0; k < K; ++k) v[k] += __shfl_xor(v[k], o, 64);
    const int w = threadIdx.x >> 6, nw = (blockDim.x + 63) >> 6;
    if ((threadIdx.x & 63) == 0)
#pragma unroll
        for (int k = 0; k < K; ++k) sh[w * K + k] = v[k];
    __syncthreads();
    if (threadIdx.x == 0) {
#pragma unroll
        for (int k = 0; k < K; ++k) {
            double s = 0.0;
            for (int q = 0; q < nw; ++q) s += sh[q * K + k];
            v[k] = s;
        }
    }
    __syncthreads();
}

// Sum K per-thread values over the block, store the block total as this
// tile's partial for its replica; the last block of the replica to arrive
// reduces all partials in tile order into `out` (K values) and returns true
// in every thread of that block.  Every thread of the block must call it.
template <int K>
__device__ bool replica_reduce(const double (&vin)[K], double* part, uint32_t* cnt, const RepDesc& R, int tile_idx,
                               double* out, double* sh)
{
    __shared__ int last;
    double v[K];
#pragma unroll
    for (int k = 0; k < K; ++k) v[k] = vin[k];
    block_sum<K>(v, sh);
    if (threadIdx.x == 0) {
#pragma unroll
        for (int k = 0; k < K; ++k) part[(size_t)(R.tile_base + tile_idx) * K + k] = v[k];
        __threadfence();
        const uint32_t prev = atomicAdd(cnt, 1u);
        last = (prev == (uint32_t)(R.n_tiles - 1));
    }
    __syncthreads();
    if (!last) return false;
    __threadfence();
    double s[K];
#pragma unroll
    for (int k = 0; k < K; ++k) s[k] = 0.0;
    for (int t = threadIdx.x; t < R.n_tiles; t += blockDim.x)
#pragma unroll
        for (int k = 0; k < K; ++k) s[k] += part[(size_t)(R.tile_base + t) * K + k];
    block_sum<K>(s, sh);
    if (threadIdx.x == 0) {
#pragma unroll
        for (int k = 0; k < K; ++k) out[k] = s[k];
        *cnt = 0u;
    }
    return true;
}

// --------------------------------------------------------------------------
// Packed positions: the pair kernels gather one 32-byte record per neighbour
// (x, y, z and, after the density pass, F'(rho)) instead of four arrays.
// --------------------------------------------------------------------------
__global__ void k_pack(double4* P, const double* x, int N)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < N) P[i] = make_double4(x[i], x[N + i], x[2 * N + i], 0.0);
}

__global__ void k_unpack(double* x, const double4* P, int N)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < N) {
        const double4 p = P[i];
        x[i] = p.x;
        x[N + i] = p.y;
        x[2 * N + i] = p.z;
    }
}

__device__ __forceinline__ double3 sep(const RepDesc& R, const double4& a, const double4& b)
{
    double dx = a.x - b.x, dy = a.y - b.y, dz = a.z - b.z;
    min_image(R, dx, dy, dz);
    return make_double3(dx, dy, dz);
}

// --------------------------------------------------------------------------
// Neighbour lists.  Rebuilds run only for replicas whose flag is set (an
// atom moved more than skin/2 since the last build).  Atoms are binned into
// cells of edge >= r_cut + skin, each cell's atoms are sorted by id, and
// every row is the in-order concatenation of the 27 surrounding cells'
// members within r_cut + skin, so rows have a fixed order.
// --------------------------------------------------------------------------
__global__ void k_check_displacement(NeighArgs a)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= a.N) return;
    const double4 p = a.P[i];
    const double dx = p.x - a.xref[i], dy = p.y - a.xref[a.N + i], dz = p.z - a.xref[2 * a.N + i];
    if (dx * dx + dy * dy + dz * dz > a.half_skin2) a.rebuild[a.rep_of[i]] = 1;
}

__device__ __forceinline__ int cell_coord(double x, double L, double invL, int nc)
{
    double s = x - L * floor(x * invL);   // fold into [0, L)
    int c = (int)(s * invL * nc);
    c = c < 0 ? 0 : c;
    return c >= nc ? nc - 1 : c;
}

__global__ void k_bin(NeighArgs a)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= a.N) return;
    const int r = a.rep_of[i];
    if (!a.rebuild[r]) return;
    const RepDesc& R = a.reps[r];
    if (R.nc[0] == 0) return;
    const double4 p = a.P[i];
    const int cx = cell_coord(p.x, R.L[0], R.invL[0], R.nc[0]);
    const int cy = cell_coord(p.y, R.L[1], R.invL[1], R.nc[1]);
    const int cz = cell_coord(p.z, R.L[2], R.invL[2], R.nc[2]);
    const int c = R.cell_base + (cx * R.nc[1] + cy) * R.nc[2] + cz;
    const int slot = atomicAdd(&a.cell_cnt[c], 1);
    if (slot < a.ccap)
        a.cell_atoms[(size_t)c * a.ccap + slot] = i - R.off;
    else
        atomicOr(a.status, ST_CELL_OVERFLOW);
}

// One 64-thread block per cell (grid-stride): bitonic sort of the cell's
// atom ids in LDS, occupancy copied to cell_n, bin counter reset.
__global__ __launch_bounds__(64) void k_cellsort(NeighArgs a)
{
    extern __shared__ int32_t sv[];
    for (int c = blockIdx.x; c < a.n_cells; c += gridDim.x) {
        if (!a.rebuild[a.cell_rep[c]]) continue;   // uniform in the block
        int n = a.cell_cnt[c];
        n = n > a.ccap ? a.ccap : n;
        int32_t* p = a.cell_atoms + (size_t)c * a.ccap;
        int P2 = 1;
        while (P2 < n) P2 <<= 1;
        for (int k = threadIdx.x; k < P2; k += blockDim.x) sv[k] = k < n ? p[k] : 0x7fffffff;
        __syncthreads();
        for (int size = 2; size <= P2; size <<= 1) {
            for (int stride = size >> 1; stride > 0; stride >>= 1) {
                for (int k = threadIdx.x; k < P2; k += blockDim.x) {
                    const int q = k ^ stride;
                    if (q > k) {
                        const int x = sv[k], y = sv[q];
                        if ((x > y) == ((k & size) == 0)) {
                            sv[k] = y;
                            sv[q] = x;
                        }
                    }
                }
                __syncthreads();
            }
        }
        for (int k = threadIdx.x; k < n; k += blockDim.x) p[k] = sv[k];
        __syncthreads();
        if (threadIdx.x == 0) {
            a.cell_n[c] = n;
            a.cell_cnt[c] = 0;
        }
    }
}

// Rows, T lanes per atom: each pass tests T consecutive candidates and the
// accepted ones are appended in candidate order (ballot + prefix count).
template <int T>
__global__ __launch_bounds__(kMaxBlock) void k_list(NeighArgs a)
{
    const Tile tl = a.tiles[blockIdx.x];
    if (tl.count == 0 || !a.rebuild[tl.rep]) return;
    const int lane = threadIdx.x % T;
    const int la = threadIdx.x / T;
    if (la >= tl.count) return;   // the whole T-lane group leaves together
    const RepDesc& R = a.reps[tl.rep];
    const int i = tl.first + la;
    const int il = i - R.off;
    const double4 pi = a.P[i];
    int32_t* row = a.nbr + (size_t)i * a.cap;
    const int lw = threadIdx.x & 63;
    const int gb = lw & ~(T - 1);
    const uint64_t gmask = (T == 64) ? ~0ull : ((1ull << T) - 1ull);
    const uint64_t below = (1ull << (lw - gb)) - 1ull;
    int cnt = 0;
    auto pass = [&](int jl, bool in) {
        bool acc = false;
        int j = 0;
        if (in && jl != il) {
            j = R.off + jl;
            const double3 d = sep(R, pi, a.P[j]);
            acc = d.x * d.x + d.y * d.y + d.z * d.z < a.rl2;
        }
        const uint64_t m = (__ballot(acc) >> gb) & gmask;
        const int rank = __popcll(m & below);
        if (acc && cnt + rank < a.cap) row[cnt + rank] = j;
        cnt += __popcll(m);
    };
    if (R.nc[0] == 0) {
        for (int s0 = 0; s0 < R.n; s0 += T) pass(s0 + lane, s0 + lane < R.n);
    } else {
        const int cx = cell_coord(pi.x, R.L[0], R.invL[0], R.nc[0]);
        const int cy = cell_coord(pi.y, R.L[1], R.invL[1], R.nc[1]);
        const int cz = cell_coord(pi.z, R.L[2], R.invL[2], R.nc[2]);
        for (int ox = -1; ox <= 1; ++ox) {
            const int ux = (cx + ox + R.nc[0]) % R.nc[0];
            for (int oy = -1; oy <= 1; ++oy) {
                const int uy = (cy + oy + R.nc[1]) % R.nc[1];
                for (int oz = -1; oz <= 1; ++oz) {
                    const int uz = (cz + oz + R.nc[2]) % R.nc[2];
                    const int c = R.cell_base + (ux * R.nc[1] + uy) * R.nc[2] + uz;
                    const int n = a.cell_n[c];
                    const int32_t* p = a.cell_atoms + (size_t)c * a.ccap;
                    for (int s0 = 0; s0 < n; s0 += T) {
                        const int s = s0 + lane;
                        pass(s < n ? p[s] : -1, s < n);
                    }
                }
            }
        }
    }
    if (lane == 0) {
        if (cnt > a.cap) {
            atomicOr(a.status, ST_NEIGH_OVERFLOW);
            cnt = a.cap;
        }
        a.nnb[i] = cnt;
        a.xref[i] = pi.x;
        a.xref[a.N + i] = pi.y;
        a.xref[2 * a.N + i] = pi.z;
    }
}

// --------------------------------------------------------------------------
// Density pass.  FP32 tables are staged in LDS (32 KB for rho).
// --------------------------------------------------------------------------
template <typename real, int T>
__global__ __launch_bounds__(kMaxBlock) void k_density(StepArgs a)
{
    extern __shared__ float4 lds_tab[];
    __shared__ double sh[16 * 3];
    constexpr bool kLds = sizeof(real) == 4;
    const Tile tl = a.tiles[blockIdx.x];
    if (tl.count == 0) return;   // padding tile: whole block leaves
    const RepDesc& R = a.reps[tl.rep];
    const int lane = threadIdx.x % T;
    const int la = threadIdx.x / T;
    const bool valid = la < tl.count;
    const int i = tl.first + (valid ? la : 0);
    const int N = a.N;
    const int64_t it = a.step_kernel ? *a.iter : 0;
    const int nr = a.tab.n_r;

    if (kLds && a.has_eam) {
        const float4* g = (const float4*)a.tab.rho;
        for (int k = threadIdx.x; k < nr - 1; k += blockDim.x) lds_tab[k] = g[k];
        __syncthreads();
    }

    double acc = 0.0;
    double4 pi = a.P[i];
    if (valid && a.has_eam) {
        const int n = a.nnb[i];
        const int32_t* row = a.nbr + (size_t)i * a.cap;
        const real rc2 = (real)a.tab.rc2, inv_h = (real)a.tab.inv_h_r;
        for (int b0 = lane * SB; b0 < n; b0 += T * SB) {
            real part = (real)0;
#pragma unroll
            for (int s = 0; s < SB; ++s) {
                const int q = b0 + s;
                if (q < n) {
                    const double3 d = sep(R, pi, a.P[row[q]]);
                    const real rx = (real)d.x, ry = (real)d.y, rz = (real)d.z;
                    const real r2 = rx * rx + ry * ry + rz * rz;
                    if (r2 < rc2) {
                        real t;
                        const int m = interval<real>(sqrt(r2), inv_h, nr, t);
                        if constexpr (kLds) {
                            const float4 c = lds_tab[m];
                            part += c.x + t * (c.y + t * (c.z + t * c.w));
                        } else {
                            const auto c = Tab<real>::ld4(a.tab.rho, m);
                            part += c.x + t * (c.y + t * (c.z + t * c.w));
                        }
                    }
                }
            }
            acc += Acc<real>::q(part);
        }
    }
#pragma unroll
    for (int o = T / 2; o > 0; o >>= 1) acc += __shfl_xor(acc, o, T);
    if (valid && lane == 0 && a.has_eam) {
        const double rho = Acc<real>::fin(acc);
        real t;
        const int m = interval<real>((real)rho, (real)a.tab.inv_h_rho, a.tab.n_rho, t);
        const auto c = Tab<real>::ld4(a.tab.F, m);
        const real F = c.x + t * (c.y + t * (c.z + t * c.w));
        const real Fp = (c.y + t * ((real)2 * c.z + (real)3 * t * c.w)) * (real)a.tab.inv_h_rho;
        a.P[i].w = (double)Fp;
        a.e_emb[i] = (double)F;
        if (rho > a.tab.rho_max) atomicOr(a.status, ST_TABLE_RANGE);
        if (!isfinite(rho)) atomicOr(a.status, ST_NONFINITE);
    }
    if (tl.idx == 0 && threadIdx.x == 0) a.rebuild[tl.rep] = 0;   // lists are current now

    // thermostat noise of step `it` and (fixed centre of mass) its replica sum
    if (a.step_kernel && it < a.it_last) {
        double z[3] = {0.0, 0.0, 0.0};
        if (valid && lane == 0) {
            gauss3(R.seed, (uint32_t)(i - R.off), it, 0u, z[0], z[1], z[2]);
            a.xi[i] = z[0];
            a.xi[N + i] = z[1];
            a.xi[2 * N + i] = z[2];
        }
        if (a.fix_com)
            replica_reduce<3>(z, a.noise_part, a.cnt_density + tl.rep, R, tl.idx, a.noise_sum + 3 * tl.rep, sh);
    }
}

// --------------------------------------------------------------------------
// Force pass + integration + energies + work.  FP32 pair table in LDS (64 KB).
// --------------------------------------------------------------------------
__device__ __forceinline__ void total_force(int mode, const double (&fe)[3], const double (&d)[3], double k,
                                            double k2, double lam, double (&F)[3])
{
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        switch (mode) {
        case MODE_FL: F[c] = (1.0 - lam) * fe[c] - lam * k * d[c]; break;
        case MODE_RS: F[c] = lam * fe[c]; break;
        case MODE_HH: F[c] = -((1.0 - lam) * k + lam * k2) * d[c]; break;
        default: F[c] = -lam * k * d[c]; break;
        }
    }
}

template <typename real, int T>
__global__ __launch_bounds__(kMaxBlock) void k_force(StepArgs a)
{
    extern __shared__ float4 lds_tab[];
    __shared__ double sh[16 * 2];
    constexpr bool kLds = sizeof(real) == 4;
    const Tile tl = a.tiles[blockIdx.x];
    if (tl.count == 0) return;
    const RepDesc& R = a.reps[tl.rep];
    const int lane = threadIdx.x % T;
    const int la = threadIdx.x / T;
    const bool valid = la < tl.count;
    const int i = tl.first + (valid ? la : 0);
    const int N = a.N;
    const int64_t it = a.step_kernel ? *a.iter : 0;
    const int nr = a.tab.n_r;

    if (kLds && a.has_eam) {
        const float4* g = (const float4*)a.tab.pair;
        for (int k = threadIdx.x; k < 2 * (nr - 1); k += blockDim.x) lds_tab[k] = g[k];
        __syncthreads();
    }

    const double4 pi = a.P[i];
    double f0 = 0.0, f1 = 0.0, f2 = 0.0, ep = 0.0;
    if (valid && a.has_eam) {
        const int n = a.nnb[i];
        const int32_t* row = a.nbr + (size_t)i * a.cap;
        const real Fpi = (real)pi.w;
        const real rc2 = (real)a.tab.rc2, inv_h = (real)a.tab.inv_h_r;
        for (int b0 = lane * SB; b0 < n; b0 += T * SB) {
            real p0 = (real)0, p1 = (real)0, p2 = (real)0, pe = (real)0;
#pragma unroll
            for (int s = 0; s < SB; ++s) {
                const int q = b0 + s;
                if (q < n) {
                    const double4 pj = a.P[row[q]];
                    const double3 d = sep(R, pi, pj);
                    const real rx = (real)d.x, ry = (real)d.y, rz = (real)d.z;
                    const real r2 = rx * rx + ry * ry + rz * rz;
                    if (r2 < rc2) {
                        const real r = sqrt(r2);
                        real t;
                        const int m = interval<real>(r, inv_h, nr, t);
                        real ua, ub, uc, ud, wb, wc, wd;
                        if constexpr (kLds) {
                            const float4 u = lds_tab[2 * m], w = lds_tab[2 * m + 1];
                            ua = u.x; ub = u.y; uc = u.z; ud = u.w; wb = w.x; wc = w.y; wd = w.z;
                        } else {
                            decltype(Tab<real>::ld4(a.tab.rho, 0)) u, w;
                            Tab<real>::ld8(a.tab.pair, m, u, w);
                            ua = u.x; ub = u.y; uc = u.z; ud = u.w; wb = w.x; wc = w.y; wd = w.z;
                        }
                        const real phi = ua + t * (ub + t * (uc + t * ud));
                        const real dphi = (ub + t * ((real)2 * uc + (real)3 * t * ud)) * inv_h;
                        const real drho = wb + t * (wc + t * wd);
                        const real g = dphi + (Fpi + (real)pj.w) * drho;   // dU/dr_ij
                        const real s_ = -g / r;
                        p0 += s_ * rx;
                        p1 += s_ * ry;
                        p2 += s_ * rz;
                        pe += phi;
                    }
                }
            }
            f0 += Acc<real>::q(p0);
            f1 += Acc<real>::q(p1);
            f2 += Acc<real>::q(p2);
            ep += Acc<real>::q(pe);
        }
    }
#pragma unroll
    for (int o = T / 2; o > 0; o >>= 1) {
        f0 += __shfl_xor(f0, o, T);
        f1 += __shfl_xor(f1, o, T);
        f2 += __shfl_xor(f2, o, T);
        ep += __shfl_xor(ep, o, T);
    }

    double e[2] = {0.0, 0.0};   // U_EAM contribution, |x - x0|^2
    if (valid && lane == 0) {
        const double fe[3] = {Acc<real>::fin(f0), Acc<real>::fin(f1), Acc<real>::fin(f2)};
        double x[3] = {pi.x, pi.y, pi.z};
        const double d[3] = {x[0] - a.x0[i], x[1] - a.x0[N + i], x[2] - a.x0[2 * N + i]};
        e[0] = a.has_eam ? a.e_emb[i] + 0.5 * Acc<real>::fin(ep) : 0.0;
        e[1] = d[0] * d[0] + d[1] * d[1] + d[2] * d[2];
        if (!isfinite(fe[0] + fe[1] + fe[2] + e[0] + e[1])) atomicOr(a.status, ST_NONFINITE);
        if (a.f_out) {
            a.f_out[i] = fe[0];
            a.f_out[N + i] = fe[1];
            a.f_out[2 * N + i] = fe[2];
        }
        if (a.e_atom_out) a.e_atom_out[i] = e[0];
        if (a.step_kernel) {
            const double hdt_m = 0.5 * a.dt * R.inv_m;
            double v[3] = {a.v[i], a.v[N + i], a.v[2 * N + i]};
            double F[3];
            if (it > a.it_first) {   // closing kick of step it-1 at lambda_it
                total_force(a.mode, fe, d, R.k, R.k2, a.lam[it], F);
#pragma unroll
                for (int c = 0; c < 3; ++c) v[c] += hdt_m * F[c];
            }
            if (it < a.it_last) {    // step it: B A O A with lambda_{it+1}
                total_force(a.mode, fe, d, R.k, R.k2, a.lam[it + 1], F);
                const double inv_n = 1.0 / (double)R.n;
#pragma unroll
                for (int c = 0; c < 3; ++c) {
                    v[c] += hdt_m * F[c];
                    x[c] += 0.5 * a.dt * v[c];
                    const double m = a.fix_com ? a.noise_sum[3 * tl.rep + c] * inv_n : 0.0;
                    v[c] = a.c1 * v[c] + R.c2 * (a.xi[c * N + i] - m);
                    x[c] += 0.5 * a.dt * v[c];
                }
                const double r0 = x[0] - a.xref[i], r1 = x[1] - a.xref[N + i], r2 = x[2] - a.xref[2 * N + i];
                if (r0 * r0 + r1 * r1 + r2 * r2 > a.half_skin2) a.rebuild[tl.rep] = 1;
            }
            a.Pn[i] = make_double4(x[0], x[1], x[2], 0.0);
            a.v[i] = v[0];
            a.v[N + i] = v[1];
            a.v[2 * N + i] = v[2];
        }
    }

    double tot[2];
    if (replica_reduce<2>(e, a.energy_part, a.cnt_force + tl.rep, R, tl.idx, tot, sh)) {
        if (threadIdx.x == 0) {
            a.U_rep[2 * tl.rep] = tot[0];
            a.U_rep[2 * tl.rep + 1] = tot[1];
            if (a.step_kernel && it < a.it_last) {
                const double UE = 0.5 * R.k * tot[1];
                double dH;
                switch (a.mode) {
                case MODE_FL: dH = UE - tot[0]; break;
                case MODE_RS: dH = tot[0]; break;
                case MODE_HH: dH = 0.5 * (R.k2 - R.k) * tot[1]; break;
                default: dH = UE; break;
                }
                const double W = a.W_state[tl.rep] + (a.lam[it + 1] - a.lam[it]) * dH;
                a.W_state[tl.rep] = W;
                const size_t o = (size_t)tl.rep * a.S + (size_t)(it - a.trace_off);
                if (a.dHdl_out) a.dHdl_out[o] = dH;
                if (a.W_out) a.W_out[o] = W;
            }
        }
    }
    // the last block of the whole grid advances the iteration counter
    if (a.step_kernel && threadIdx.x == 0) {
        __threadfence();
        const uint32_t prev = atomicAdd(a.cnt_all, 1u);
        if (prev == (uint32_t)(a.n_tiles - 1)) {
            *a.iter = it + 1;
            *a.cnt_all = 0u;
        }
    }
}

// --------------------------------------------------------------------------
// Initial velocities: v = sqrt(kT/m) z(stream 1, step 0), centre of mass removed
// --------------------------------------------------------------------------
__global__ void k_init_v(StepArgs a, int fix_com)
{
    __shared__ double sh[16 * 3];
    const Tile tl = a.tiles[blockIdx.x];
    if (tl.count == 0) return;
    const RepDesc& R = a.reps[tl.rep];
    const bool valid = (int)threadIdx.x < tl.count;
    const int i = tl.first + (valid ? (int)threadIdx.x : 0);
    double z[3] = {0.0, 0.0, 0.0};
    if (valid) {
        gauss3(R.seed, (uint32_t)(i - R.off), 0, 1u, z[0], z[1], z[2]);
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            z[c] *= R.sig_v;
            a.v[c * a.N + i] = z[c];
        }
    }
    if (fix_com) replica_reduce<3>(z, a.noise_part, a.cnt_density + tl.rep, R, tl.idx, a.noise_sum + 3 * tl.rep, sh);
}

__global__ void k_sub_mean_v(StepArgs a)
{
    const Tile tl = a.tiles[blockIdx.x];
    if (tl.count == 0 || (int)threadIdx.x >= tl.count) return;
    const RepDesc& R = a.reps[tl.rep];
    const int i = tl.first + threadIdx.x;
    const double inv_n = 1.0 / (double)R.n;
#pragma unroll
    for (int c = 0; c < 3; ++c) a.v[c * a.N + i] -= a.noise_sum[3 * tl.rep + c] * inv_n;
}

// --------------------------------------------------------------------------
// Launchers
// --------------------------------------------------------------------------
static int grid1(int n, int b) { return (n + b - 1) / b; }

int launch_pack(double4* P, const double* x, int N, hipStream_t s)
{
    if (N <= 0) return 0;
    hipLaunchKernelGGL(k_pack, dim3(grid1(N, 256)), dim3(256), 0, s, P, x, N);
    return (int)hipGetLastError();
}

int launch_unpack(double* x, const double4* P, int N, hipStream_t s)
{
    if (N <= 0) return 0;
    hipLaunchKernelGGL(k_unpack, dim3(grid1(N, 256)), dim3(256), 0, s, x, P, N);
    return (int)hipGetLastError();
}

int launch_check_displacement(const NeighArgs& a, hipStream_t s)
{
    if (a.N <= 0) return 0;
    hipLaunchKernelGGL(k_check_displacement, dim3(grid1(a.N, 256)), dim3(256), 0, s, a);
    return (int)hipGetLastError();
}

int launch_neigh_rebuild(const NeighArgs& a, int lanes, int block, hipStream_t s)
{
    if (a.N <= 0) return 0;
    hipLaunchKernelGGL(k_bin, dim3(grid1(a.N, 256)), dim3(256), 0, s, a);
    if (a.n_cells > 0) {
        int p2 = 1;
        while (p2 < a.ccap) p2 <<= 1;
        hipLaunchKernelGGL(k_cellsort, dim3(a.n_cells < 4096 ? a.n_cells : 4096), dim3(64), p2 * sizeof(int32_t), s,
                           a);
    }
    dim3 g(a.n_grid), b(block);
    switch (lanes) {
    case 1: hipLaunchKernelGGL((k_list<1>), g, b, 0, s, a); break;
    case 2: hipLaunchKernelGGL((k_list<2>), g, b, 0, s, a); break;
    case 4: hipLaunchKernelGGL((k_list<4>), g, b, 0, s, a); break;
    case 8: hipLaunchKernelGGL((k_list<8>), g, b, 0, s, a); break;
    case 16: hipLaunchKernelGGL((k_list<16>), g, b, 0, s, a); break;
    default: return (int)hipErrorInvalidValue;
    }
    return (int)hipGetLastError();
}

template <typename real>
static size_t lds_bytes(const StepArgs& a, int tables)
{
    return (sizeof(real) == 4 && a.has_eam) ? (size_t)tables * (a.tab.n_r - 1) * sizeof(float4) : 0;
}

template <typename real>
static int launch_density_t(const StepArgs& a, int lanes, int block, hipStream_t s)
{
    dim3 g(a.n_grid), b(block);
    const size_t sh = lds_bytes<real>(a, 1);
    switch (lanes) {
    case 1: hipLaunchKernelGGL((k_density<real, 1>), g, b, sh, s, a); break;
    case 2: hipLaunchKernelGGL((k_density<real, 2>), g, b, sh, s, a); break;
    case 4: hipLaunchKernelGGL((k_density<real, 4>), g, b, sh, s, a); break;
    case 8: hipLaunchKernelGGL((k_density<real, 8>), g, b, sh, s, a); break;
    case 16: hipLaunchKernelGGL((k_density<real, 16>), g, b, sh, s, a); break;
    default: return (int)hipErrorInvalidValue;
    }
    return (int)hipGetLastError();
}

template <typename real>
static int launch_force_t(const StepArgs& a, int lanes, int block, hipStream_t s)
{
    dim3 g(a.n_grid), b(block);
    const size_t sh = lds_bytes<real>(a, 2);
    switch (lanes) {
    case 1: hipLaunchKernelGGL((k_force<real, 1>), g, b, sh, s, a); break;
    case 2: hipLaunchKernelGGL((k_force<real, 2>), g, b, sh, s, a); break;
    case 4: hipLaunchKernelGGL((k_force<real, 4>), g, b, sh, s, a); break;
    case 8: hipLaunchKernelGGL((k_force<real, 8>), g, b, sh, s, a); break;
    case 16: hipLaunchKernelGGL((k_force<real, 16>), g, b, sh, s, a); break;
    default: return (int)hipErrorInvalidValue;
    }
    return (int)hipGetLastError();
}

int launch_density(const StepArgs& a, int precision, int lanes, int block, hipStream_t s)
{
    return precision ? launch_density_t<float>(a, lanes, block, s) : launch_density_t<double>(a, lanes, block, s);
}

int launch_force(const StepArgs& a, int precision, int lanes, int block, hipStream_t s)
{
    return precision ? launch_force_t<float>(a, lanes, block, s) : launch_force_t<double>(a, lanes, block, s);
}

int launch_init_velocities(const StepArgs& a, int n_rep, int fix_com, hipStream_t s)
{
    (void)n_rep;
    // tiles hold at most block/lanes <= 1024 atoms; one thread per atom
    hipLaunchKernelGGL(k_init_v, dim3(a.n_grid), dim3(kMaxBlock), 0, s, a, fix_com);
    if (fix_com) hipLaunchKernelGGL(k_sub_mean_v, dim3(a.n_grid), dim3(kMaxBlock), 0, s, a);
    return (int)hipGetLastError();
}

int launch_adjoint(const AdjointArgs&, const StepArgs&, int, int, int, hipStream_t) { return (int)hipErrorNotSupported; }
int launch_adjoint_finish(const unsigned long long*, int, int, double, double*, hipStream_t)
{
    return (int)hipErrorNotSupported;
}
int launch_rho_dump(const StepArgs&, double*, int, int, int, hipStream_t) { return (int)hipErrorNotSupported; }

}  // namespace eamfe
