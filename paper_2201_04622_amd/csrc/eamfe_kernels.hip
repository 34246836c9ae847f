// gfx950 kernels of the EAM switching engine.
//
// One MD iteration of a batch (every replica in the same launches):
//
//   k_bin      : finish of the previous force pass (replica energies, dH/dl,
//                the work increment of Eq. w_irr, iteration counter) and the
//                prefix of the replicas whose lists are due, in blocks 0
//                and 1; binning of those replicas' atoms into cells in the
//                others;
//   k_list     : Verlet rows within r_cut + skin, one wavefront per atom,
//                each cell's members taken in id order;
//   k_density  : rho_i = sum_j rho(r_ij) over the row, F(rho_i), F'(rho_i),
//                the thermostat noise of the step with its replica sum, and
//                the bin counters of the rebuilt replicas cleared;
//   k_force    : pair + embedding forces, the Einstein spring, the lambda
//                blend (Eq. interp) or scale (Eq. H_rs), the closing B
//                half-kick of the previous step and B-A-O-A of the next one
//                (BAOAB), per-unit energy partials and the list-due flags.
//
// The pair kernels run a persistent grid over work units (one wavefront's
// atoms of one replica); T lanes cooperate on one atom, lane t taking blocks
// of SB consecutive neighbour slots t, t+T, ...  In FP32 each block's
// partial sum is rounded to a 2^-32 grid and added as an exact integer held
// in a float64, so the per-atom sums do not depend on T or on the block
// size.  Rows have a fixed order and per-replica sums are taken over unit
// partials in a fixed order, so runs are bitwise reproducible.
#include "eamfe_internal.h"

#include <hip/hip_ext.h>

#include <vector>

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

// The same deviates split over two lanes that share the counter: half 0
// gives (z0, z1) from u0, u1 and half 1 gives z2 from u2, u3, so a
// wavefront evaluates one logarithm, one root and one sine/cosine pair for
// the three.
__device__ __forceinline__ void gauss3_half(uint64_t seed, uint32_t atom, int64_t step, uint32_t stream, int half,
                                            double& za, double& zb)
{
    const uint64_t st = (uint64_t)step;
    uint32_t c0 = atom, c1 = (uint32_t)st, c2 = stream, c3 = (uint32_t)(st >> 32);
    philox4x32_10(c0, c1, c2, c3, (uint32_t)seed, (uint32_t)(seed >> 32));
    const double s = 2.3283064365386963e-10;
    const double twopi = 6.283185307179586476925286766559;
    const double ua = ((double)(half ? c2 : c0) + 1.0) * s, ub = ((double)(half ? c3 : c1) + 1.0) * s;
    const double r = sqrt(-2.0 * log(ua));
    double sn, cs;
    sincos(twopi * ub, &sn, &cs);
    za = r * cs;
    zb = r * sn;
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
// FP32 with kFix: the partial is rounded to the 2^-32 grid and carried as an
// exact integer, so the sum does not depend on how slots are grouped into
// lanes; without kFix the float32 partials are added in float64 as they are
// (a fixed order for one launch shape, so still reproducible run to run).
template <typename real, bool kFix>
struct Acc;
template <bool kFix>
struct Acc<double, kFix> {
    static __device__ __forceinline__ double q(double p) { return p; }
    static __device__ __forceinline__ double fin(double a) { return a; }
};
template <>
struct Acc<float, true> {
    static __device__ __forceinline__ double q(float p) { return rint((double)p * kFixScale); }
    static __device__ __forceinline__ double fin(double a) { return a * kFixInv; }
};
template <>
struct Acc<float, false> {
    static __device__ __forceinline__ double q(float p) { return (double)p; }
    static __device__ __forceinline__ double fin(double a) { return a; }
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

// The same without the clamp, for the FP32 tables in LDS: they carry one
// padding interval past the last knot (the end value, zero slope), so any
// 0 <= x <= x_max (1 + a few ulp), which is what the callers pass, stays in
// range.  x = r comes from a masked r^2 and is finite.
__device__ __forceinline__ int interval_pad(float x, float inv_h, float& t)
{
    const float p = x * inv_h;
    const int m = (int)p;
    t = p - (float)m;
    return m;
}

__device__ __forceinline__ void min_image(const RepDesc& R, double& dx, double& dy, double& dz)
{
    dx -= R.L[0] * rint(dx * R.invL[0]);
    dy -= R.L[1] * rint(dy * R.invL[1]);
    dz -= R.L[2] * rint(dz * R.invL[2]);
}


// 1/r and r from r^2: hardware reciprocal square root in FP32 (about 1 ulp),
// correctly rounded sqrt and division in FP64.
template <typename real>
struct Root;
template <>
struct Root<float> {
    static __device__ __forceinline__ void of(float r2, float& r, float& ir)
    {
        ir = __builtin_amdgcn_rsqf(r2);
        r = r2 * ir;
    }
};
template <>
struct Root<double> {
    static __device__ __forceinline__ void of(double r2, double& r, double& ir)
    {
        r = sqrt(r2);
        ir = 1.0 / r;
    }
};

// Neighbour rows are stored in slabs of four slots: slot s of atom i is at
// nbr[((s / 4) * N + i) * 4 + s % 4].  A lane reads four consecutive slots
// with one 16-byte load, and the lanes of a wavefront, which hold
// consecutive atoms, read consecutive 16-byte words.  The list builder pads
// every row with the atom's own id up to a multiple of four, so whole slabs
// below the row length are always valid ids.
__device__ __forceinline__ size_t slot_index(int i, int s, int N)
{
    return ((size_t)(s >> 2) * (size_t)N + (size_t)i) * 4 + (size_t)(s & 3);
}

__device__ __forceinline__ int4 row_slab(const int32_t* nbr, int i, int b0, int N)
{
    return *(const int4*)(nbr + ((size_t)(b0 >> 2) * (size_t)N + (size_t)i) * 4);
}

// Records of one lane block's SB neighbours: box coordinates and F' bits
// (FP32 form: record j - qoff of Q, a 32-bit byte offset from its base, with
// Q the global array and qoff 0, or a replica's records staged in LDS and
// qoff its first atom) or packed positions (FP64 form).
template <bool kQ>
struct Nb;
template <>
struct Nb<true> {
    uint4 v[SB];
};
template <>
struct Nb<false> {
    double4 v[SB];
};

template <bool kQ>
__device__ __forceinline__ Nb<kQ> gather(const double4* P, const uint4* Q, int qoff, int4 j)
{
    Nb<kQ> g;
    const int js[SB] = {j.x, j.y, j.z, j.w};
#pragma unroll
    for (int s = 0; s < SB; ++s) {
        if constexpr (kQ) g.v[s] = *(const uint4*)((const char*)Q + (uint32_t)(js[s] - qoff) * 16u);
        else g.v[s] = P[js[s]];
    }
    return g;
}

// One lane's walk over the row of atom i (n slots): its blocks k = 0..nb-1
// hold slots lane SB + k T SB .. + SB - 1 (slab lane + k T).  Software
// pipeline: while block k is computed, the ids of block k+2 and (FP32 form;
// the FP64 records are too large to hold twice) the records of block k+1
// are in flight, so a wavefront does not wait on memory between blocks.
// Each iteration issues the slab load before the gathers, so the next
// iteration's wait for the ids does not also wait for those gathers.  Past
// the end the last block's slab and records are read again (in bounds,
// unused).  The scheduling barrier keeps the loads ahead of the arithmetic
// they overlap.
template <bool kQ, int T, typename Body>
__device__ __forceinline__ void walk_row(const int32_t* nbr, const double4* P, const uint4* Q, int qoff, int N,
                                         int i, int lane, int n, Body&& body)
{
    const int first = lane * SB;
    if (first >= n) return;
    const int nb = (n - first + T * SB - 1) / (T * SB);
    const size_t str = (size_t)T * N;
    const int4* slab = (const int4*)nbr + (size_t)lane * N + i;
    const int4* last = slab + (size_t)(nb - 1) * str;
    if constexpr (kQ) {
        // two record buffers in turn (no copies between iterations)
        // both slab loads ahead of the first gathers, as in the loop, so the
        // loop's waits on entry are the same as on its back edge
        const int4 id0 = slab[0];
        const int4* pn = nb > 1 ? slab + str : last;   // slab of block k+1
        int4 ids = *pn;
        __builtin_amdgcn_sched_barrier(0);
        Nb<true> A = gather<true>(P, Q, qoff, id0), B;
        for (int k = 0;;) {
            int4 idn = ids;
            pn = pn == last ? last : pn + str;          // block k+2
            ids = *pn;
            __builtin_amdgcn_sched_barrier(0);
            B = gather<true>(P, Q, qoff, idn);
            __builtin_amdgcn_sched_barrier(0);
            body(A, first + k * T * SB);
            if (++k == nb) break;
            idn = ids;
            pn = pn == last ? last : pn + str;
            ids = *pn;
            __builtin_amdgcn_sched_barrier(0);
            A = gather<true>(P, Q, qoff, idn);
            __builtin_amdgcn_sched_barrier(0);
            body(B, first + k * T * SB);
            if (++k == nb) break;
        }
    } else {
        const int4* pn = slab;
        int4 ids = *pn;
        for (int k = 0; k < nb; ++k) {
            const int4 idc = ids;
            pn = pn == last ? last : pn + str;          // block k+1
            ids = *pn;
            const Nb<false> cur = gather<false>(P, Q, qoff, idc);
            __builtin_amdgcn_sched_barrier(0);
            body(cur, first + k * T * SB);
        }
    }
}

// --------------------------------------------------------------------------
// Work distribution and deterministic reductions
//
// The pair kernels run persistent blocks whose wavefronts each take a fixed
// stride of work units (one unit = the atoms of one wavefront, 64/T atoms of
// one replica).  With XCD affinity the units are split into eight groups
// (the replicas binned to XCD x) and group x is spread over the blocks with
// blockIdx.x % 8 == x, the blocks the hardware places on XCD x.  Per-replica
// sums are never finished inside a pass: each unit writes its partial to a
// fixed slot, and a later kernel (the stream orders them) adds a replica's
// slots in unit order.  Results therefore do not depend on which wavefront
// took which unit, and the pair kernels need no atomics or fences.
// --------------------------------------------------------------------------
__device__ __forceinline__ int wave_lane() { return (int)(threadIdx.x & 63u); }

// The value of lane (l xor o) of a wavefront.  For o = 1, 2, 4, 8 the lanes
// move through DPP within each 16-lane row, which costs no LDS traffic and
// little latency: quad permutations for 1 and 2, a half-row mirror (l xor 7)
// followed by a quad reversal (l xor 3) for 4, a row rotation by 8 for 8;
// wider partners go through the LDS permute.  o is a compile-time constant
// at every call (unrolled loops), and every lane of the wavefront is active
// there (wave-uniform control flow), so each lane reads a live value.
__device__ __forceinline__ int xor_lanes(int v, int o)
{
    switch (o) {
    case 1: return __builtin_amdgcn_update_dpp(0, v, 0xB1, 0xF, 0xF, false);   // quad_perm [1, 0, 3, 2]
    case 2: return __builtin_amdgcn_update_dpp(0, v, 0x4E, 0xF, 0xF, false);   // quad_perm [2, 3, 0, 1]
    case 4: {
        const int t = __builtin_amdgcn_update_dpp(0, v, 0x141, 0xF, 0xF, false);   // row_half_mirror: l xor 7
        return __builtin_amdgcn_update_dpp(0, t, 0x1B, 0xF, 0xF, false);          // quad_perm [3, 2, 1, 0]
    }
    case 8: return __builtin_amdgcn_update_dpp(0, v, 0x128, 0xF, 0xF, false);  // row_ror:8
    default: return __shfl_xor(v, o, 64);
    }
}

__device__ __forceinline__ double xor_lanes(double v, int o)
{
    const unsigned long long b = (unsigned long long)__double_as_longlong(v);
    const unsigned int lo = (unsigned int)xor_lanes((int)(unsigned int)b, o);
    const unsigned int hi = (unsigned int)xor_lanes((int)(unsigned int)(b >> 32), o);
    return __longlong_as_double((long long)(((unsigned long long)hi << 32) | lo));
}

// Inclusive prefix sum over the 64 lanes of a wavefront (every lane active):
// within each 16-lane row by DPP row shifts of 1, 2, 4 and 8 (a lane shifted
// in from outside the row adds the zero of the update's old value), then
// across rows by broadcasting lane 15 into row 1 and lane 47 into row 3, and
// lane 31 into rows 2 and 3.  Integer adds: the same result as any order.
__device__ __forceinline__ int wave_scan(int x)
{
    x += __builtin_amdgcn_update_dpp(0, x, 0x111, 0xF, 0xF, false);   // row_shr:1
    x += __builtin_amdgcn_update_dpp(0, x, 0x112, 0xF, 0xF, false);   // row_shr:2
    x += __builtin_amdgcn_update_dpp(0, x, 0x114, 0xF, 0xF, false);   // row_shr:4
    x += __builtin_amdgcn_update_dpp(0, x, 0x118, 0xF, 0xF, false);   // row_shr:8
    x += __builtin_amdgcn_update_dpp(0, x, 0x142, 0xA, 0xF, false);   // row_bcast:15, rows 1 and 3
    x += __builtin_amdgcn_update_dpp(0, x, 0x143, 0xC, 0xF, false);   // row_bcast:31, rows 2 and 3
    return x;
}

// sum over the 64 lanes of a wavefront in a fixed butterfly order
template <int K>
__device__ __forceinline__ void wave_sum(double (&v)[K])
{
#pragma unroll
    for (int o = 32; o > 0; o >>= 1)
#pragma unroll
        for (int k = 0; k < K; ++k) v[k] += xor_lanes(v[k], o);
}

// Store the wavefront's sum of K per-lane values as unit `idx`'s partial
// (tile_base: the replica's first unit slot).
template <int K>
__device__ __forceinline__ void unit_partial(const double (&vin)[K], double* part, int tile_base, int idx)
{
    double v[K];
#pragma unroll
    for (int k = 0; k < K; ++k) v[k] = vin[k];
    wave_sum<K>(v);
    if (wave_lane() == 0)
#pragma unroll
        for (int k = 0; k < K; ++k) part[(size_t)(tile_base + idx) * K + k] = v[k];
}

template <int K>
__device__ __forceinline__ void unit_partial(const double (&vin)[K], double* part, const RepDesc& R, int idx)
{
    unit_partial<K>(vin, part, R.tile_base, idx);
}

// Exact replica sums of the fixed-point form: each lane's value is rounded to
// a multiple of 2^-36 (noise, velocities) or 2^-24 (energies, virials) before
// its unit partial, so every float64 add of partials and totals is exact while
// a replica's total stays below 2^17 or 2^29 in magnitude.  The totals are
// then the same for every grouping of atoms into units, i.e. for every number
// of lanes per atom.
constexpr double kGridZ = 68719476736.0, kGridZInv = 1.0 / 68719476736.0;
constexpr double kGridE = 16777216.0, kGridEInv = 1.0 / 16777216.0;

template <int M, int K>   // the first M of the K values
__device__ __forceinline__ void on_grid(double (&v)[K], double g, double gi)
{
#pragma unroll
    for (int k = 0; k < M; ++k) v[k] = rint(v[k] * g) * gi;
}

// A replica's total of the partials written by an earlier kernel: lanes take
// the units in a fixed stride, then a fixed butterfly; every lane gets it.
template <int K>
__device__ __forceinline__ void replica_total(const double* part, const RepDesc& R, double (&out)[K])
{
#pragma unroll
    for (int k = 0; k < K; ++k) out[k] = 0.0;
    for (int t = wave_lane(); t < R.n_tiles; t += 64)
#pragma unroll
        for (int k = 0; k < K; ++k) out[k] += part[(size_t)(R.tile_base + t) * K + k];
    wave_sum<K>(out);
}

// The same total in two halves, so that its loads can go out with other
// loads: replica_loads issues the partials of the lane's first two units
// (t = lane, lane + 64; a unit past the replica's last reads unit 0 and is
// dropped), replica_finish adds them and any further units in the order of
// replica_total and takes the butterfly, so the result is the same bits.
// tb, nt: the replica's first unit slot and its number of units.
template <int K>
struct PartPair {
    double p[2][K];
};

template <int K>
__device__ __forceinline__ PartPair<K> replica_loads(const double* part, int tb, int nt)
{
    PartPair<K> q;
#pragma unroll
    for (int h = 0; h < 2; ++h) {
        const int t = wave_lane() + 64 * h;
        const size_t o = (size_t)(tb + (t < nt ? t : 0)) * K;
#pragma unroll
        for (int k = 0; k < K; ++k) q.p[h][k] = part[o + k];
    }
    return q;
}

template <int K>
__device__ __forceinline__ void replica_finish(const PartPair<K>& q, const double* part, int tb, int nt,
                                               double (&out)[K])
{
#pragma unroll
    for (int k = 0; k < K; ++k) out[k] = 0.0;
#pragma unroll
    for (int h = 0; h < 2; ++h)
        if (wave_lane() + 64 * h < nt)
#pragma unroll
            for (int k = 0; k < K; ++k) out[k] += q.p[h][k];
    for (int t = wave_lane() + 128; t < nt; t += 64)
#pragma unroll
        for (int k = 0; k < K; ++k) out[k] += part[(size_t)(tb + t) * K + k];
    wave_sum<K>(out);
}

// Run body(u) for every unit of this wavefront's stride.  Uniform loop
// bounds (scalar values) keep the whole body wave-uniform.
template <typename Body>
__device__ __forceinline__ void for_each_unit(const int* qoff, int nq, int grid, Body&& body)
{
    const int wpb = (int)(blockDim.x >> 6);
    const int wib = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
    const int x = nq > 1 ? (int)(blockIdx.x % (unsigned)nq) : 0;
    const int lb = (int)(blockIdx.x / (unsigned)nq);                 // block index among group x's blocks
    const int nb = (grid - x + nq - 1) / nq;                       // blocks serving group x (of the grid's first `grid`)
    const int first = qoff[x], len = qoff[x + 1] - qoff[x];
    for (int u = lb * wpb + wib; u < len; u += nb * wpb) body(first + u);
}

// Block-wide copy of n 16-byte items, U per thread per round: a round's
// loads all go out before its first store, so the copy waits on memory once
// per round rather than once per item.  Past the end a lane reads item n - 1
// again (in bounds, not stored): loads without a condition cannot be moved
// behind the stores.
template <int U, typename V, typename Ld, typename St>
__device__ __forceinline__ void copy_rounds(int n, Ld&& ld, St&& st)
{
    const int bs = (int)blockDim.x;
    for (int k0 = threadIdx.x; k0 < n; k0 += U * bs) {
        V v[U];
#pragma unroll
        for (int u = 0; u < U; ++u) v[u] = ld(min(k0 + u * bs, n - 1));
        __builtin_amdgcn_sched_barrier(0);   // every load of the round issued before the stores
#pragma unroll
        for (int u = 0; u < U; ++u)
            if (k0 + u * bs < n) st(k0 + u * bs, v[u]);
    }
}

// Units of a pair launch.  Persistent form: for_each_unit over the unit
// groups.  Staged form: block b serves slice b (a run of units of one
// replica): it copies that replica's records into LDS at st and its
// wavefronts take the slice's units in turn, gathering neighbours from LDS.
// stage_table() copies the pair kernel's table into LDS; in the staged
// form the records are copied in the same phase, behind one barrier (the
// slice carries its replica's first atom and size, so nothing waits on
// further descriptor loads), and each wavefront's first unit descriptor is
// read before the copy, so its latency hides under the copy's.
// body(tile) runs one unit.
template <bool kStage, typename Table, typename Body>
__device__ __forceinline__ void run_units(const StepArgs& a, uint4* st, Table&& stage_table, Body&& body)
{
    if constexpr (kStage) {
        const int4 sl = a.slices[blockIdx.x];   // first unit, units, replica's first atom, atoms
        if (sl.y <= 0) return;                  // uniform over the block
        const int wpb = (int)(blockDim.x >> 6);
        const int wib = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
        Tile first{};
        if (wib < sl.y) first = a.tiles[sl.x + wib];
        stage_table();
        copy_rounds<4, uint4>(sl.w, [&](int k) { return a.Q[sl.z + k]; }, [&](int k, const uint4& q) { st[k] = q; });
        __syncthreads();
        for (int u = wib; u < sl.y; u += wpb) body(u == wib ? first : a.tiles[sl.x + u]);
    } else {
        if (a.has_eam) {
            stage_table();
            __syncthreads();
        }
        for_each_unit(a.qoff, a.nq, (int)gridDim.x - a.finish_prev,
                      [&](int tix) { body(a.tiles[tix]); });   // a finish block is the last
    }
}

// --------------------------------------------------------------------------
// Packed positions: the pair kernels gather one 32-byte record per neighbour
// (x, y, z and, after the density pass, F'(rho)) instead of four arrays.
// --------------------------------------------------------------------------
// Box coordinate of x along an axis of length L: frac(x/L) as a 32-bit
// fixed-point number.  The signed 32-bit difference of two box coordinates
// is the minimum-image separation in units of L/2^32 (integer wrap-around is
// the periodicity), exact up to the 2^-32 L quantum.
__device__ __forceinline__ uint32_t box_code(double x, double invL)
{
    double f = x * invL;
    f -= floor(f);
    return (uint32_t)(unsigned long long)(f * 4294967296.0);   // f == 1.0 wraps to 0
}

__device__ __forceinline__ uint4 box_codes(const RepDesc& R, double x, double y, double z, uint32_t w)
{
    return make_uint4(box_code(x, R.invL[0]), box_code(y, R.invL[1]), box_code(z, R.invL[2]), w);
}

// A stencil cell index cell + d, d in -2..2, folded into 0..n-1: with five
// or more cells per edge (the list planner's condition for cells) it wraps
// at most once, so no integer division is needed.
__device__ __forceinline__ int wrap_cell(int u, int n)
{
    u = u < 0 ? u + n : u;
    return u >= n ? u - n : u;
}

// Cell of a box coordinate on an nc-cell axis (exact integer arithmetic).
__device__ __forceinline__ int box_cell(uint32_t q, int nc) { return (int)(((uint64_t)q * (uint64_t)nc) >> 32); }

__global__ void k_pack(double4* P, uint4* Q, const double* x, const int32_t* rep_of, const RepDesc* reps, int N)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= N) return;
    P[i] = make_double4(x[i], x[N + i], x[2 * N + i], 0.0);
    Q[i] = box_codes(reps[rep_of[i]], x[i], x[N + i], x[2 * N + i], 0u);
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
// cells of edge >= (r_cut + skin) / 2 (in arrival order), and every row is
// the concatenation, cell by cell in stencil order with each cell's members
// in id order, of the members within r_cut + skin of the 5 x 5 x 5 cells
// around the atom's own, so rows have a fixed order.
// --------------------------------------------------------------------------
// Prefix sums over the replicas of the global builder (not k_rows_lds) of
// the atoms and of the cells to rebuild:
// pre[r] (atoms of flagged replicas before r), pre[n_rep + 1 + r] (cells of
// flagged replicas before r), totals at index n_rep and 2 n_rep + 1.  One
// block (any size, multiple of 64); the list kernels take their work items
// from these, so each of them needs no pass over all atoms or cells.  Every
// thread returns the number of flagged replicas.
__device__ int flag_prefix(const RepDesc* reps, const int32_t* rebuild, int n_rep, int32_t* pre)
{
    __shared__ int wa[16], wc[16], wr[16];
    const int lw = threadIdx.x & 63, w = threadIdx.x >> 6, nw = blockDim.x >> 6;
    int ca = 0, cc = 0, cr = 0;
    for (int base = 0; base < n_rep; base += blockDim.x) {
        const int r = base + threadIdx.x;
        int va = 0, vc = 0;
        if (r < n_rep && rebuild[r] && !reps[r].lds) {   // replicas of the global builder only
            va = reps[r].n;
            vc = reps[r].nc[0] * reps[r].nc[1] * reps[r].nc[2];
        }
        const int xa = wave_scan(va), xc = wave_scan(vc);
        const int nf = __popcll(__ballot(va > 0));   // flagged replicas of this wavefront
        if (lw == 63) {
            wa[w] = xa;
            wc[w] = xc;
            wr[w] = nf;
        }
        __syncthreads();
        int oa = 0, oc = 0, ta = 0, tc = 0, tr = 0;
        for (int q = 0; q < nw; ++q) {
            oa += q < w ? wa[q] : 0;
            oc += q < w ? wc[q] : 0;
            ta += wa[q];
            tc += wc[q];
            tr += wr[q];
        }
        if (r < n_rep) {
            pre[r] = ca + oa + xa - va;
            pre[n_rep + 1 + r] = cc + oc + xc - vc;
        }
        ca += ta;
        cc += tc;
        cr += tr;
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        pre[n_rep] = ca;
        pre[2 * n_rep + 1] = cc;
    }
    return cr;
}

// Replica holding work item f of a prefix p[0..n_rep] (non-decreasing,
// p[0] = 0, p[n_rep] > f): the last r with p[r] <= f, which skips replicas
// with no items; p_lo returns p[r] and r_off the replica's first atom, both
// from the probes (each probe also reads its replica's first atom, in the same
// round).  Called by a whole wavefront with a uniform f: each round its 64
// lanes probe 64 evenly spaced entries and a ballot counts those <= f, so up
// to 64 replicas take one round of loads (a binary search, one load per
// level, would chain six).  Every probe is in bounds whatever f is.
__device__ __forceinline__ int item_replica(const int32_t* p, const RepDesc* reps, int n_rep, int f, int& p_lo,
                                            int& r_off)
{
    const int lw = threadIdx.x & 63;
    int lo = 0, hi = n_rep;   // p[lo] <= f < p[hi]
    int plo = 0, olo = 0;     // p[0] and the first atom of replica 0
    while (hi - lo > 1) {
        const int stride = (hi - lo + 63) >> 6;
        const int idx = lo + stride * (lw + 1);
        const bool in = idx < hi;
        const int v = in ? p[idx] : 0x7fffffff;
        const int o = in ? reps[idx].off : 0;
        const int k = __popcll(__ballot(v <= f));   // the probes <= f are a prefix of the lanes
        if (k > 0) {
            plo = __builtin_amdgcn_readlane(v, k - 1);
            olo = __builtin_amdgcn_readlane(o, k - 1);
        }
        lo += stride * k;
        hi = min(hi, lo + stride);
    }
    p_lo = plo;
    r_off = olo;
    return lo;
}

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

__device__ void finish_body(const StepArgs& a, int64_t it);   // below, with the force pass

// First kernel of the global list pass; its blocks take two independent
// jobs.  Block 0 forms the prefix of the flagged replicas' atoms and cells
// that the next two kernels take their work items from; the other blocks
// bin the atoms of the flagged replicas, one atom per thread with a flag
// test each (the prefix is not formed yet).
constexpr int kBinBlock = 1024;

__global__ __launch_bounds__(kBinBlock) void k_bin(NeighArgs a, StepArgs s)
{
    if (blockIdx.x == 0) {
        const int flagged = flag_prefix(a.reps, a.rebuild, a.n_rep, a.flag_pre);
        if (s.step_kernel && threadIdx.x == 0 && flagged > 0) {   // rebuild history of the step passes (no zeros)
            s.row_acc[a.n_rep + 1] += (double)flagged;
            s.row_acc[a.n_rep + 2] += (double)a.flag_pre[a.n_rep];
        }
        return;
    }
    const int stride = (gridDim.x - 1) * blockDim.x;
    for (int i = (blockIdx.x - 1) * blockDim.x + threadIdx.x; i < a.N; i += stride) {
        // the atom's record goes out with its replica id, and the flag with the
        // replica's fields: two rounds of loads ahead of the count, not four
        // (the empty asm takes every value before the tests, so the compiler
        // cannot sink the reads behind them; the record is used only for an
        // atom of a flagged replica)
        const int r = a.rep_of[i];
        const uint4 q = a.Q[i];
        const int fl = a.rebuild[r];
        const RepDesc& R = a.reps[r];
        const int nc0 = R.nc[0], nc1 = R.nc[1], nc2 = R.nc[2], lds = R.lds, cbase = R.cell_base, roff = R.off;
        __asm__ volatile("" : : "v"(q.x), "v"(q.y), "v"(q.z), "v"(fl), "v"(nc0), "v"(nc1), "v"(nc2), "v"(lds),
                         "v"(cbase), "v"(roff));
        if (!fl || nc0 == 0 || lds) continue;   // all-pairs rows, or rows built from LDS: no global cells
        const int c = cbase + (box_cell(q.x, nc0) * nc1 + box_cell(q.y, nc1)) * nc2 + box_cell(q.z, nc2);
        const int slot = atomicAdd(&a.cell_cnt[c], 1);
        if (slot < a.ccap)
            a.cell_atoms[(size_t)c * a.ccap + slot] = i - roff;
        else
            atomicOr(a.status, ST_CELL_OVERFLOW);
    }
}

// Rows: one wavefront per atom of a flagged replica (waves of the whole grid
// stride over the flagged atoms, work items from the prefix).  The 125
// stencil cells' members form one candidate stream in a fixed order (cells
// by offset, atoms by id).  The stream is staged in LDS a chunk at a time:
// each lane copies one cell's members (their loads in flight together) and
// sorts them (a sorting network of eight, an insertion sort beyond), so the
// cells need no sorting pass of their own and a candidate costs one LDS read.
// Each pass tests 64 candidates with exact minimum-image box coordinates and
// appends the accepted ones in stream order (ballot + prefix count) to a row
// buffer in LDS, which is written out as whole 16-byte slabs at the end (row
// stores inside the loop would make every pass's loads wait for them).
constexpr int kListBlock = 256;
constexpr int kListGrid = 2048;
constexpr int kStencil = 125;   // 5 x 5 x 5 cells

__global__ __launch_bounds__(kListBlock) void k_list(NeighArgs a, int n_rep)
{
    extern __shared__ int rowbuf[];             // [waves][cap] accepted ids, then [waves][chunk] candidates
    __shared__ int cend[kListBlock / 64][kStencil];   // per wave: inclusive prefix of stencil cell sizes
    __shared__ int cid[kListBlock / 64][kStencil];    // per wave: global stencil cell ids
    const int lw = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int cap = a.cap, N = a.N;
    const float rl2 = a.rl2_f;
    int* row = rowbuf + (size_t)w * cap;
    int* cb = rowbuf + (size_t)(kListBlock / 64) * cap + (size_t)w * a.chunk;   // this wave's candidate chunk
    const int32_t* pre = a.flag_pre;
    const uint64_t below = (1ull << lw) - 1ull;
    const int waves = gridDim.x * (kListBlock / 64);
    // the wave's first item: its replica's probes go out with the total's
    // read (the empty asm takes their results before the loop's test, so the
    // compiler cannot sink them behind it)
    const int f0 = blockIdx.x * (kListBlock / 64) + w;
    const int total = pre[n_rep];
    int plo0, off0;
    const int lo0 = item_replica(pre, a.reps, n_rep, f0, plo0, off0);
    __asm__ volatile("" : : "v"(lo0), "v"(plo0), "v"(off0));
    for (int f = f0; f < total; f += waves) {
        int plo = plo0, roff = off0;
        const int lo = f == f0 ? lo0 : item_replica(pre, a.reps, n_rep, f, plo, roff);
        const RepDesc& R = a.reps[lo];
        const int il = f - plo;
        const int i = roff + il;
        // the atom's record and reference position go out with the
        // replica's fields (the empty asm again keeps the field reads from
        // sinking into the branches that use them)
        const uint4 qi = a.Q[i];
        const double4 pi = a.P[i];   // the list's reference position, read with the record
        const int rn = R.n, nc0 = R.nc[0], nc1 = R.nc[1], nc2 = R.nc[2], cbase = R.cell_base;
        const double L0 = R.L[0], L1 = R.L[1], L2 = R.L[2];
        __asm__ volatile("" : : "v"(rn), "v"(nc0), "v"(nc1), "v"(nc2), "v"(cbase));
        const float sx = (float)(L0 * 2.3283064365386963e-10), sy = (float)(L1 * 2.3283064365386963e-10),
                    sz = (float)(L2 * 2.3283064365386963e-10);
        int cnt = 0;
        auto test = [&](int jl) {
            const uint4 qj = a.Q[roff + jl];
            const float dx = (float)(int)(qi.x - qj.x) * sx, dy = (float)(int)(qi.y - qj.y) * sy,
                        dz = (float)(int)(qi.z - qj.z) * sz;
            return jl != il && dx * dx + dy * dy + dz * dz < rl2;
        };
        auto append = [&](bool acc, int j) {
            const uint64_t m = __ballot(acc);
            const int rank = __popcll(m & below);
            if (acc && cnt + rank < cap) row[cnt + rank] = j;
            cnt += __popcll(m);
        };
        if (nc0 == 0) {
            for (int s0 = 0; s0 < rn; s0 += 64) {
                const int jl = s0 + lw;
                append(jl < rn && test(jl), roff + jl);
            }
        } else {   // cells
            const int cx = box_cell(qi.x, nc0), cy = box_cell(qi.y, nc1), cz = box_cell(qi.z, nc2);
            // lane l holds stencil cells l and 64 + l: both cells' counts are
            // read together, then prefix-summed in stencil order
            int n_c[2] = {0, 0}, cc[2] = {0, 0};
#pragma unroll
            for (int h = 0; h < 2; ++h) {
                const int q = 64 * h + lw;
                if (q < kStencil) {
                    const int ux = wrap_cell(cx + q / 25 - 2, nc0);
                    const int uy = wrap_cell(cy + (q / 5) % 5 - 2, nc1);
                    const int uz = wrap_cell(cz + q % 5 - 2, nc2);
                    cc[h] = cbase + (ux * nc1 + uy) * nc2 + uz;
                    n_c[h] = min(a.cell_cnt[cc[h]], a.ccap);
                }
            }
            int tot_c = 0;   // running total of the stencil cells' sizes
#pragma unroll
            for (int h = 0; h < 2; ++h) {
                const int q = 64 * h + lw;
                const int incl = wave_scan(n_c[h]) + tot_c;
                if (q < kStencil) {
                    cend[w][q] = incl;
                    cid[w][q] = cc[h];
                }
                tot_c = __builtin_amdgcn_readlane(incl, 63);
            }
            __builtin_amdgcn_wave_barrier();
            constexpr int U = 4;   // passes per iteration: their independent loads are in flight together
            int q0 = 0, base = 0;  // first stencil cell of the chunk, candidates before it
            while (q0 < kStencil) {
                // the cells (up to 128, two per lane) whose members fit the chunk
                // (a cell always does: chunk >= ccap)
                int q1 = q0;
#pragma unroll
                for (int h = 0; h < 2; ++h) {
                    const int qq = q0 + 64 * h + lw;
                    const int c = __popcll(__ballot(qq < kStencil && cend[w][qq] - base <= a.chunk));
                    if (q1 == q0 + 64 * h) q1 += c;   // uniform
                }
                q1 = q1 > q0 ? q1 : q0 + 1;
                const int end = cend[w][q1 - 1] - base;
                // lane l stages cells q0 + l and q0 + 64 + l in id order with a
                // sorting network (Batcher's odd-even merge): eight inputs, or
                // sixteen when some cell of the wavefront holds more than eight
                // (a uniform branch), an insertion sort beyond
                int s0[2], n[2];
                const int32_t* src[2];
#pragma unroll
                for (int h = 0; h < 2; ++h) {
                    const int qq = q0 + 64 * h + lw;
                    const bool mine = qq < q1;
                    s0[h] = mine ? (qq ? cend[w][qq - 1] : 0) - base : 0;
                    n[h] = mine ? cend[w][qq] - base - s0[h] : 0;
                    src[h] = a.cell_atoms + (size_t)(mine ? cid[w][qq] : 0) * a.ccap;
                }
                auto cmpx = [](int* v, int p, int r) {
                    const int lo = min(v[p], v[r]), hi = max(v[p], v[r]);
                    v[p] = lo;
                    v[r] = hi;
                };
                if (__ballot(n[0] > 8 || n[1] > 8) == 0) {
                    int m[2][8];   // both cells' loads in flight together
#pragma unroll
                    for (int h = 0; h < 2; ++h)
#pragma unroll
                        for (int t = 0; t < 8; ++t) m[h][t] = t < n[h] ? src[h][t] : 0x7fffffff;
#pragma unroll
                    for (int h = 0; h < 2; ++h) {
                        int* v = m[h];
                        cmpx(v, 0, 1); cmpx(v, 2, 3); cmpx(v, 4, 5); cmpx(v, 6, 7);
                        cmpx(v, 0, 2); cmpx(v, 1, 3); cmpx(v, 4, 6); cmpx(v, 5, 7);
                        cmpx(v, 1, 2); cmpx(v, 5, 6);
                        cmpx(v, 0, 4); cmpx(v, 1, 5); cmpx(v, 2, 6); cmpx(v, 3, 7);
                        cmpx(v, 2, 4); cmpx(v, 3, 5);
                        cmpx(v, 1, 2); cmpx(v, 3, 4); cmpx(v, 5, 6);
#pragma unroll
                        for (int t = 0; t < 8; ++t)
                            if (t < n[h]) cb[s0[h] + t] = v[t];
                    }
                } else {
#pragma unroll
                    for (int h = 0; h < 2; ++h) {
                        int v[16];
#pragma unroll
                        for (int t = 0; t < 16; ++t) v[t] = t < n[h] ? src[h][t] : 0x7fffffff;
                        cmpx(v, 0, 1); cmpx(v, 2, 3); cmpx(v, 0, 2); cmpx(v, 1, 3); cmpx(v, 1, 2);
                        cmpx(v, 4, 5); cmpx(v, 6, 7); cmpx(v, 4, 6); cmpx(v, 5, 7); cmpx(v, 5, 6);
                        cmpx(v, 0, 4); cmpx(v, 2, 6); cmpx(v, 2, 4); cmpx(v, 1, 5); cmpx(v, 3, 7);
                        cmpx(v, 3, 5); cmpx(v, 1, 2); cmpx(v, 3, 4); cmpx(v, 5, 6); cmpx(v, 8, 9);
                        cmpx(v, 10, 11); cmpx(v, 8, 10); cmpx(v, 9, 11); cmpx(v, 9, 10); cmpx(v, 12, 13);
                        cmpx(v, 14, 15); cmpx(v, 12, 14); cmpx(v, 13, 15); cmpx(v, 13, 14); cmpx(v, 8, 12);
                        cmpx(v, 10, 14); cmpx(v, 10, 12); cmpx(v, 9, 13); cmpx(v, 11, 15); cmpx(v, 11, 13);
                        cmpx(v, 9, 10); cmpx(v, 11, 12); cmpx(v, 13, 14); cmpx(v, 0, 8); cmpx(v, 4, 12);
                        cmpx(v, 4, 8); cmpx(v, 2, 10); cmpx(v, 6, 14); cmpx(v, 6, 10); cmpx(v, 2, 4);
                        cmpx(v, 6, 8); cmpx(v, 10, 12); cmpx(v, 1, 9); cmpx(v, 5, 13); cmpx(v, 5, 9);
                        cmpx(v, 3, 11); cmpx(v, 7, 15); cmpx(v, 7, 11); cmpx(v, 3, 5); cmpx(v, 7, 9);
                        cmpx(v, 11, 13); cmpx(v, 1, 2); cmpx(v, 3, 4); cmpx(v, 5, 6); cmpx(v, 7, 8);
                        cmpx(v, 9, 10); cmpx(v, 11, 12); cmpx(v, 13, 14);
#pragma unroll
                        for (int t = 0; t < 16; ++t)
                            if (t < n[h]) cb[s0[h] + t] = v[t];
                        if (n[h] > 16) {   // the rest in, then an insertion sort of the whole cell
                            for (int t = 16; t < n[h]; ++t) cb[s0[h] + t] = src[h][t];
                            for (int t = 1; t < n[h]; ++t) {
                                const int x = cb[s0[h] + t];
                                int u = t;
                                while (u > 0 && cb[s0[h] + u - 1] > x) {
                                    cb[s0[h] + u] = cb[s0[h] + u - 1];
                                    --u;
                                }
                                cb[s0[h] + u] = x;
                            }
                        }
                    }
                }
                __builtin_amdgcn_wave_barrier();
                for (int k0 = 0; k0 < end; k0 += 64 * U) {
                    int jl[U];
                    uint4 qj[U];
#pragma unroll
                    for (int u = 0; u < U; ++u) {
                        const int k = k0 + 64 * u + lw;
                        jl[u] = k < end ? cb[k] : -1;
                    }
#pragma unroll
                    for (int u = 0; u < U; ++u) qj[u] = a.Q[roff + (jl[u] < 0 ? il : jl[u])];
#pragma unroll
                    for (int u = 0; u < U; ++u) {
                        const float dx = (float)(int)(qi.x - qj[u].x) * sx, dy = (float)(int)(qi.y - qj[u].y) * sy,
                                    dz = (float)(int)(qi.z - qj[u].z) * sz;
                        const bool acc = jl[u] >= 0 && jl[u] != il && dx * dx + dy * dy + dz * dz < rl2;
                        append(acc, roff + jl[u]);
                    }
                }
                __builtin_amdgcn_wave_barrier();   // the chunk is refilled next
                base = cend[w][q1 - 1];
                q0 = q1;
            }
        }
        // pad the last slab with the atom itself (cap is a multiple of 32), then
        // write the row as whole slabs
        const int used = cnt < cap ? cnt : cap;
        const int pad_end = min((used + 3) & ~3, cap);
        if (used + lw < pad_end) row[used + lw] = i;
        __builtin_amdgcn_wave_barrier();
        for (int b = lw; 4 * b < pad_end; b += 64)
            *(int4*)(a.nbr + ((size_t)b * (size_t)N + (size_t)i) * 4) =
                make_int4(row[4 * b], row[4 * b + 1], row[4 * b + 2], row[4 * b + 3]);
        if (lw == 0) {
            if (cnt > cap) {
                atomicOr(a.status, ST_NEIGH_OVERFLOW);
                cnt = cap;
            }
            a.nnb[i] = cnt;
            a.xref[i] = pi.x;
            a.xref[N + i] = pi.y;
            a.xref[2 * N + i] = pi.z;
        }
        __builtin_amdgcn_wave_barrier();   // the row buffer is reused by the next atom
    }
}

// --------------------------------------------------------------------------
// Rows of replicas small enough for one block's LDS (k_rows_lds).  The grid
// is one block per CU; every block reads the rebuild flags of
// these replicas, splits the flagged ones into `parts` slices of atoms so
// that the items fill the grid, and takes items in a fixed stride.  For its
// item a block stages the replica's records in LDS, sorts its atoms into
// the cells of the global builder (counting sort by cell, then each cell's
// members by id) and builds the rows of the item's atoms from LDS alone: the
// same candidate stream (stencil cells by offset, members by id) and the
// same test as k_list, so the rows are identical to that builder's.
// LDS: records [atoms], sorted ids [atoms] (16 bit), cell starts [cells + 1],
// then per wavefront a row buffer [cap], the stencil's inclusive ends and
// starts [2][128] and a candidate chunk [kRowsChunk] (16 bit).
// --------------------------------------------------------------------------

__global__ __launch_bounds__(1024) void k_rows_lds(NeighArgs a, StepArgs s)
{
    extern __shared__ uint4 lds_rows[];
    const int lw = threadIdx.x & 63, w = threadIdx.x >> 6, nw = blockDim.x >> 6;
    uint4* st = lds_rows;
    uint16_t* ids = (uint16_t*)(st + a.lds_atoms);
    int* cst = (int*)((char*)ids + (((size_t)a.lds_atoms * 2 + 15) & ~(size_t)15));
    int* row = (int*)((char*)cst + (((size_t)(a.lds_cells + 1) * 4 + 15) & ~(size_t)15) +
                      (size_t)w * rows_lds_wave_bytes(a.cap));
    __shared__ int sh_nf, sh_atoms, sh_items, sh_rep, sh_part, sh_parts, sh_roff, sh_rn;
    __shared__ int wsum[16];
    // the builder's k-th replica: the list holds them in replica order, so
    // when it holds every replica it is the identity, and the flag and size
    // reads need not wait for it
    const bool all = a.n_lds == a.n_rep;
    auto lds_rep = [&](int k) { return all ? k : a.lds_list[k]; };
    const int G = gridDim.x;
    // items: each flagged replica cut into parts in proportion to its atoms,
    // about G items in all, numbered replica by replica.  Wave 0 finds the
    // replica, part, first atom and size of item `it` (sh_*); atoms_f: the
    // flagged replicas' atoms.  Returns the number of items.
    auto select = [&](int it, int atoms_f) {
        int seen = 0;
        bool found = false;
        for (int k0 = 0; k0 < a.n_lds; k0 += 64) {
            const int k = k0 + lw;
            const int r = k < a.n_lds ? lds_rep(k) : 0;
            const bool f = k < a.n_lds && a.rebuild[r] != 0;
            const int2 on = f ? *(const int2*)&a.reps[r].off : make_int2(0, 0);   // first atom, atoms
            const int pr = f ? max(1, (int)(((long long)on.y * G) / atoms_f)) : 0;
            int incl = wave_scan(pr);
            const int chunk_total = __builtin_amdgcn_readlane(incl, 63);
            if (!found && it < seen + chunk_total) {   // uniform: the lane whose parts hold it
                const bool mine = pr > 0 && it >= seen + incl - pr && it < seen + incl;
                const int src = (int)__ffsll((long long)__ballot(mine)) - 1;
                const int rsel = __shfl(r, src, 64);
                const int first = __shfl(seen + incl - pr, src, 64);
                const int psel = __shfl(pr, src, 64);
                const int osel = __shfl(on.x, src, 64), nsel = __shfl(on.y, src, 64);
                if (lw == 0) {
                    sh_rep = rsel;
                    sh_part = it - first;
                    sh_parts = psel;
                    sh_roff = osel;
                    sh_rn = nsel;
                }
                found = true;
            }
            seen += chunk_total;
        }
        return seen;
    };

    // flagged replicas of this builder (their number and atoms) and this
    // block's first item, behind one barrier
    if (w == 0) {
        int nf = 0, at = 0;
        for (int k0 = 0; k0 < a.n_lds; k0 += 64) {
            const int k = k0 + lw;
            const int r = k < a.n_lds ? lds_rep(k) : 0;
            const bool f = k < a.n_lds && a.rebuild[r] != 0;
            nf += __popcll(__ballot(f));
            int n = f ? a.reps[r].n : 0;
#pragma unroll
            for (int o = 32; o > 0; o >>= 1) n += __shfl_xor(n, o, 64);
            at += n;
        }
        const int items = nf > 0 ? select(blockIdx.x, at) : 0;
        if (lw == 0) {
            sh_nf = nf;
            sh_atoms = at;
            sh_items = items;
        }
    }
    __syncthreads();
    const int nf = sh_nf, atoms_f = sh_atoms, items = sh_items;
    if (nf == 0) return;   // (the history below would add zeros)
    if (blockIdx.x == 0 && threadIdx.x == 0 && s.step_kernel) {   // rebuild history of the step passes
        s.row_acc[a.n_rep + 1] += (double)nf;
        s.row_acc[a.n_rep + 2] += (double)atoms_f;
    }
    const uint64_t below = (1ull << lw) - 1ull;
    const float rl2 = a.rl2_f;
    for (int it = blockIdx.x; it < items; it += G) {
        if (it != (int)blockIdx.x) {   // a later item of this block (the first one is selected above)
            if (w == 0) select(it, atoms_f);
            __syncthreads();
        }
        const int rr = sh_rep, part = sh_part, parts = sh_parts, roff = sh_roff, rn = sh_rn;
        const RepDesc& R = a.reps[rr];
        // the cell counts and box go out with the record copy's loads
        const int nc0 = R.nc[0], nc1 = R.nc[1], nc2 = R.nc[2];
        const float sx = (float)(R.L[0] * 2.3283064365386963e-10), sy = (float)(R.L[1] * 2.3283064365386963e-10),
                    sz = (float)(R.L[2] * 2.3283064365386963e-10);
        copy_rounds<4, uint4>(rn, [&](int k) { return a.Q[roff + k]; }, [&](int k, const uint4& q) { st[k] = q; });
        const int ncell = nc0 * nc1 * nc2;
        if (nc0 > 0)
            for (int c = threadIdx.x; c <= ncell; c += blockDim.x) cst[c] = 0;
        __syncthreads();
        auto cell_of = [&](const uint4& q) {
            return (box_cell(q.x, nc0) * nc1 + box_cell(q.y, nc1)) * nc2 + box_cell(q.z, nc2);
        };
        if (nc0 > 0) {
            for (int k = threadIdx.x; k < rn; k += blockDim.x) atomicAdd(&cst[cell_of(st[k])], 1);
            __syncthreads();
            // inclusive scan of the counts over the cells: contiguous segments
            // per thread, then the segment totals across the block
            {
                const int per = (ncell + (int)blockDim.x - 1) / (int)blockDim.x;
                const int c0 = threadIdx.x * per, c1 = min(ncell, c0 + per);
                int tot = 0;
                for (int c = c0; c < c1; ++c) tot += cst[c];
                int incl = wave_scan(tot);
                if (lw == 63) wsum[w] = incl;
                __syncthreads();
                int before = incl - tot;
                for (int q = 0; q < w; ++q) before += wsum[q];
                for (int c = c0; c < c1; ++c) {
                    before += cst[c];
                    cst[c] = before;
                }
                __syncthreads();
            }
            if (threadIdx.x == 0) cst[ncell] = rn;
            // scatter: each cell's end pointer walks down to its start
            for (int k = threadIdx.x; k < rn; k += blockDim.x) {
                const int pos = atomicSub(&cst[cell_of(st[k])], 1) - 1;
                ids[pos] = (uint16_t)k;
            }
            __syncthreads();
            // each cell's members in id order: up to eight in registers through
            // a sorting network (Batcher's odd-even merge; their reads in flight
            // together), an insertion sort in LDS beyond
            for (int c = threadIdx.x; c < ncell; c += blockDim.x) {
                const int b = cst[c], e = cst[c + 1], m = e - b;
                if (m <= 1) continue;
                if (m <= 8) {
                    int v[8];
#pragma unroll
                    for (int t = 0; t < 8; ++t) v[t] = t < m ? (int)ids[b + t] : 0xffff;
                    auto cmpx = [&](int p, int q) {
                        const int lo = min(v[p], v[q]), hi = max(v[p], v[q]);
                        v[p] = lo;
                        v[q] = hi;
                    };
                    cmpx(0, 1); cmpx(2, 3); cmpx(4, 5); cmpx(6, 7);
                    cmpx(0, 2); cmpx(1, 3); cmpx(4, 6); cmpx(5, 7);
                    cmpx(1, 2); cmpx(5, 6);
                    cmpx(0, 4); cmpx(1, 5); cmpx(2, 6); cmpx(3, 7);
                    cmpx(2, 4); cmpx(3, 5);
                    cmpx(1, 2); cmpx(3, 4); cmpx(5, 6);
#pragma unroll
                    for (int t = 0; t < 8; ++t)
                        if (t < m) ids[b + t] = (uint16_t)v[t];
                } else {
                    for (int t = b + 1; t < e; ++t) {
                        const uint16_t x = ids[t];
                        int u = t;
                        while (u > b && ids[u - 1] > x) {
                            ids[u] = ids[u - 1];
                            --u;
                        }
                        ids[u] = x;
                    }
                }
            }
        }
        __syncthreads();
        // rows of this item's atoms, one wavefront per atom
        const int a0 = (int)((long long)rn * part / parts), a1 = (int)((long long)rn * (part + 1) / parts);
        for (int il = a0 + w; il < a1; il += nw) {
            const int i = roff + il;
            const uint4 qi = st[il];
            const double4 pi = a.P[i];   // the list's reference position, read ahead of the row work
            auto close_to = [&](const uint4& qj) {
                const float dx = (float)(int)(qi.x - qj.x) * sx, dy = (float)(int)(qi.y - qj.y) * sy,
                            dz = (float)(int)(qi.z - qj.z) * sz;
                return dx * dx + dy * dy + dz * dz < rl2;
            };
            int cnt = 0;
            if (nc0 == 0) {   // all-pairs rows: every other atom in id order
                for (int s0 = 0; s0 < rn; s0 += 64) {
                    const int jl = s0 + lw;
                    const bool acc = jl < rn && jl != il && close_to(st[jl < rn ? jl : il]);
                    const uint64_t m = __ballot(acc);
                    const int rank = __popcll(m & below);
                    if (acc && cnt + rank < a.cap) row[cnt + rank] = roff + jl;
                    cnt += __popcll(m);
                }
            } else {
                // lane l tests stencil cells l and 64 + l (cells by offset, the
                // 125 of a 5 x 5 x 5 block), keeping a mask of its members in
                // range; a prefix sum of the accepted counts over the cells then
                // gives every accepted member its slot, so the row is the stream
                // of cells in offset order, members in id order.  Five or more
                // cells per edge: an offset of -2..2 wraps at most once.
                const int cx = box_cell(qi.x, nc0), cy = box_cell(qi.y, nc1), cz = box_cell(qi.z, nc2);
                int cb[2], cn[2];
                uint64_t mask[2];
#pragma unroll
                for (int h = 0; h < 2; ++h) {
                    const int q = 64 * h + lw;
                    cb[h] = 0;
                    cn[h] = 0;
                    mask[h] = 0ull;
                    if (q < kStencil) {
                        const int ux = wrap_cell(cx + q / 25 - 2, nc0);
                        const int uy = wrap_cell(cy + (q / 5) % 5 - 2, nc1);
                        const int uz = wrap_cell(cz + q % 5 - 2, nc2);
                        const int c = (ux * nc1 + uy) * nc2 + uz;
                        cb[h] = cst[c];
                        cn[h] = cst[c + 1] - cb[h];
                        if (cn[h] > 64) {   // a mask holds 64 members (only overlapping atoms crowd a cell so)
                            atomicOr(a.status, ST_CELL_OVERFLOW);
                            cn[h] = 64;
                        }
                    }
                }
                // both cells' members four at a time: their id and record reads
                // in flight together
                for (int t0 = 0; t0 < max(cn[0], cn[1]); t0 += 4) {
                    int jl[2][4];
                    uint4 qj[2][4];
#pragma unroll
                    for (int h = 0; h < 2; ++h)
#pragma unroll
                        for (int u = 0; u < 4; ++u) jl[h][u] = t0 + u < cn[h] ? (int)ids[cb[h] + t0 + u] : il;
#pragma unroll
                    for (int h = 0; h < 2; ++h)
#pragma unroll
                        for (int u = 0; u < 4; ++u) qj[h][u] = st[jl[h][u]];
#pragma unroll
                    for (int h = 0; h < 2; ++h)
#pragma unroll
                        for (int u = 0; u < 4; ++u)
                            if (jl[h][u] != il && close_to(qj[h][u])) mask[h] |= 1ull << (t0 + u);
                }
                int base = 0;
#pragma unroll
                for (int h = 0; h < 2; ++h) {
                    const int n_acc = __popcll(mask[h]);
                    int incl = wave_scan(n_acc);
                    int slot = base + incl - n_acc;
                    if (cn[h] <= 8) {   // the first eight members: reads in flight together
                        int id8[8];
#pragma unroll
                        for (int t = 0; t < 8; ++t) id8[t] = (int)ids[cb[h] + min(t, max(cn[h] - 1, 0))];
#pragma unroll
                        for (int t = 0; t < 8; ++t)
                            if ((mask[h] >> t) & 1ull) {
                                if (slot < a.cap) row[slot] = roff + id8[t];
                                ++slot;
                            }
                    } else {
                        for (uint64_t m = mask[h]; m; m &= m - 1ull) {
                            const int t = (int)__ffsll((long long)m) - 1;
                            if (slot < a.cap) row[slot] = roff + (int)ids[cb[h] + t];
                            ++slot;
                        }
                    }
                    base += __builtin_amdgcn_readlane(incl, 63);
                }
                cnt = base;
            }
            __builtin_amdgcn_wave_barrier();
            // pad the last slab with the atom itself (cap is a multiple of 32), then
            // write the row as whole slabs
            const int used = cnt < a.cap ? cnt : a.cap;
            const int pad_end = min((used + 3) & ~3, a.cap);
            if (used + lw < pad_end) row[used + lw] = i;
            __builtin_amdgcn_wave_barrier();
            for (int b = lw; 4 * b < pad_end; b += 64)
                *(int4*)(a.nbr + ((size_t)b * (size_t)a.N + (size_t)i) * 4) =
                    make_int4(row[4 * b], row[4 * b + 1], row[4 * b + 2], row[4 * b + 3]);
            if (lw == 0) {
                if (cnt > a.cap) {
                    atomicOr(a.status, ST_NEIGH_OVERFLOW);
                    cnt = a.cap;
                }
                a.nnb[i] = cnt;
                a.xref[i] = pi.x;
                a.xref[a.N + i] = pi.y;
                a.xref[2 * a.N + i] = pi.z;
            }
            __builtin_amdgcn_wave_barrier();   // the row buffer is reused by the next atom
        }
        if (it + G < items) __syncthreads();   // the staged replica is replaced by the next item's
    }
}

// --------------------------------------------------------------------------
// Density pass.  FP32 tables are staged in LDS (32 KB for rho).
// --------------------------------------------------------------------------
template <typename real, int T, bool kStage = false, bool kFix = true, bool kLds = (sizeof(real) == 4)>
__global__ __launch_bounds__(kMaxBlock) void k_density(StepArgs a)
{
    extern __shared__ float4 lds_tab[];
    constexpr bool kQ = sizeof(real) == 4;   // FP32 form gathers 16-byte box-coordinate records
    const int N = a.N;
    const int64_t it = a.step_kernel ? *a.iter + a.it_k : 0;
    if (a.finish_prev && blockIdx.x == gridDim.x - 1) {   // the extra block: finish the force pass of step it - 1
        finish_body(a, it - 1);
        return;
    }
    const int nr = a.tab.n_r;
    // kLds: the table in LDS once per block; its wavefronts then take units
    // (FP32 always; FP64 when its 32-byte intervals fit, copied as they are)
    auto stage_table = [&]() {
        if constexpr (kLds && kQ) {
            const float4* g = (const float4*)a.tab.rho;
            copy_rounds<2, float4>(nr - 1, [&](int k) { return g[k]; }, [&](int k, const float4& c) { lds_tab[k] = c; });
            if (threadIdx.x == 0) {   // padding interval: the value at r_cut
                const float4 c = g[nr - 2];
                lds_tab[nr - 1] = make_float4(c.x + c.y + c.z + c.w, 0.f, 0.f, 0.f);
            }
        } else if constexpr (kLds) {
            const uint4* g = (const uint4*)a.tab.rho;
            uint4* l = (uint4*)lds_tab;
            copy_rounds<4, uint4>(2 * (nr - 1), [&](int k) { return g[k]; }, [&](int k, const uint4& c) { l[k] = c; });
        }
    };
    uint4* const st = (uint4*)(lds_tab + nr);   // staged form: the block's replica records, after the table
    auto unit = [&](const Tile& tl) {
    const RepDesc& R = a.reps[tl.rep];
    const int lane = wave_lane() % T;
    const int la = wave_lane() / T;
    const bool valid = la < tl.count;
    const int i = tl.first + (valid ? la : 0);

    double acc = 0.0;
    const double4 pi = a.P[i];
    const uint4 qi = kQ ? a.Q[i] : make_uint4(0u, 0u, 0u, 0u);
    const float qsx = (float)(R.L[0] * 2.3283064365386963e-10), qsy = (float)(R.L[1] * 2.3283064365386963e-10),
                qsz = (float)(R.L[2] * 2.3283064365386963e-10);
    if (valid && a.has_eam) {
        const int n = a.nnb[i];
        const real rc2 = (real)a.tab.rc2, inv_h = (real)a.tab.inv_h_r;
        const uint32_t rc2m1 = __float_as_uint((float)a.tab.rc2) - 1u;   // FP32 form's cutoff test
        walk_row<kQ, T>(a.nbr, a.P, kStage ? st : a.Q, kStage ? R.off : 0, N, i, lane, n,
                        [&](const Nb<kQ>& g, int b0) {
            real r[SB], t[SB];
            int m[SB];
            bool in[SB];
#pragma unroll
            for (int s = 0; s < SB; ++s) {
                real rx, ry, rz;
                if constexpr (kQ) {
                    rx = (real)(int)(qi.x - g.v[s].x) * qsx;
                    ry = (real)(int)(qi.y - g.v[s].y) * qsy;
                    rz = (real)(int)(qi.z - g.v[s].z) * qsz;
                } else {
                    const double3 d = sep(R, pi, g.v[s]);
                    rx = (real)d.x;
                    ry = (real)d.y;
                    rz = (real)d.z;
                }
                const real r2 = rx * rx + ry * ry + rz * rz;
                real ir;
                if constexpr (kQ) {
                    // 0 < r^2 < rc^2 in one unsigned compare of the bits; the
                    // self-padded slots of a row's last slab give r^2 = 0
                    in[s] = __float_as_uint(r2) - 1u < rc2m1;
                    Root<real>::of(in[s] ? r2 : (real)1, r[s], ir);
                    m[s] = interval_pad(r[s], inv_h, t[s]);
                } else {
                    in[s] = (b0 + s < n) && r2 < rc2;
                    Root<real>::of(r2, r[s], ir);
                    m[s] = interval<real>(in[s] ? r[s] : (real)0, inv_h, nr, t[s]);
                }
            }
            real part = (real)0;
#pragma unroll
            for (int s = 0; s < SB; ++s) {
                real v;
                if constexpr (kLds && kQ) {
                    const float4 c = lds_tab[m[s]];
                    v = c.x + t[s] * (c.y + t[s] * (c.z + t[s] * c.w));
                } else {
                    const auto c = Tab<real>::ld4(kLds ? (const void*)lds_tab : a.tab.rho, m[s]);
                    v = c.x + t[s] * (c.y + t[s] * (c.z + t[s] * c.w));
                }
                if constexpr (kQ) part += v * (in[s] ? 1.f : 0.f);   // a product: the table read stays unconditional
                else part += in[s] ? v : (real)0;
            }
            acc += Acc<real, kFix>::q(part);
        });
    }
#pragma unroll
    for (int o = T / 2; o > 0; o >>= 1) acc += xor_lanes(acc, o);   // (o < T: the partner is in the atom's lanes)
    // one memory round trip for the epilogue: the embedding table's interval
    // and what the epilogue needs of the replica go out together, ahead of
    // the unit's stores (after a store every descriptor read would be a round
    // trip of its own)
    const bool emb = valid && lane == 0 && a.has_eam;
    double rho = 0.0;
    real tF = (real)0;
    decltype(Tab<real>::ld4(a.tab.F, 0)) cF{};
    if (emb) {
        rho = Acc<real, kFix>::fin(acc);
        const int m = interval<real>((real)rho, (real)a.tab.inv_h_rho, a.tab.n_rho, tF);
        cF = Tab<real>::ld4(a.tab.F, m);
    }
    const uint64_t seed_raw = R.seed;
    const int roff_raw = R.off, tbase_raw = R.tile_base, ntile_raw = R.n_tiles, cbase_raw = R.cell_base;
    // a replica rebuilt in this step: the list pass has read its cell
    // counters, which the unit clears for its next binning (every operand
    // read at once, no chain of conditional reads)
    const int nc0 = R.nc[0], nc1 = R.nc[1], nc2 = R.nc[2], rlds = R.lds;
    const int fp0 = a.flag_pre[tl.rep], fp1 = a.flag_pre[tl.rep + 1];
    const uint64_t seed = ((uint64_t)__builtin_amdgcn_readfirstlane((uint32_t)(seed_raw >> 32)) << 32) |
                          (uint64_t)__builtin_amdgcn_readfirstlane((uint32_t)seed_raw);
    const int roff = __builtin_amdgcn_readfirstlane(roff_raw);
    const int tbase = __builtin_amdgcn_readfirstlane(tbase_raw);
    const int ntile = __builtin_amdgcn_readfirstlane(ntile_raw);
    const int cbase = __builtin_amdgcn_readfirstlane(cbase_raw);
    const bool clear = (a.cell_cnt != nullptr) & (nc0 > 0) & (rlds == 0) & (fp1 > fp0);
    const int ncell_clear = __builtin_amdgcn_readfirstlane(clear ? nc0 * nc1 * nc2 : 0);

    // thermostat noise of step `it` and (fixed centre of mass) its replica sum.
    // In the exact-sum form the deviates themselves go on the 2^-36 grid, so
    // the mean the step removes is the exact mean of the values it applies
    // (a lone atom stays put bit for bit)
    if (a.step_kernel && it < a.it_last) {
        constexpr bool kGrid = sizeof(real) == 4 && kFix;
        double z[3] = {0.0, 0.0, 0.0};
        if constexpr (T == 1) {
            if (valid) {
                gauss3(seed, (uint32_t)(i - roff), it, 0u, z[0], z[1], z[2]);
                if (kGrid && a.fix_com) on_grid<3>(z, kGridZ, kGridZInv);
                a.xi[i] = z[0];
                a.xi[N + i] = z[1];
                a.xi[2 * N + i] = z[2];
            }
        } else if (valid && lane < 2) {   // lane 0: x and y components, lane 1: z
            double za, zb;
            gauss3_half(seed, (uint32_t)(i - roff), it, 0u, lane, za, zb);
            if (kGrid && a.fix_com) {
                za = rint(za * kGridZ) * kGridZInv;
                zb = rint(zb * kGridZ) * kGridZInv;
            }
            if (lane == 0) {
                z[0] = za;
                z[1] = zb;
                a.xi[i] = za;
                a.xi[N + i] = zb;
            } else {
                z[2] = za;
                a.xi[2 * N + i] = za;
            }
        }
        if (a.fix_com) unit_partial<3>(z, a.noise_part, tbase, tl.idx);
    }
    if (emb) {
        const auto& c = cF;
        const real t = tF;
        const real F = c.x + t * (c.y + t * (c.z + t * c.w));
        const real Fp = (c.y + t * ((real)2 * c.z + (real)3 * t * c.w)) * (real)a.tab.inv_h_rho;
        if constexpr (kQ) a.Q[i].w = __float_as_uint((float)Fp);
        else a.P[i].w = (double)Fp;
        a.e_emb[i] = (double)F;
        if (a.rho_out) a.rho_out[i] = rho;
        if (rho > a.tab.rho_max) atomicOr(a.status, ST_TABLE_RANGE);
        if (!isfinite(rho)) atomicOr(a.status, ST_NONFINITE);
    }
    if (tl.idx == 0 && wave_lane() == 0) a.rebuild[tl.rep] = 0;   // lists are current now
    for (int c = tl.idx * 64 + wave_lane(); c < ncell_clear; c += ntile * 64) a.cell_cnt[cbase + c] = 0;
    };   // unit
    run_units<kStage>(a, st, stage_table, unit);
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

template <typename real, int T, bool kStage = false, bool kVir = false, bool kFix = true,
          bool kLds = (sizeof(real) == 4)>
__global__ __launch_bounds__(kMaxBlock) void k_force(StepArgs a)
{
    extern __shared__ float4 lds_tab[];
    constexpr bool kQ = sizeof(real) == 4;   // FP32 form gathers 16-byte box-coordinate records
    const int N = a.N;
    const int64_t it = a.step_kernel ? *a.iter + a.it_k : 0;
    const int nr = a.tab.n_r;
    // kLds: the table in LDS once per block; its wavefronts then take units.
    // FP32: the two 16-byte halves of an interval's record (phi's
    // coefficients, rho's slope coefficients) sit in two arrays of nr entries,
    // so the random reads of each half spread over every bank, not over the
    // even or the odd 16-byte bank groups only.  FP64 (when its 64-byte
    // intervals fit): the table as it is in global memory.
    auto stage_table = [&]() {
        if constexpr (kLds && kQ) {
            const float4* g = (const float4*)a.tab.pair;
            // the two halves as 2 (nr - 1) items: item k is half k % 2 of interval k / 2
            copy_rounds<4, float4>(2 * (nr - 1), [&](int k) { return g[k]; },
                                   [&](int k, const float4& c) { lds_tab[(k & 1) * nr + (k >> 1)] = c; });
            if (threadIdx.x == 0) {   // padding interval: phi(r_cut), zero slopes
                const float4 c = g[2 * (nr - 2)];
                lds_tab[nr - 1] = make_float4(c.x + c.y + c.z + c.w, 0.f, 0.f, 0.f);
                lds_tab[2 * nr - 1] = make_float4(0.f, 0.f, 0.f, 0.f);
            }
        } else if constexpr (kLds) {
            const uint4* g = (const uint4*)a.tab.pair;
            uint4* l = (uint4*)lds_tab;
            copy_rounds<4, uint4>(4 * (nr - 1), [&](int k) { return g[k]; }, [&](int k, const uint4& c) { l[k] = c; });
        }
    };
    // this step's lambda values, read once per block
    const double lam_it = a.step_kernel ? a.lam[it] : 0.0;
    const double lam_next = a.step_kernel && it < a.it_last ? a.lam[it + 1] : 0.0;
    uint4* const st = (uint4*)(lds_tab + 2 * nr);   // staged form: the block's replica records, after the table
    auto unit = [&](const Tile& tl) {
    const RepDesc& R = a.reps[tl.rep];
    const int lane = wave_lane() % T;
    const int la = wave_lane() / T;
    const bool valid = la < tl.count;
    const int i = tl.first + (valid ? la : 0);

    const double4 pi = a.P[i];
    const uint4 qi = kQ ? a.Q[i] : make_uint4(0u, 0u, 0u, 0u);
    const int nrow = a.has_eam ? a.nnb[i] : 0;   // row length: the walk, then the list work of the pass
    // the replica's unit slots, held in scalar registers across the walk so
    // that the noise partials' loads need no descriptor read after it
    const int tbase = __builtin_amdgcn_readfirstlane(R.tile_base);
    const int ntile = __builtin_amdgcn_readfirstlane(R.n_tiles);
    const float qsx = (float)(R.L[0] * 2.3283064365386963e-10), qsy = (float)(R.L[1] * 2.3283064365386963e-10),
                qsz = (float)(R.L[2] * 2.3283064365386963e-10);
    double f0 = 0.0, f1 = 0.0, f2 = 0.0, ep = 0.0;
    double w0 = 0.0, w1 = 0.0, w2 = 0.0;   // virial (kVir): sum_j (x_i - x_j)_a f_ij,a per axis
    if (valid && a.has_eam) {
        const int n = nrow;
        const real Fpi = kQ ? (real)__uint_as_float(qi.w) : (real)pi.w;
        const real rc2 = (real)a.tab.rc2, inv_h = (real)a.tab.inv_h_r;
        const uint32_t rc2m1 = __float_as_uint((float)a.tab.rc2) - 1u;   // FP32 form's cutoff test
        walk_row<kQ, T>(a.nbr, a.P, kStage ? st : a.Q, kStage ? R.off : 0, N, i, lane, n,
                        [&](const Nb<kQ>& g, int b0) {
            real rx[SB], ry[SB], rz[SB], ir[SB], t[SB], fpj[SB];
            int m[SB];
            bool in[SB];
#pragma unroll
            for (int s = 0; s < SB; ++s) {
                if constexpr (kQ) {
                    rx[s] = (real)(int)(qi.x - g.v[s].x) * qsx;
                    ry[s] = (real)(int)(qi.y - g.v[s].y) * qsy;
                    rz[s] = (real)(int)(qi.z - g.v[s].z) * qsz;
                    fpj[s] = (real)__uint_as_float(g.v[s].w);
                } else {
                    const double3 d = sep(R, pi, g.v[s]);
                    rx[s] = (real)d.x;
                    ry[s] = (real)d.y;
                    rz[s] = (real)d.z;
                    fpj[s] = (real)g.v[s].w;
                }
                const real r2 = rx[s] * rx[s] + ry[s] * ry[s] + rz[s] * rz[s];
                real r;
                if constexpr (kQ) {
                    in[s] = __float_as_uint(r2) - 1u < rc2m1;   // 0 < r^2 < rc^2, as in the density pass
                    Root<real>::of(in[s] ? r2 : (real)1, r, ir[s]);
                    m[s] = interval_pad(r, inv_h, t[s]);
                } else {
                    in[s] = (b0 + s < n) && r2 < rc2;
                    Root<real>::of(in[s] ? r2 : (real)1, r, ir[s]);
                    m[s] = interval<real>(in[s] ? r : (real)0, inv_h, nr, t[s]);
                }
            }
            real p0 = (real)0, p1 = (real)0, p2 = (real)0, pe = (real)0;
            real q0 = (real)0, q1 = (real)0, q2 = (real)0;
#pragma unroll
            for (int s = 0; s < SB; ++s) {
                real ua, ub, uc, ud, wb, wc, wd;
                if constexpr (kLds && kQ) {
                    const float4 u = lds_tab[m[s]], w = lds_tab[nr + m[s]];
                    ua = u.x; ub = u.y; uc = u.z; ud = u.w; wb = w.x; wc = w.y; wd = w.z;
                } else {
                    decltype(Tab<real>::ld4(a.tab.rho, 0)) u, w;
                    Tab<real>::ld8(kLds ? (const void*)lds_tab : a.tab.pair, m[s], u, w);
                    ua = u.x; ub = u.y; uc = u.z; ud = u.w; wb = w.x; wc = w.y; wd = w.z;
                }
                const real ts = t[s];
                if constexpr (kQ) {
                    // phi and h dphi/dr = b + 2 c t + 3 d t^2 share their Horner
                    // terms; pairs outside the cutoff are weighted by zero (a
                    // product, not a select, so every table read stays one 16-byte load)
                    const float cu = uc + ts * ud, cv = ub + ts * cu;
                    const float phi = ua + ts * cv;
                    const float dphi_h = cv + ts * (cu + ts * ud);
                    const float drho = wb + ts * (wc + ts * wd);
                    const float fm = in[s] ? 1.f : 0.f;
                    const float g = dphi_h * inv_h + (Fpi + fpj[s]) * drho;   // dU/dr_ij
                    const float sc = -g * (ir[s] * fm);
                    p0 += sc * rx[s];
                    p1 += sc * ry[s];
                    p2 += sc * rz[s];
                    pe += phi * fm;
                    if constexpr (kVir) {
                        q0 += sc * rx[s] * rx[s];
                        q1 += sc * ry[s] * ry[s];
                        q2 += sc * rz[s] * rz[s];
                    }
                } else {
                    const real phi = ua + ts * (ub + ts * (uc + ts * ud));
                    const real dphi = (ub + ts * ((real)2 * uc + (real)3 * ts * ud)) * inv_h;
                    const real drho = wb + ts * (wc + ts * wd);
                    const real g = dphi + (Fpi + fpj[s]) * drho;   // dU/dr_ij
                    const real sc = in[s] ? -g * ir[s] : (real)0;
                    p0 += sc * rx[s];
                    p1 += sc * ry[s];
                    p2 += sc * rz[s];
                    pe += in[s] ? phi : (real)0;
                    if constexpr (kVir) {
                        q0 += sc * rx[s] * rx[s];
                        q1 += sc * ry[s] * ry[s];
                        q2 += sc * rz[s] * rz[s];
                    }
                }
            }
            f0 += Acc<real, kFix>::q(p0);
            f1 += Acc<real, kFix>::q(p1);
            f2 += Acc<real, kFix>::q(p2);
            ep += Acc<real, kFix>::q(pe);
            if constexpr (kVir) {
                w0 += Acc<real, kFix>::q(q0);
                w1 += Acc<real, kFix>::q(q1);
                w2 += Acc<real, kFix>::q(q2);
            }
        });
    }
#pragma unroll
    for (int o = T / 2; o > 0; o >>= 1) {
        f0 += xor_lanes(f0, o);   // (o < T: the partner is in the atom's lanes)
        f1 += xor_lanes(f1, o);
        f2 += xor_lanes(f2, o);
        ep += xor_lanes(ep, o);
        if constexpr (kVir) {
            w0 += xor_lanes(w0, o);
            w1 += xor_lanes(w1, o);
            w2 += xor_lanes(w2, o);
        }
    }

    // the atom's operands of the integration and the replica's noise
    // partials go out together, one memory round trip after the walk (i is in
    // range on every lane; arrays a pass does not use are stood in for by x0,
    // which every pass has, and their values are not used)
    const bool stepping = a.step_kernel != 0, opening = stepping && it < a.it_last;
    const bool noise_total = opening && a.fix_com;
    // the replica's constants of the integration (after the first store below
    // each would be a round trip of its own)
    const double r_inv_m = R.inv_m, r_k = R.k, r_k2 = R.k2, r_c2 = R.c2, r_n = (double)R.n;
    const double r_invL[3] = {R.invL[0], R.invL[1], R.invL[2]};
    const double* vsrc = stepping ? a.v : a.x0;
    const double* xisrc = opening ? a.xi : a.x0;
    const double* xrsrc = opening ? a.xref : a.x0;
    const double x0i[3] = {a.x0[i], a.x0[N + i], a.x0[2 * N + i]};
    const double ks_raw = a.kscale ? a.kscale[i] : 1.0;   // this atom's spring is k ks
    const double eemb_raw = a.has_eam ? a.e_emb[i] : 0.0;
    const double vraw[3] = {vsrc[i], vsrc[N + i], vsrc[2 * N + i]};
    const double xiraw[3] = {xisrc[i], xisrc[N + i], xisrc[2 * N + i]};
    const double xrraw[3] = {xrsrc[i], xrsrc[N + i], xrsrc[2 * N + i]};
    PartPair<3> zp;
    if (noise_total) zp = replica_loads<3>(a.noise_part, tbase, ntile);
    const double ks = ks_raw, eemb = eemb_raw;
    double vi[3] = {0.0, 0.0, 0.0}, xii[3] = {0.0, 0.0, 0.0}, xr[3] = {0.0, 0.0, 0.0};
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        vi[c] = stepping ? vraw[c] : 0.0;
        xii[c] = opening ? xiraw[c] : 0.0;
        xr[c] = opening ? xrraw[c] : 0.0;
    }

    // the replica's thermostat noise of this step, from the density pass's unit partials
    double zsum[3] = {0.0, 0.0, 0.0};
    if (noise_total) replica_finish<3>(zp, a.noise_part, tbase, ntile, zsum);

    double e[3] = {0.0, 0.0, 0.0};   // U_EAM contribution, |x - x0|^2, row length (list work of the pass)
    if (valid && lane == 0) {
        const double fe[3] = {Acc<real, kFix>::fin(f0), Acc<real, kFix>::fin(f1), Acc<real, kFix>::fin(f2)};
        double x[3] = {pi.x, pi.y, pi.z};
        // the spring displacement weighted by the atom's spring scale: the
        // spring force is -k ks (x - x0) and its energy k ks |x - x0|^2 / 2
        const double d[3] = {ks * (x[0] - x0i[0]), ks * (x[1] - x0i[1]), ks * (x[2] - x0i[2])};
        e[0] = a.has_eam ? eemb + 0.5 * Acc<real, kFix>::fin(ep) : 0.0;
        e[1] = (d[0] * (x[0] - x0i[0]) + d[1] * (x[1] - x0i[1]) + d[2] * (x[2] - x0i[2]));
        e[2] = (double)nrow;
        if (!isfinite(fe[0] + fe[1] + fe[2] + e[0] + e[1])) atomicOr(a.status, ST_NONFINITE);
        if (a.f_out) {
            a.f_out[i] = fe[0];
            a.f_out[N + i] = fe[1];
            a.f_out[2 * N + i] = fe[2];
        }
        if (a.e_atom_out) a.e_atom_out[i] = e[0];
        if (stepping) {
            const double hdt_m = 0.5 * a.dt * r_inv_m;
            double v[3] = {vi[0], vi[1], vi[2]};
            double F[3];
            if (it > a.it_first) {   // closing kick of step it-1 at lambda_it
                total_force(a.mode, fe, d, r_k, r_k2, lam_it, F);
#pragma unroll
                for (int c = 0; c < 3; ++c) v[c] += hdt_m * F[c];
            }
            if (opening) {    // step it: B A O A with lambda_{it+1}
                total_force(a.mode, fe, d, r_k, r_k2, lam_next, F);
                const double inv_n = 1.0 / r_n;
#pragma unroll
                for (int c = 0; c < 3; ++c) {
                    v[c] += hdt_m * F[c];
                    x[c] += 0.5 * a.dt * v[c];
                    const double m = a.fix_com ? zsum[c] * inv_n : 0.0;
                    v[c] = a.c1 * v[c] + r_c2 * (xii[c] - m);
                    x[c] += 0.5 * a.dt * v[c];
                }
                const double r0 = x[0] - xr[0], r1 = x[1] - xr[1], r2 = x[2] - xr[2];
                if (r0 * r0 + r1 * r1 + r2 * r2 > a.half_skin2) a.rebuild[tl.rep] = 1;
            }
            a.Pn[i] = make_double4(x[0], x[1], x[2], 0.0);
            // list builder uses box coordinates in both forms
            a.Qn[i] = make_uint4(box_code(x[0], r_invL[0]), box_code(x[1], r_invL[1]), box_code(x[2], r_invL[2]), 0u);
            a.v[i] = v[0];
            a.v[N + i] = v[1];
            a.v[2 * N + i] = v[2];
        }
    }

    if constexpr (sizeof(real) == 4 && kFix) on_grid<2>(e, kGridE, kGridEInv);
    unit_partial<3>(e, a.energy_part, tbase, tl.idx);   // e[2], a row length, is an integer
    if constexpr (kVir) {   // pressure evaluation: (1/2) pair virial plus m v_a^2 of the atom, per unit
        double pv[3] = {0.0, 0.0, 0.0};
        if (valid && lane == 0) {
            const double wv[3] = {Acc<real, kFix>::fin(w0), Acc<real, kFix>::fin(w1), Acc<real, kFix>::fin(w2)};
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                const double vc = a.v ? a.v[c * N + i] : 0.0;
                pv[c] = 0.5 * wv[c] + vc * vc / r_inv_m;
            }
        }
        if constexpr (sizeof(real) == 4 && kFix) on_grid<3>(pv, kGridE, kGridEInv);
        unit_partial<3>(pv, a.vir_part, tbase, tl.idx);
    }
    };   // unit
    run_units<kStage>(a, st, stage_table, unit);
}

// After a force pass: each replica's U_EAM and |x - x0|^2 from the unit
// partials (fixed order), dH/dl and the work increment of Eq. w_irr, and the
// iteration counter.  Run by one block of any size (multiple of 64), every
// thread of which calls it: g lanes per replica (the largest power of two up
// to 64 that fits the block), so the replicas load in parallel.
__device__ void finish_body(const StepArgs& a, int64_t it)
{
    int g = 64;
    while (g > 1 && g * a.n_rep > (int)blockDim.x) g >>= 1;
    const int grp = (int)threadIdx.x / g, sub = (int)threadIdx.x % g, ngrp = (int)blockDim.x / g;
    for (int r0 = 0; r0 < a.n_rep; r0 += ngrp) {
        const int r = r0 + grp;
        const bool work = r < a.n_rep && sub == 0 && a.step_kernel && it < a.it_last;
        // loads of the work state go out with the partials' loads
        const double W0 = work ? a.W_state[r] : 0.0;
        const double dl = work ? a.lam[it + 1] - a.lam[it] : 0.0;
        double tot[3] = {0.0, 0.0, 0.0};
        if (r < a.n_rep) {
            const RepDesc& R = a.reps[r];
            // the lane's units t = sub, sub + g, ... in batches of eight: every load of
            // a batch is issued before the first add, the adds keep the unit order
            constexpr int kB = 8;
            for (int t0 = sub; t0 < R.n_tiles; t0 += kB * g) {
                double p[kB][3];
#pragma unroll
                for (int b = 0; b < kB; ++b) {
                    const int t = t0 + b * g;
#pragma unroll
                    for (int k = 0; k < 3; ++k)
                        p[b][k] = t < R.n_tiles ? a.energy_part[(size_t)(R.tile_base + t) * 3 + k] : 0.0;
                }
#pragma unroll
                for (int b = 0; b < kB; ++b)
                    if (t0 + b * g < R.n_tiles)
#pragma unroll
                        for (int k = 0; k < 3; ++k) tot[k] += p[b][k];
            }
        }
        for (int o = g / 2; o > 0; o >>= 1)
#pragma unroll
            for (int k = 0; k < 3; ++k) tot[k] += __shfl_xor(tot[k], o, g);
        if (r < a.n_rep && sub == 0) {
            const RepDesc& R = a.reps[r];
            if (a.step_kernel) a.row_acc[r] += tot[2];   // list work of this pass
            a.U_rep[2 * r] = tot[0];
            a.U_rep[2 * r + 1] = tot[1];
            if (work) {
                const double UE = 0.5 * R.k * tot[1];
                double dH;
                switch (a.mode) {
                case MODE_FL: dH = UE - tot[0]; break;
                case MODE_RS: dH = tot[0]; break;
                case MODE_HH: dH = 0.5 * (R.k2 - R.k) * tot[1]; break;
                default: dH = UE; break;
                }
                const double W = W0 + dl * dH;
                a.W_state[r] = W;
                const size_t o = (size_t)r * a.S + (size_t)(it - a.trace_off);
                if (a.dHdl_out) a.dHdl_out[o] = dH;
                if (a.W_out) a.W_out[o] = W;
            }
        }
    }
    if (threadIdx.x == 0 && a.step_kernel) a.row_acc[a.n_rep] += 1.0;   // one more force pass in the history
}

// Finish of a force pass that no density pass of the same range follows:
// evaluation-only passes, the last pass of a range, and the modes without
// EAM (the other step passes are finished by an extra block of the next
// density pass, off the path of the list pass).
__global__ __launch_bounds__(1024) void k_finish(StepArgs a)
{
    finish_body(a, a.step_kernel ? *a.iter + a.it_k : 0);
}

// The device step counter of a captured graph's iterations, advanced once
// per replay (the graph's kernels read the step as the counter plus their
// iteration's offset).
__global__ void k_advance_iter(int64_t* iter, int64_t by) { *iter += by; }

int launch_advance_iter(int64_t* iter, int64_t by, hipStream_t s)
{
    hipLaunchKernelGGL(k_advance_iter, dim3(1), dim3(1), 0, s, iter, by);
    return (int)hipGetLastError();
}

// --------------------------------------------------------------------------
// Initial velocities: v = sqrt(kT/m) z(stream 1, step 0), centre of mass removed
// --------------------------------------------------------------------------
__global__ void k_init_v(StepArgs a, int fix_com)
{
    // one wavefront (block) per unit, one lane per atom
    const Tile tl = a.tiles[blockIdx.x];
    const RepDesc& R = a.reps[tl.rep];
    const bool valid = (int)threadIdx.x < tl.count;
    const int i = tl.first + (valid ? (int)threadIdx.x : 0);
    double z[3] = {0.0, 0.0, 0.0};
    if (valid) {
        gauss3(R.seed, (uint32_t)(i - R.off), 0, 1u, z[0], z[1], z[2]);
#pragma unroll
        for (int c = 0; c < 3; ++c) z[c] *= R.sig_v;
        // exact-sum form: the velocities on the 2^-36 grid, their mean an exact sum
        if (fix_com && a.fix) on_grid<3>(z, kGridZ, kGridZInv);
#pragma unroll
        for (int c = 0; c < 3; ++c) a.v[c * a.N + i] = z[c];
    }
    if (fix_com) unit_partial<3>(z, a.noise_part, R, tl.idx);
}

__global__ void k_sub_mean_v(StepArgs a)
{
    const Tile tl = a.tiles[blockIdx.x];
    const RepDesc& R = a.reps[tl.rep];
    double m[3];
    replica_total<3>(a.noise_part, R, m);
    if ((int)threadIdx.x >= tl.count) return;
    const int i = tl.first + threadIdx.x;
    const double inv_n = 1.0 / (double)R.n;
#pragma unroll
    for (int c = 0; c < 3; ++c) a.v[c * a.N + i] -= m[c] * inv_n;
}

// --------------------------------------------------------------------------
// Launchers
// --------------------------------------------------------------------------
static int grid1(int n, int b) { return (n + b - 1) / b; }

int launch_pack(double4* P, uint4* Q, const double* x, const int32_t* rep_of, const RepDesc* reps, int N,
                hipStream_t s)
{
    if (N <= 0) return 0;
    hipLaunchKernelGGL(k_pack, dim3(grid1(N, 256)), dim3(256), 0, s, P, Q, x, rep_of, reps, N);
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

static void allow_lds(const void* f, size_t bytes);

int launch_neigh_rebuild(const NeighArgs& a, const StepArgs& st, int lanes, int block, hipStream_t s)
{
    if (a.N <= 0) return 0;
    (void)lanes;
    (void)block;
    if (a.n_global > 0) {
        const int bin_blocks = 1 + std::min(1024, (a.N + kBinBlock - 1) / kBinBlock);
        hipLaunchKernelGGL(k_bin, dim3(bin_blocks), dim3(kBinBlock), 0, s, a, st);
        // one row buffer and one candidate chunk per wavefront
        const size_t lds = (size_t)((kListBlock / 64) * (a.cap + a.chunk)) * sizeof(int);
        if (lds > 64 * 1024) return (int)hipErrorInvalidValue;
        hipLaunchKernelGGL(k_list, dim3(kListGrid), dim3(kListBlock), lds, s, a, a.n_rep);
    }
    if (a.n_lds > 0) {
        const size_t lds = rows_lds_bytes(a.lds_atoms, a.lds_cells, a.cap, a.lds_waves);
        const void* f = reinterpret_cast<const void*>(&k_rows_lds);
        allow_lds(f, lds);
        hipLaunchKernelGGL(k_rows_lds, dim3(a.lds_grid), dim3(64 * a.lds_waves), lds, s, a, st);
    }
    return (int)hipGetLastError();
}

__global__ void k_rows_rowmajor(const int32_t* nbr, const int32_t* nnb, int N, int cap, int32_t* out, int out_cap)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= N) return;
    const int n = nnb[i] < cap ? nnb[i] : cap;
    for (int q = 0; q < n; ++q) out[(size_t)i * out_cap + q] = nbr[slot_index(i, q, N)];
    for (int q = n; q < out_cap; ++q) out[(size_t)i * out_cap + q] = -1;
}

__global__ void k_fill_u64(unsigned long long* p, size_t n, unsigned long long v)
{
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x)
        p[i] = v;
}

int launch_fill_u64(unsigned long long* p, size_t n, unsigned long long v, hipStream_t s)
{
    if (n == 0) return 0;
    const size_t blocks = std::min<size_t>((n + 255) / 256, 4096);
    hipLaunchKernelGGL(k_fill_u64, dim3((unsigned)blocks), dim3(256), 0, s, p, n, v);
    return (int)hipGetLastError();
}

int launch_rows_rowmajor(const int32_t* nbr, const int32_t* nnb, int N, int cap, int32_t* out, int out_cap,
                         hipStream_t s)
{
    if (N <= 0) return 0;
    hipLaunchKernelGGL(k_rows_rowmajor, dim3(grid1(N, 256)), dim3(256), 0, s, nbr, nnb, N, cap, out, out_cap);
    return (int)hipGetLastError();
}

template <typename real>
static size_t lds_bytes(const StepArgs& a, int tables)
{
    if (!a.has_eam) return 0;
    // FP32: n_r - 1 intervals and one padding interval per table, 16 bytes
    // each; FP64 (the density table, or the pair table as two): n_r - 1
    // intervals of 32 bytes
    return sizeof(real) == 4 ? (size_t)tables * a.tab.n_r * sizeof(float4) : (size_t)tables * (a.tab.n_r - 1) * 32;
}

// LDS one block may take on the current device (cached per device).
static size_t device_lds()
{
    static thread_local int cached[64] = {};
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return 65536;
    if (!cached[dev]) {
        int v = 0;
        cached[dev] = hipDeviceGetAttribute(&v, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) == hipSuccess && v > 0
                          ? v
                          : 65536;
    }
    return (size_t)cached[dev];
}

// FP64 pair kernels read their tables from LDS when the force pass's pair
// table (64 bytes per interval) fits one block's and the launch holds at
// least two units per compute unit; otherwise from global memory.  Staging
// the table costs each block a fixed latency (128 KB at 2000 knots), which
// a launch of few units, such as one replica of a few thousand atoms, does
// not earn back: there the pass is latency bound and the table's reads
// come from L2 at little cost.
template <typename real>
static bool fp64_lds(const StepArgs& a)
{
    return sizeof(real) == 8 && a.has_eam && lds_bytes<real>(a, 2) <= device_lds() && a.n_tiles >= 2 * a.n_cu;
}

// Resident blocks per CU of a pair kernel at this block size and LDS use
// (cached per kernel and shape; the query is host-only).
static int blocks_per_cu(const void* f, int block, size_t lds)
{
    struct Entry {
        const void* f;
        int block;
        size_t lds;
        int nb;
    };
    static thread_local std::vector<Entry> cache;
    for (const auto& e : cache)
        if (e.f == f && e.block == block && e.lds == lds) return e.nb;
    int nb = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, f, block, lds) != hipSuccess || nb < 1) nb = 1;
    cache.push_back({f, block, lds, nb});
    return nb;
}

// Persistent grid: every resident slot of the chip (or the caller's block
// count), but no more wavefronts than units.
static int pair_grid(const StepArgs& a, const void* f, int block, size_t lds)
{
    const int waves = block / 64;
    int need = 0;   // blocks that give every unit its own wavefront, per group
    for (int q = 0; q < a.nq; ++q) {
        const int len = a.qoff[q + 1] - a.qoff[q];
        need = need > (len + waves - 1) / waves ? need : (len + waves - 1) / waves;
    }
    need *= a.nq;
    int g = a.grid_blocks > 0 ? a.grid_blocks : a.n_cu * blocks_per_cu(f, block, lds);
    g = g < need ? g : need;
    return (g + a.nq - 1) / a.nq * a.nq;   // every group has blocks
}

// Dynamic LDS beyond the default limit needs the kernel's attribute raised
// once per size.
static void allow_lds(const void* f, size_t bytes)
{
    static thread_local std::vector<std::pair<const void*, size_t>> done;
    for (auto& d : done)
        if (d.first == f && d.second >= bytes) return;
    (void)hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
    done.push_back({f, bytes});
}

// Staged launch of the FP32 pair kernels: one block per slice, the table
// and the largest replica's records in LDS.
template <typename real>
static bool staged(const StepArgs& a)
{
    return sizeof(real) == 4 && a.has_eam && a.slice_grid > 0;
}

// Events stamped with a pair kernel's own start and end (HIP's extended
// launch), for sampled timing; null events: a plain launch.
struct Stamp {
    hipEvent_t t0, t1;
};

template <typename K>
static void launch_pair(K kernel, dim3 grid, dim3 block, size_t sh, hipStream_t s, const Stamp& ts,
                        const StepArgs& a)
{
    if (ts.t0)
        hipExtLaunchKernelGGL(kernel, grid, block, (uint32_t)sh, s, ts.t0, ts.t1, 0u, a);
    else
        hipLaunchKernelGGL(kernel, grid, block, sh, s, a);
}

template <typename real, int T, bool kFix>
static void density_one(const StepArgs& a, int block, hipStream_t s, const Stamp& ts)
{
    if constexpr (sizeof(real) == 4) {
        if (staged<real>(a)) {
            const size_t sh = lds_bytes<real>(a, 1) + (size_t)a.stage_atoms * sizeof(uint4);
            const void* f = reinterpret_cast<const void*>(&k_density<real, T, true, kFix>);
            allow_lds(f, sh);
            launch_pair(k_density<real, T, true, kFix>, dim3(a.slice_grid + a.finish_prev), dim3(block), sh, s, ts,
                        a);
            return;
        }
    }
    if constexpr (sizeof(real) == 8) {
        if (fp64_lds<real>(a)) {
            const size_t sh = lds_bytes<real>(a, 1);
            const void* f = reinterpret_cast<const void*>(&k_density<real, T, false, kFix, true>);
            allow_lds(f, sh);
            launch_pair(k_density<real, T, false, kFix, true>, dim3(pair_grid(a, f, block, sh) + a.finish_prev),
                        dim3(block), sh, s, ts, a);
            return;
        }
    }
    const size_t sh = sizeof(real) == 4 ? lds_bytes<real>(a, 1) : 0;
    const void* f = reinterpret_cast<const void*>(&k_density<real, T, false, kFix>);
    launch_pair(k_density<real, T, false, kFix>, dim3(pair_grid(a, f, block, sh) + a.finish_prev), dim3(block), sh,
                s, ts, a);
}

template <typename real, int T, bool kFix>
static void force_one(const StepArgs& a, int block, hipStream_t s, const Stamp& ts)
{
    if (a.vir_part) {   // pressure evaluation (not a step): the persistent form with the virial
        if constexpr (sizeof(real) == 8) {
            if (fp64_lds<real>(a)) {
                const size_t sh = lds_bytes<real>(a, 2);
                const void* f = reinterpret_cast<const void*>(&k_force<real, T, false, true, kFix, true>);
                allow_lds(f, sh);
                launch_pair(k_force<real, T, false, true, kFix, true>, dim3(pair_grid(a, f, block, sh)), dim3(block),
                            sh, s, ts, a);
                return;
            }
        }
        const size_t sh = sizeof(real) == 4 ? lds_bytes<real>(a, 2) : 0;
        const void* f = reinterpret_cast<const void*>(&k_force<real, T, false, true, kFix>);
        launch_pair(k_force<real, T, false, true, kFix>, dim3(pair_grid(a, f, block, sh)), dim3(block), sh, s, ts,
                    a);
        return;
    }
    if constexpr (sizeof(real) == 4) {
        if (staged<real>(a)) {
            const size_t sh = lds_bytes<real>(a, 2) + (size_t)a.stage_atoms * sizeof(uint4);
            const void* f = reinterpret_cast<const void*>(&k_force<real, T, true, false, kFix>);
            allow_lds(f, sh);
            launch_pair(k_force<real, T, true, false, kFix>, dim3(a.slice_grid), dim3(block), sh, s, ts, a);
            return;
        }
    }
    if constexpr (sizeof(real) == 8) {
        if (fp64_lds<real>(a)) {
            const size_t sh = lds_bytes<real>(a, 2);
            const void* f = reinterpret_cast<const void*>(&k_force<real, T, false, false, kFix, true>);
            allow_lds(f, sh);
            launch_pair(k_force<real, T, false, false, kFix, true>, dim3(pair_grid(a, f, block, sh)), dim3(block), sh,
                        s, ts, a);
            return;
        }
    }
    const size_t sh = sizeof(real) == 4 ? lds_bytes<real>(a, 2) : 0;
    const void* f = reinterpret_cast<const void*>(&k_force<real, T, false, false, kFix>);
    launch_pair(k_force<real, T, false, false, kFix>, dim3(pair_grid(a, f, block, sh)), dim3(block), sh, s, ts, a);
}

// lanes per atom and, in FP32, the accumulation form as template arguments
template <typename real, bool kFix>
static int density_lanes(const StepArgs& a, int lanes, int block, hipStream_t s, const Stamp& ts)
{
    switch (lanes) {
    case 1: density_one<real, 1, kFix>(a, block, s, ts); break;
    case 2: density_one<real, 2, kFix>(a, block, s, ts); break;
    case 4: density_one<real, 4, kFix>(a, block, s, ts); break;
    case 8: density_one<real, 8, kFix>(a, block, s, ts); break;
    case 16: density_one<real, 16, kFix>(a, block, s, ts); break;
    default: return (int)hipErrorInvalidValue;
    }
    return (int)hipGetLastError();
}

template <typename real, bool kFix>
static int force_lanes(const StepArgs& a, int lanes, int block, hipStream_t s, const Stamp& ts)
{
    switch (lanes) {
    case 1: force_one<real, 1, kFix>(a, block, s, ts); break;
    case 2: force_one<real, 2, kFix>(a, block, s, ts); break;
    case 4: force_one<real, 4, kFix>(a, block, s, ts); break;
    case 8: force_one<real, 8, kFix>(a, block, s, ts); break;
    case 16: force_one<real, 16, kFix>(a, block, s, ts); break;
    default: return (int)hipErrorInvalidValue;
    }
    return (int)hipGetLastError();
}

template <typename real>
static int launch_density_t(const StepArgs& a, int lanes, int block, hipStream_t s, const Stamp& ts)
{
    if (a.n_tiles <= 0) return 0;
    if (block < 64 || block > kMaxBlock || block % 64) return (int)hipErrorInvalidValue;
    if (sizeof(real) == 4 && !a.fix) return density_lanes<real, false>(a, lanes, block, s, ts);
    return density_lanes<real, true>(a, lanes, block, s, ts);
}

template <typename real>
static int launch_force_t(const StepArgs& a, int lanes, int block, hipStream_t s, const Stamp& ts)
{
    if (a.n_tiles <= 0) return 0;
    if (block < 64 || block > kMaxBlock || block % 64) return (int)hipErrorInvalidValue;
    if (sizeof(real) == 4 && !a.fix) return force_lanes<real, false>(a, lanes, block, s, ts);
    return force_lanes<real, true>(a, lanes, block, s, ts);
}

// --------------------------------------------------------------------------
// Mean-squared displacement from the lattice sites with the centre-of-mass
// displacement removed (Eq. msd): one block per replica, per-thread sums in a
// fixed stride, then a fixed tree.  msd = sum |d|^2 / n - |sum d / n|^2.
// --------------------------------------------------------------------------
constexpr int kMsdBlock = 256;

__global__ __launch_bounds__(kMsdBlock) void k_msd(const double* x, const double* x0, const RepDesc* reps, int N,
                                                   double* out)
{
    __shared__ double sh[4][kMsdBlock];
    const RepDesc& R = reps[blockIdx.x];
    double s[4] = {0.0, 0.0, 0.0, 0.0};
    for (int k = threadIdx.x; k < R.n; k += blockDim.x) {
        const int i = R.off + k;
        const double d0 = x[i] - x0[i], d1 = x[N + i] - x0[N + i], d2 = x[2 * N + i] - x0[2 * N + i];
        s[0] += d0;
        s[1] += d1;
        s[2] += d2;
        s[3] += d0 * d0 + d1 * d1 + d2 * d2;
    }
#pragma unroll
    for (int c = 0; c < 4; ++c) sh[c][threadIdx.x] = s[c];
    __syncthreads();
    for (int h = kMsdBlock / 2; h > 0; h >>= 1) {
        if ((int)threadIdx.x < h)
#pragma unroll
            for (int c = 0; c < 4; ++c) sh[c][threadIdx.x] += sh[c][threadIdx.x + h];
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        const double n = (double)R.n;
        const double m0 = sh[0][0] / n, m1 = sh[1][0] / n, m2 = sh[2][0] / n;
        out[blockIdx.x] = sh[3][0] / n - (m0 * m0 + m1 * m1 + m2 * m2);
    }
}

int launch_msd(const double* x, const double* x0, const RepDesc* reps, int n_rep, int N, double* out, hipStream_t s)
{
    if (n_rep <= 0) return 0;
    hipLaunchKernelGGL(k_msd, dim3(n_rep), dim3(kMsdBlock), 0, s, x, x0, reps, N, out);
    return (int)hipGetLastError();
}

int launch_finish(const StepArgs& a, hipStream_t s)
{
    if (a.n_rep <= 0) return 0;
    hipLaunchKernelGGL(k_finish, dim3(1), dim3(1024), 0, s, a);
    return (int)hipGetLastError();
}

int launch_density(const StepArgs& a, int precision, int lanes, int block, hipStream_t s, hipEvent_t t0,
                   hipEvent_t t1)
{
    const Stamp ts{t0, t1};
    return precision ? launch_density_t<float>(a, lanes, block, s, ts)
                     : launch_density_t<double>(a, lanes, block, s, ts);
}

int launch_force(const StepArgs& a, int precision, int lanes, int block, hipStream_t s, hipEvent_t t0, hipEvent_t t1)
{
    const Stamp ts{t0, t1};
    return precision ? launch_force_t<float>(a, lanes, block, s, ts) : launch_force_t<double>(a, lanes, block, s, ts);
}

int launch_init_velocities(const StepArgs& a, int n_rep, int fix_com, hipStream_t s)
{
    (void)n_rep;
    // units hold at most 64 atoms; one wavefront per unit, one lane per atom
    if (a.n_tiles <= 0) return 0;
    hipLaunchKernelGGL(k_init_v, dim3(a.n_tiles), dim3(64), 0, s, a, fix_com);
    if (fix_com) hipLaunchKernelGGL(k_sub_mean_v, dim3(a.n_tiles), dim3(64), 0, s, a);
    return (int)hipGetLastError();
}

// --------------------------------------------------------------------------
// Knot gradient dU/dtheta (theta = knot values of phi, rho, F).
// U is linear in the interval coefficients of phi and F, and rho_i is linear
// in those of rho, so with B(t) = (1, t, t^2, t^3) of every evaluation:
//   dU/dc_phi[m] = 1/2 sum over ordered pairs in interval m of B
//   dU/dc_rho[m] = sum_i F'(rho_i) sum_j over pairs in interval m of B
//   dU/dc_F[m]   = sum over atoms with rho_i in interval m of B
// Each block accumulates one function's bins in an LDS histogram (2^-32
// fixed point, 64-bit) over a contiguous range of work units and adds it to
// the replica's global bins when the replica changes.
// --------------------------------------------------------------------------
constexpr int kAdjBlock = 256;
constexpr int kAdjLanes = 8;

__device__ __forceinline__ unsigned long long fix64(double v)
{
    return (unsigned long long)__double2ll_rn(v * kFixScale);
}

template <typename real, int WHICH>
__global__ __launch_bounds__(kAdjBlock) void k_adjoint(AdjointArgs a)
{
    extern __shared__ unsigned long long hist[];
    constexpr bool kQ = sizeof(real) == 4;
    const int nint = (WHICH == 2 ? a.tab.n_rho : a.tab.n_r) - 1;
    for (int k = threadIdx.x; k < 4 * nint; k += blockDim.x) hist[k] = 0ull;
    __syncthreads();
    const int per = (a.n_units + gridDim.x - 1) / gridDim.x;
    const int u0 = blockIdx.x * per, u1 = min(a.n_units, u0 + per);
    int rep = -1;
    auto flush = [&]() {
        __syncthreads();
        unsigned long long* g = a.bins + ((size_t)rep * 3 + WHICH) * (size_t)a.nb * 4;
        for (int k = threadIdx.x; k < 4 * nint; k += blockDim.x) {
            const unsigned long long v = hist[k];
            if (v) {
                atomicAdd(&g[k], v);
                hist[k] = 0ull;
            }
        }
        __syncthreads();
    };
    const int A = a.tile_atoms;
    const int lane = threadIdx.x % kAdjLanes;
    const int slot = threadIdx.x / kAdjLanes;
    constexpr int per_pass = kAdjBlock / kAdjLanes;
    for (int u = u0; u < u1; ++u) {
        int r = rep < 0 ? 0 : rep;   // replica of unit u (units are replica-major)
        while (u >= a.reps[r].tile_base + a.reps[r].n_tiles) ++r;
        if (r != rep) {
            if (rep >= 0) flush();
            rep = r;
        }
        const RepDesc& R = a.reps[r];
        const int first = R.off + (u - R.tile_base) * A;
        const int count = min(A, R.n - (u - R.tile_base) * A);
        for (int c0 = 0; c0 < count; c0 += per_pass) {
            const int la = c0 + slot;
            if (la >= count) continue;
            const int i = first + la;
            if constexpr (WHICH == 2) {
                if (lane == 0) {
                    double td;
                    const int m = interval<double>(a.rho[i], a.tab.inv_h_rho, a.tab.n_rho, td);
                    atomicAdd(&hist[4 * m + 0], fix64(1.0));
                    atomicAdd(&hist[4 * m + 1], fix64(td));
                    atomicAdd(&hist[4 * m + 2], fix64(td * td));
                    atomicAdd(&hist[4 * m + 3], fix64(td * td * td));
                }
            } else {
                const double4 pi = a.P[i];
                const uint4 qi = kQ ? a.Q[i] : make_uint4(0u, 0u, 0u, 0u);
                const double wgt = WHICH == 0 ? 0.5 : (kQ ? (double)__uint_as_float(qi.w) : pi.w);
                const int n = a.nnb[i];
                for (int q = lane; q < n; q += kAdjLanes) {
                    // geometry in float64 in both forms: the basis weights B(t) vary on the
                    // scale of one interval, so t needs more than single precision
                    const int j = a.nbr[slot_index(i, q, a.N)];
                    double dx, dy, dz;
                    if constexpr (kQ) {
                        const uint4 qj = a.Q[j];
                        dx = (double)(int)(qi.x - qj.x) * (R.L[0] * 2.3283064365386963e-10);
                        dy = (double)(int)(qi.y - qj.y) * (R.L[1] * 2.3283064365386963e-10);
                        dz = (double)(int)(qi.z - qj.z) * (R.L[2] * 2.3283064365386963e-10);
                    } else {
                        const double3 d = sep(R, pi, a.P[j]);
                        dx = d.x;
                        dy = d.y;
                        dz = d.z;
                    }
                    const double r2 = dx * dx + dy * dy + dz * dz;
                    if (r2 < a.tab.rc2) {
                        double td;
                        const int m = interval<double>(sqrt(r2), a.tab.inv_h_r, a.tab.n_r, td);
                        atomicAdd(&hist[4 * m + 0], fix64(wgt));
                        atomicAdd(&hist[4 * m + 1], fix64(wgt * td));
                        atomicAdd(&hist[4 * m + 2], fix64(wgt * td * td));
                        atomicAdd(&hist[4 * m + 3], fix64(wgt * td * td * td));
                    }
                }
            }
        }
    }
    if (rep >= 0) flush();
}

// One thread per (output row, function): fixed-point bins -> coefficient
// gradients g = (g_a, g_b, g_c, d_d) per interval -> knot gradient through the
// transpose of the natural-spline map.  With y the knots and M the second
// derivatives (M_0 = M_{n-1} = 0, K M = r, K = tridiag(1, 4, 1),
// r_l = 6 (y_{l+1} - 2 y_l + y_{l-1}) / h^2):
//   a_m = y_m, b_m = y_{m+1} - y_m - h^2 (2 M_m + M_{m+1})/6,
//   c_m = h^2 M_m / 2, d_m = h^2 (M_{m+1} - M_m)/6,
// so dU/dy = direct terms + (dr/dy)^T K^{-1} (dU/dM).
__global__ void k_adjoint_finish(AdjointArgs a, const double* w, int reduce, double* out, double* scratch)
{
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    const int rows = reduce ? 1 : a.n_rep;
    if (t >= rows * 3) return;
    const int row = t / 3, f = t % 3;
    const int n = f == 2 ? a.tab.n_rho : a.tab.n_r;
    const double h = f == 2 ? 1.0 / a.tab.inv_h_rho : 1.0 / a.tab.inv_h_r;
    const int nmax = a.nb + 1;
    double* gM = scratch + (size_t)t * 2 * nmax;
    double* dg = gM + nmax;
    double* o = out + ((size_t)row * 3 + f) * nmax;
    const int r0 = reduce ? 0 : row, r1 = reduce ? a.n_rep : row + 1;
    auto g = [&](int m, int q) {   // coefficient gradient, fixed replica order
        double s = 0.0;
        for (int r = r0; r < r1; ++r) {
            const long long v = (long long)a.bins[(((size_t)r * 3 + f) * a.nb + m) * 4 + q];
            s += (w ? w[r] : 1.0) * ((double)v * kFixInv);
        }
        return s;
    };
    const double h2 = h * h;
    // dU/dM for interior knots, and the direct y terms
    for (int k = 0; k < n; ++k) {
        double dy = 0.0, gm = 0.0;
        if (k <= n - 2) dy += g(k, 0) - g(k, 1);
        if (k >= 1) dy += g(k - 1, 1);
        if (k >= 1 && k <= n - 2)
            gm = h2 / 6.0 * (-2.0 * g(k, 1) - g(k - 1, 1) + 3.0 * g(k, 2) - g(k, 3) + g(k - 1, 3));
        o[k] += dy;
        gM[k] = gm;
    }
    // solve K z = gM on the interior (Thomas); z overwrites gM
    dg[1] = 4.0;
    for (int k = 2; k <= n - 2; ++k) {
        const double q = 1.0 / dg[k - 1];
        dg[k] = 4.0 - q;
        gM[k] -= q * gM[k - 1];
    }
    gM[n - 2] /= dg[n - 2];
    for (int k = n - 3; k >= 1; --k) gM[k] = (gM[k] - gM[k + 1]) / dg[k];
    gM[0] = 0.0;
    gM[n - 1] = 0.0;
    const double s6 = 6.0 / h2;
    for (int k = 0; k < n; ++k) {
        double v = -2.0 * gM[k];
        if (k >= 1) v += gM[k - 1];
        if (k + 1 <= n - 1) v += gM[k + 1];
        o[k] += s6 * v;
    }
}

template <typename real>
static int launch_adjoint_t(const AdjointArgs& a, int grid, hipStream_t s)
{
    const size_t sh_r = (size_t)(a.tab.n_r - 1) * 4 * sizeof(unsigned long long);
    const size_t sh_f = (size_t)(a.tab.n_rho - 1) * 4 * sizeof(unsigned long long);
    hipLaunchKernelGGL((k_adjoint<real, 0>), dim3(grid), dim3(kAdjBlock), sh_r, s, a);
    hipLaunchKernelGGL((k_adjoint<real, 1>), dim3(grid), dim3(kAdjBlock), sh_r, s, a);
    hipLaunchKernelGGL((k_adjoint<real, 2>), dim3(grid), dim3(kAdjBlock), sh_f, s, a);
    return (int)hipGetLastError();
}

int launch_adjoint(const AdjointArgs& a, int precision, int grid, hipStream_t s)
{
    return precision ? launch_adjoint_t<float>(a, grid, s) : launch_adjoint_t<double>(a, grid, s);
}

int launch_adjoint_finish(const AdjointArgs& a, const double* w, int reduce, double* out, double* scratch,
                          hipStream_t s)
{
    const int threads = (reduce ? 1 : a.n_rep) * 3;
    hipLaunchKernelGGL(k_adjoint_finish, dim3((threads + 63) / 64), dim3(64), 0, s, a, w, reduce, out, scratch);
    return (int)hipGetLastError();
}

}  // namespace eamfe
