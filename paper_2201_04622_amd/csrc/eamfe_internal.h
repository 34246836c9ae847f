// Internal declarations shared by the host orchestration (eamfe_host.cpp) and
// the gfx950 kernels (eamfe_kernels.hip).  Not part of the public ABI.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace eamfe {

// Units: LAMMPS metal.
constexpr double kB = 8.617333262e-5;      // eV/K
constexpr double hbar = 6.582119569e-4;    // eV ps
constexpr double mvv2e = 1.0364269e-4;     // eV per amu A^2/ps^2

// Device status bits (latched with atomicOr, mapped to EAMFE_E* on read).
enum : int {
    ST_NEIGH_OVERFLOW = 1,
    ST_CELL_OVERFLOW = 2,
    ST_TABLE_RANGE = 4,
    ST_NONFINITE = 8,
};

enum : int { MODE_FL = 0, MODE_RS = 1, MODE_HH = 2, MODE_EIN_RS = 3 };

// Replicas per context (bounded by the list builder's LDS prefix table).
constexpr int kMaxRepsList = 8192;

// Fixed-point quantum of the FP32 accumulators: sums are carried as exact
// integers (multiples of 2^-32) inside float64, so addition is associative.
constexpr double kFixScale = 4294967296.0;          // 2^32
constexpr double kFixInv = 2.3283064365386963e-10;  // 2^-32

// Replica descriptor as the kernels see it.
struct RepDesc {
    int32_t off;        // first global atom
    int32_t n;          // atoms
    int32_t tile_base;  // first slot of this replica in per-unit partial arrays
    int32_t n_tiles;    // work units of this replica
    int32_t cell_base;  // first global cell (replicas whose lists are built in global memory)
    int32_t nc[3];      // cells per edge; nc[0] == 0 selects all-pairs lists
    int32_t lds;        // 1: lists built from LDS by k_rows_lds (no global cells); 0: k_bin / k_list
    int32_t pad_;
    double L[3];
    double invL[3];
    double T, k, k2, mass;
    double inv_m;       // 1 / (m mvv2e): (A/ps^2) per (eV/A)
    double sig_v;       // sqrt(kB T / (m mvv2e)), A/ps
    double c2;          // thermostat noise amplitude of the current protocol
    uint64_t seed;
};

// A tile (work unit) is a contiguous run of at most 64/T atoms of one
// replica: the atoms of one wavefront of the pair kernels.
struct Tile {
    int32_t rep;
    int32_t first;   // global atom index of the first atom
    int32_t count;   // atoms in the unit
    int32_t idx;     // unit index within its replica
};

// Spline tables (device pointers, element type set by precision).
// pair[m]: {phi a, b, c, d, rho' b/h, 2c/h, 3d/h, 0}; rho[m], F[m]: {a, b, c, d}
struct Tables {
    const void* pair;
    const void* rho;
    const void* F;
    int n_r, n_rho;
    double r_cut, rc2, inv_h_r, inv_h_rho, rho_max;
};

struct NeighArgs {
    const Tile* tiles;
    const RepDesc* reps;
    const int32_t* rep_of;      // [N] replica of each atom
    const int32_t* cell_rep;    // [n_cells] replica of each cell
    const double4* P;           // [N] packed positions (x, y, z, .)
    const uint4* Q;             // [N] box coordinates frac(x/L) 2^32
    double* xref;               // SoA [3][N]
    int32_t* cell_cnt;          // [n_cells]
    int32_t* cell_atoms;        // [n_cells][ccap] local atom ids
    int32_t* nbr;               // [N][cap] global atom ids
    int32_t* nnb;               // [N]
    int32_t* rebuild;           // [n_rep] flags
    int32_t* flag_pre;          // [2 (n_rep + 1)] prefix of flagged atoms, then of flagged cells
    int32_t* status;
    int N, n_cells, ccap, cap;
    int chunk;                  // candidates staged per wavefront in the row builder (>= ccap)
    int n_rep;
    const int32_t* lds_list;    // [n_lds] replicas whose lists k_rows_lds builds, in replica order
    int n_lds;                  // their number (0: none)
    int n_global;               // replicas whose lists k_bin / k_list build
    int lds_atoms;              // the largest of them: atoms (records and sorted ids staged per block)
    int lds_cells;              // and cells (cell starts staged per block)
    int lds_waves;              // wavefronts per block of k_rows_lds
    int lds_grid;               // row-building blocks of k_rows_lds (one more block finishes the force pass)
    double rl2;                 // (r_cut + skin)^2
    float rl2_f;                // (r_cut + skin + margin)^2 for the single-precision candidate test
    double half_skin2;          // (skin/2)^2
};

// Everything one MD iteration's kernels need.
struct StepArgs {
    const Tile* tiles;
    const RepDesc* reps;
    double4* P;             // [N] positions at the start of the iteration, .w = F'(rho_i) (FP64 form)
    double4* Pn;            // [N] positions after the step
    uint4* Q;               // [N] FP32 form: box coordinates frac(x/L) 2^32 per axis, .w = F'(rho_i) bits
    uint4* Qn;              // [N] box coordinates after the step
    double* v;              // SoA, in place
    const double* x0;       // SoA
    const double* kscale;   // [N] per-atom spring scales s_i (atom i's spring k s_i) or null (all 1)
    const double* xref;     // SoA, list reference positions
    const int32_t* nbr;
    const int32_t* nnb;
    int cap;
    double* e_emb;          // [N] F(rho_i)
    double* xi;             // [3][N] thermostat noise of this step
    double* noise_part;     // [units][3] thermostat noise summed per unit
    double* energy_part;    // [units][3] U_EAM, |x - x0|^2 and row lengths summed per unit
    double* vir_part;       // [units][3] pressure evaluation: virial/2 + m v^2 per axis per unit, or null
    double* U_rep;          // [n_rep][2]: U_EAM, sum |x-x0|^2 at x
    int32_t* rebuild;       // [n_rep]
    int32_t* cell_cnt;      // [n_cells] bin counters (cleared by the density pass after a rebuild)
    int32_t* flag_pre;      // [2 (n_rep + 1)] rebuild prefix (formed by the list pass's first kernel)
    double* row_acc;        // [n_rep + 3] row lengths summed over the step force passes, their count, then
                            // the replicas and the atoms whose lists those passes rebuilt
    int32_t* status;
    const double* lam;      // lambda table [S+1]
    int64_t* iter;          // device step counter: a pass's step is *iter + it_k
    int64_t it_k;           // this pass's step offset from the counter (its iteration within a captured graph)
    int finish_prev;        // density pass: an extra block finishes the force pass of the step before
    int64_t it_first;       // first iteration of this launch sequence: no closing kick
    int64_t it_last;        // last iteration: no new step (only the closing kick)
    double* dHdl_out;       // [n_rep][S] or null
    double* W_out;          // [n_rep][S] or null
    int64_t S;              // row stride of the traces
    int64_t trace_off;      // trace column = it - trace_off
    double* W_state;        // [n_rep]
    double* f_out;          // SoA [3][N] EAM forces or null
    double* e_atom_out;     // [N] per-atom EAM energy or null
    double* rho_out;        // [N] densities rho_i or null
    Tables tab;
    int N;
    int mode;
    int fix_com;
    int has_eam;
    int n_tiles;            // work units (one wavefront's atoms of one replica each)
    int n_rep;
    int grid_blocks;        // persistent blocks of the pair kernels (0: fill every resident slot)
    int n_cu;               // compute units of the device
    int nq;                 // unit groups (8 with XCD affinity, else 1)
    int qoff[9];            // units of group q: tiles[qoff[q] .. qoff[q+1])
    const int4* slices;     // [slice_grid] per block of a staged launch: first unit, units (one replica),
                            // the replica's first atom and atom count
    int slice_grid;         // blocks of the staged FP32 pair launches (0: records gathered from global memory)
    int stage_atoms;        // records staged per block (atoms of the largest replica)
    int step_kernel;        // 1: integrate; 0: evaluate only (eam_forces)
    int fix;                // FP32 only: fixed-point per-atom sums and exact replica sums (1), plain float64 sums (0)
    double dt;
    double c1;
    double half_skin2;
};

// Knot gradient dU/dtheta.  Bins hold per-interval sums of (1, t, t^2, t^3)
// times the weight of each evaluation, in 2^-32 fixed point (two's
// complement in 64 bits), so accumulation order does not matter.
struct AdjointArgs {
    const RepDesc* reps;
    const double4* P;           // positions (FP64 form), .w = F'(rho_i)
    const uint4* Q;             // box coordinates (FP32 form), .w = F'(rho_i) bits
    const int32_t* nbr;
    const int32_t* nnb;
    int cap;
    const double* rho;          // [N] densities from the density pass
    unsigned long long* bins;   // [n_rep][3][nb][4], nb = max(n_r, n_rho) - 1; functions (phi, rho, F)
    int nb;
    Tables tab;
    int N;
    int n_rep;
    int tile_atoms;             // atoms per work unit
    int n_units;                // total work units (replica-major)
};

// LDS of one block of the LDS row builder (k_rows_lds): the records and
// sorted ids of up to `atoms` atoms, `cells` + 1 cell starts, and per
// wavefront a row buffer of `cap` slots.
constexpr int kRowsAtomsMax = 4096;    // replicas of at most this many atoms (16-bit ids, 64 KB of records)
constexpr int kRowsCellsMax = 4096;    // and at most this many cells use it

__host__ __device__ inline size_t rows_lds_wave_bytes(int cap)
{
    return (size_t)cap * 4;   // the row buffer
}

__host__ __device__ inline size_t rows_lds_bytes(int atoms, int cells, int cap, int waves)
{
    const size_t head = (size_t)atoms * 16 + (((size_t)atoms * 2 + 15) & ~(size_t)15) +
                        (((size_t)(cells + 1) * 4 + 15) & ~(size_t)15);
    return head + (size_t)waves * rows_lds_wave_bytes(cap);
}

// Launchers (eamfe_kernels.hip).  Each returns a hipError_t as int.
int launch_pack(double4* P, uint4* Q, const double* x, const int32_t* rep_of, const RepDesc* reps, int N,
                hipStream_t s);
int launch_unpack(double* x, const double4* P, int N, hipStream_t s);
int launch_check_displacement(const NeighArgs& a, hipStream_t s);
// List pass.  Its first kernel also forms the prefix of the flagged replicas
// (the force pass before it is finished by the next density pass).
int launch_neigh_rebuild(const NeighArgs& a, const StepArgs& st, int lanes, int block, hipStream_t s);
// t0, t1 (optional): events stamped with the pair kernel's own start and end
int launch_density(const StepArgs& a, int precision, int lanes, int block, hipStream_t s, hipEvent_t t0 = nullptr,
                   hipEvent_t t1 = nullptr);
int launch_force(const StepArgs& a, int precision, int lanes, int block, hipStream_t s, hipEvent_t t0 = nullptr,
                 hipEvent_t t1 = nullptr);
// per-replica energies, dH/dl and work after a force pass that no density
// pass of the same range follows
int launch_finish(const StepArgs& a, hipStream_t s);
// *iter += by on the stream (the step counter of a captured graph's iterations)
int launch_advance_iter(int64_t* iter, int64_t by, hipStream_t s);
int launch_init_velocities(const StepArgs& a, int n_rep, int fix_com, hipStream_t s);
// per-replica mean-squared displacement from x0 with the centre of mass removed -> out[n_rep] (device)
int launch_msd(const double* x, const double* x0, const RepDesc* reps, int n_rep, int N, double* out, hipStream_t s);
int launch_adjoint(const AdjointArgs& a, int precision, int grid, hipStream_t s);
// Coefficient-bin sums -> knot gradients.  out[r][f][k] += w[r] dU_r/dtheta_{f,k}
// (per replica), or out[f][k] += sum_r w[r] dU_r/dtheta_{f,k} when reduce;
// scratch: device doubles, >= 3 * 3 * nmax per output row.
int launch_adjoint_finish(const AdjointArgs& a, const double* w, int reduce, double* out, double* scratch,
                          hipStream_t s);
// Rows in [N][out_cap] row-major order (slots past the row length = -1).
int launch_rows_rowmajor(const int32_t* nbr, const int32_t* nnb, int N, int cap, int32_t* out, int out_cap,
                         hipStream_t s);
int launch_rho(const StepArgs& a, double* rho_out, int precision, int lanes, int block, hipStream_t s);
// p[0 .. n) = v (a fill kernel, so that the clearing can sit inside a captured graph)
int launch_fill_u64(unsigned long long* p, size_t n, unsigned long long v, hipStream_t s);

}  // namespace eamfe
