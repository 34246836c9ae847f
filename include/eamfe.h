/*
 * eamfe.h -- C ABI of the MI355X (gfx950) nonequilibrium free-energy engine
 * for EAM solids: Langevin MD under a lambda-dependent Hamiltonian with the
 * irreversible work accumulated on the device.
 *
 * Method (arXiv 2201.04622):
 *   Frenkel--Ladd path   H(l) = (1-l) H0 + l H_E          (Eq. interp, Eq. H, Eq. einstein)
 *   Reversible scaling   H(l) = KE + l U                   (Eq. H_rs)
 *   work                 W = sum_k (l_{k+1} - l_k) dH/dl(G_k)   (Eq. w_irr, discrete form)
 *   schedules            ti/spring phases and lambda(tau) forms (Sec. fl_lammps),
 *                        RS lambda(tau) = 1/(1 + tau (1/l_f - 1)) (Sec. RS in LAMMPS)
 *   estimators           Eq. W12, Eq. Ediss, Eq. fl (+ Eq. cm), Eq. rs, Eq. jarz
 *   spring constants     Eq. msd (mean-squared displacement), per-atom springs
 *   constant pressure    pressure tensor; isotropic or orthorhombic stochastic cell
 *                        rescaling between fixed-volume stretches (RS at p = 0 gives G(T))
 *
 * Conventions for every entry point:
 *   - Units are LAMMPS "metal": eV, Angstrom, ps, amu, K.
 *   - "device" pointers are HIP device memory owned by the caller (for
 *     example a torch tensor's data_ptr()); "host" pointers are ordinary
 *     memory read or written before the call returns.  The library never
 *     frees caller memory.
 *   - Internal device buffers (neighbour lists, cell bins, tables, packed
 *     positions, partial sums, the lambda table, snapshots) live in one
 *     arena.  Once the caller hands over a workspace (eamfe_set_workspace)
 *     the arena is the caller's memory and the library allocates nothing on
 *     the device: a call that needs more (a larger system, longer rows after
 *     an overflow, a longer lambda table) returns EAMFE_ENOMEM without
 *     effect, eamfe_workspace_bytes gives the size it needs, and the caller
 *     passes a larger workspace and repeats the call (an interrupted
 *     run_switching resumes at eamfe_resume_step).  Without a workspace the
 *     library allocates its own arena in the setup calls and grows it
 *     there, and frees it in eamfe_destroy.
 *   - Positions, velocities and forces are SoA float64 [3][N_tot]
 *     (x of all atoms, then y, then z); replicas are stored back to back in
 *     the order given to eamfe_system_setup.  Positions are unwrapped
 *     (never folded into the box); pair separations use the minimum image.
 *   - Work runs on the context's HIP stream.  Every call returns an int
 *     status; calls that end with a stream synchronisation also report
 *     conditions the kernels latched (overflow, table range, non-finite).
 *     Nothing throws across the ABI.  A context is not thread safe.
 */
#ifndef EAMFE_H
#define EAMFE_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- status codes ------------------------------------------------------ */
#define EAMFE_OK               0
#define EAMFE_EINVAL           1   /* bad argument                                  */
#define EAMFE_ENOMEM           2   /* device or host allocation failed              */
#define EAMFE_EDEVICE          3   /* HIP runtime error                             */
#define EAMFE_ESTATE           4   /* call out of order (e.g. forces before setup)  */
#define EAMFE_EBOX             5   /* a box edge is <= 2 (r_cut + skin)             */
#define EAMFE_ENEIGH_OVERFLOW  6   /* an atom had more than max_neighbors candidates */
#define EAMFE_ECELL_OVERFLOW   7   /* a binning cell overflowed                     */
#define EAMFE_ETABLE_RANGE     8   /* some density rho_i > rho_max                  */
#define EAMFE_ENONFINITE       9   /* NaN/Inf in positions, forces or energies      */

/* numeric form of the pair arithmetic */
#define EAMFE_FP64 0   /* all arithmetic in float64                                    */
#define EAMFE_FP32 1   /* pair terms, densities, tables in float32; positions, velocities,
                          energies and work in float64.  Per-atom sums are float32
                          partials over groups of four consecutive list slots, rounded
                          to 2^-32 and added exactly in fixed point; replica sums
                          add energies rounded to 2^-24 and, with the centre of mass
                          held, thermostat deviates and initial velocities that are
                          themselves on the 2^-36 grid, exactly.  Results are bitwise reproducible and the
                          same for every launch shape and either list builder.  The
                          slot groups follow the rows: rebuilding the lists at
                          another step changes the rounding (the last bits). */

/* Hamiltonian family (dH/dl in brackets) */
#define EAMFE_MODE_FL      0   /* (1-l) U_EAM + l U_E(k)          [U_E - U_EAM]  Eq. interp/w_irr2 */
#define EAMFE_MODE_RS      1   /* l U_EAM                         [U_EAM]        Eq. H_rs/w_irr_rs */
#define EAMFE_MODE_HH      2   /* (1-l) U_E(k) + l U_E(k2)        [U_E(k2)-U_E(k)] harmonic test path */
#define EAMFE_MODE_EIN_RS  3   /* l U_E(k)                        [U_E(k)]       RS on an Einstein crystal */

typedef struct eamfe_ctx eamfe_ctx;

/* One replica: an independent periodic system.  x0 sites are given on the
 * device in eamfe_system_setup. */
typedef struct eamfe_replica {
    int32_t  n_atoms;
    int32_t  pad_;
    double   box[3];    /* orthorhombic box edges, Angstrom                      */
    double   T;         /* thermostat temperature, K                             */
    double   k;         /* Einstein spring (FL, EIN_RS) or k1 (HH), eV/A^2        */
    double   k2;        /* final spring of the HH test path, eV/A^2              */
    double   mass;      /* amu                                                   */
    uint64_t seed;      /* Philox key of this replica                            */
} eamfe_replica;

/* A switching protocol (shared by every replica of the context).
 * FL/HH (ti/spring phases, Sec. fl_lammps):
 *   [n_eq at l=0][n_sw forward 0->1][n_hold at 1][n_sw backward 1->0][n_hold2 at 0]
 * RS/EIN_RS (Sec. RS in LAMMPS):
 *   [n_eq at 1][n_sw forward 1->lambda_f][n_hold at lambda_f][n_sw backward][n_hold2 at 1]
 * tau = (switching steps done)/n_sw; the backward branch is the time reverse.
 * S = n_eq + 2 n_sw + n_hold + n_hold2 steps in total. */
typedef struct eamfe_protocol {
    int32_t mode;        /* EAMFE_MODE_*                                        */
    int32_t function;    /* FL/HH lambda(tau): 1 = tau, 2 = tau^5(70tau^4-315tau^3+540tau^2-420tau+126) */
    int32_t fix_com;     /* 1: thermostat noise has zero mean per replica (fixed centre of mass) */
    int32_t n_eq, n_sw, n_hold, n_hold2;
    int32_t pad_;
    double  dt;          /* ps (the paper uses 0.001)                           */
    double  damp;        /* Langevin relaxation time, ps; gamma = 1/damp; 0 = NVE (velocity Verlet) */
    double  lambda_f;    /* RS end point T0/T_f                                 */
    double  skin;        /* Verlet skin, Angstrom (list rebuilt when an atom moves > skin/2) */
} eamfe_protocol;

/* ---- context ----------------------------------------------------------- */

/* Create a context on HIP device `device`, issuing work on `hip_stream`
 * (a hipStream_t; NULL = the legacy default stream).  precision is
 * EAMFE_FP64 or EAMFE_FP32.  deterministic (EAMFE_FP32 only; 0 or 1): 1
 * rounds every float32 partial sum of four list slots to the 2^-32 grid,
 * every energy or virial term of a replica sum to 2^-24, and (centre of mass
 * held) the thermostat deviates and initial velocities themselves to 2^-36,
 * and adds them exactly (results bitwise reproducible and independent of the
 * launch shape; the removed mean is the exact mean of the applied values);
 * 0 adds them in float64 as they are (bitwise reproducible run to run for
 * one launch shape, not across shapes).
 * No device memory is taken here.  *ctx is set on success. */
int eamfe_create(eamfe_ctx** ctx, int device, void* hip_stream, int precision, int deterministic);

/* Free the library's own arena (never a caller's workspace).  NULL is accepted. */
int eamfe_destroy(eamfe_ctx* ctx);

/* Device bytes the context's buffers need now, or, after a call returned
 * EAMFE_ENOMEM for want of workspace, the bytes that call needs. */
int eamfe_workspace_bytes(const eamfe_ctx* ctx, size_t* bytes);

/* Hand the context a device workspace `dev` of `bytes` bytes (256-byte
 * aligned; for example a torch uint8 tensor's data_ptr()), owned by the
 * caller and kept valid until the next eamfe_set_workspace or
 * eamfe_destroy.  The current buffers are copied into it (the stream is
 * synchronised first), after which the previous workspace may be freed by
 * its owner.  From then on the library allocates no device memory.
 * dev = NULL with bytes = 0 selects caller-owned memory before any setup.
 * EAMFE_ENOMEM if bytes is less than eamfe_workspace_bytes reports. */
int eamfe_set_workspace(eamfe_ctx* ctx, void* dev, size_t bytes);

/* After run_switching (or switch_step) returned EAMFE_ENOMEM: the step at
 * which it stopped, with x, v and the carried work the state at that step;
 * calling run_switching again from there (after a larger workspace) continues
 * bitwise as the uninterrupted run.  -1 if no run was interrupted. */
int eamfe_resume_step(const eamfe_ctx* ctx, int64_t* step);

/* Device allocations the library made itself (hipMalloc calls); stays 0 for
 * a context given a workspace before its first setup call. */
int eamfe_device_allocations(const eamfe_ctx* ctx, int64_t* n);

/* Text of the last error of this context (static storage inside ctx). */
const char* eamfe_last_error(const eamfe_ctx* ctx);

/* Change the stream later calls use. */
int eamfe_set_stream(eamfe_ctx* ctx, void* hip_stream);

/* Launch shape of the pair kernels: lanes per atom (1, 2, 4, 8 or 16) and
 * threads per block (64..1024, multiple of 64).  0 keeps the current value.
 * In EAMFE_FP32 results are bit-identical for every shape. */
int eamfe_set_launch(eamfe_ctx* ctx, int lanes_per_atom, int block_threads);
int eamfe_get_launch(const eamfe_ctx* ctx, int* lanes_per_atom, int* block_threads);

/* Autotuner: time `trial_steps` steps of protocol p from `step` at every
 * launch shape (lanes per atom x block threads x persistent grid) on copies
 * of the caller's state (x_dev, v_dev are not modified; the work carried by
 * the context is restored) and keep the fastest shape; then, at that shape,
 * keep the faster of the two list builders (eamfe_set_list_builder), timed
 * over at least 100 steps (at most to the protocol's end).  Before it
 * returns it builds the lists again at the caller's positions x_dev (as
 * eamfe_neigh_build with the protocol's skin and automatic capacity), so a
 * deterministic EAMFE_FP32 run continues bitwise as one whose lists were
 * rebuilt at `step`, and the next pass starts from valid lists.  Outputs
 * (may be NULL): the chosen lanes and block threads, and its time per step
 * in ms. */
int eamfe_autotune(eamfe_ctx* ctx, const eamfe_protocol* p, int64_t step, const double* x_dev,
                   const double* v_dev, int trial_steps, int* lanes_out, int* block_out, double* ms_per_step);

/* Blocks of the density and force passes.  0 (default): in EAMFE_FP32,
 * when the pair table and the largest replica's gather records fit one
 * block's LDS, one block per replica slice (a run of work units of one
 * replica, about n_CU blocks in all), which copies its replica's records
 * into LDS and gathers neighbours from there; otherwise (FP64, larger
 * replicas) a persistent grid of as many blocks as the chip holds resident,
 * or fewer when every unit has its own wavefront.  blocks > 0 (rounded up
 * to a multiple of 8) asks for that persistent grid.  A work unit is the
 * atoms of one wavefront, 64/lanes atoms of one replica; in the persistent
 * form each wavefront takes a fixed stride of units.  Results are the same
 * bit for bit in every form. */
int eamfe_set_grid(eamfe_ctx* ctx, int blocks);
int eamfe_get_grid(const eamfe_ctx* ctx, int* blocks);

/* Replay the steps of run_switching from a captured HIP graph of `iters`
 * iterations (rounded up to even; 0 = eager launches, the default).  The
 * first and last iteration of every chunk run eagerly; the graph runs on an
 * internal default-priority stream ordered after and before the context's
 * stream with events.  Kernel timing or adjoint sampling switch it off. */
int eamfe_set_graph(eamfe_ctx* ctx, int iters);

/* Neighbour-list builder.  lds = 1 (default): replicas of at most 4096 atoms
 * and 4096 cells have their rows built by one kernel over one block per
 * compute unit, which stages each flagged replica's positions in LDS, sorts
 * its atoms into cells there and builds the rows from LDS; larger replicas
 * use the global-memory binning and row kernels.  lds = 0: every replica
 * through the global-memory kernels.  The rows are identical either way
 * (the same cells, stencil order and member order).  The lists are built
 * again by the next pass. */
int eamfe_set_list_builder(eamfe_ctx* ctx, int lds);
int eamfe_get_list_builder(const eamfe_ctx* ctx, int* lds);

/* 1: bin the replicas into eight groups balanced by atom count; group x is
 * spread over the blocks on XCD x (workgroup id mod 8), so a replica's atoms
 * stay in one XCD's L2.  0: one group.  Default 1. */
int eamfe_set_xcd_affinity(eamfe_ctx* ctx, int on);

/* Synchronise the stream and return the first latched device condition
 * (EAMFE_ENEIGH_OVERFLOW ...), clearing it. */
int eamfe_check(eamfe_ctx* ctx);

/* Time kernel launches with HIP events: the first iteration run after this
 * call and then every `stride`-th iteration (counted over the iterations the
 * stepping calls run, so any range of at least one iteration is sampled);
 * stride 0 stops.  `kinds` selects the kernels timed: bit 0 the density
 * pass, bit 1 the force pass (each stamped with the kernel's own start and
 * end by HIP's extended launch), bit 2 the neighbour-list rebuild sequence
 * (events recorded around its kernels on the context's stream; 0 = all
 * three).  A sampled launch costs the stream a few microseconds, so a stride
 * of tens and one kind keep the timed work essentially unperturbed.  Each
 * call resets the accumulators. */
int eamfe_set_kernel_timing(eamfe_ctx* ctx, int stride, int kinds);

/* Synchronise and return the summed event times (ms) and launch counts of
 * the density pass [0], the force pass [1] and the neighbour-list rebuild
 * sequence [2] since timing was switched on or last read; then reset.
 * ms_total and launches point to host arrays of 3 (either may be NULL). */
int eamfe_kernel_timing(eamfe_ctx* ctx, double* ms_total, int64_t* launches);

/* Neighbour-row statistics of the current lists (synchronises): mean and
 * maximum row length over all atoms, and the row capacity. */
int eamfe_list_stats(eamfe_ctx* ctx, double* mean_len, int* max_len, int* capacity);

/* List work of the step force passes (run_switching, switch_step) since the
 * last reset: their number, and the Verlet row length averaged over those
 * passes and over all atoms (each pass weighted by the rows it used), the
 * n_L of the per-atom algorithmic byte count.  Synchronises.  reset != 0
 * clears the history after reading.  A range replayed after a row or bin
 * overflow is counted once. */
int eamfe_row_history(eamfe_ctx* ctx, double* mean_len, int64_t* passes, int reset);

/* Neighbour-list rebuilds of the step passes since the last reset of the
 * row history: replica_rebuilds counts each replica whose lists a pass
 * rebuilt (an atom had moved more than skin/2, or the run started), and
 * atoms_rebuilt the atoms of those rebuilds.  Either pointer may be NULL.
 * Synchronises; a range replayed after a row or bin overflow is counted
 * once. */
int eamfe_list_rebuilds(eamfe_ctx* ctx, int64_t* replica_rebuilds, int64_t* atoms_rebuilt);

/* Diagonal of each replica's pressure tensor at positions x_dev (device SoA)
 * and velocities v_dev (device SoA, or NULL for the configurational part):
 * P_aa = (sum_i m v_ia^2 + W_aa) / V with the pair virial W_aa = sum_{i<j}
 * (x_i - x_j)_a f_ij,a of the EAM forces (H0).  The paper holds the
 * hydrostatic pressure at zero with a barostat to fix the lattice parameter
 * of its Frenkel--Ladd runs (Sec. p_fl); averaged over fixed-volume runs at
 * trial lattice parameters this gives that lattice parameter.  P[n_rep][3]
 * is a host array in eV/A^3 (1 eV/A^3 = 160.2177 GPa).  Synchronises;
 * a list or bin overflow enlarges the lists and evaluates again. */
int eamfe_pressure(eamfe_ctx* ctx, const double* x_dev, const double* v_dev, double* P);

/* Stochastic cell rescaling (Bernetti and Bussi, J. Chem. Phys. 153,
 * 114107, 2020), one coupling move per call, made between fixed-volume runs
 * of run_switching.  It holds the pressure the paper holds with a barostat:
 * at zero in its reversible-scaling runs (Sec. p_rs), while the lattice
 * parameter of its Frenkel--Ladd runs is fixed (Sec. p_fl), and with each
 * direction on its own for hcp (the per-direction barostat of the size
 * study, Sec. on free-energy size dependence).  At positions x_dev and
 * velocities v_dev (device SoA [3][N_tot] FP64, both updated in place)
 * each replica's internal pressure of H = w_eam U_EAM along axis a,
 *   P_aa = (sum_i m v_ia^2 + w_eam W_aa) / V,  W_aa the pair virial,
 * moves the box.  Isotropic (aniso = 0): eps = ln V moves by
 *   d eps = -(beta_T / tau_p) (p0 - P - kB T / V) dt + sqrt(2 kB T beta_T dt / (V tau_p)) z0,
 * P the mean of the P_aa, and positions and edges scale by exp(d eps / 3).
 * Orthorhombic (aniso = 1): each edge moves on its own, eps_a = ln L_a,
 *   d eps_a = -(beta_T / (3 tau_p)) (p0 - P_aa - kB T / V) dt + sqrt(2 kB T beta_T dt / (3 V tau_p)) z_a,
 * whose sum over the axes is the isotropic move of ln V; positions and edges
 * along a scale by exp(d eps_a).  Velocities scale by the inverse factors.
 * T is the replica's temperature and (z0, z1, z2) the three Box--Muller
 * deviates of Philox stream 3 under the replica's seed at counter (atom 0,
 * step).  w_eam is the weight of U_EAM in the Hamiltonian at the step
 * boundary `step`: lambda_step of the schedule in reversible scaling (where,
 * with p0 = 0, this keeps the scaled system at the zero pressure of the real
 * one at T0 / lambda), 1 for plain dynamics of U_EAM.  The spring anchors x0
 * are not moved, so the move suits runs without springs.  The lists are
 * planned again for the new boxes by the next pass.  mu_host[n_rep][3] and
 * P_host[n_rep][3] (host, may be NULL) return each axis's factor and P_aa.
 * EAMFE_EBOX leaves everything unchanged if a box edge would fall to
 * 2 (r_cut + skin) or below.  Synchronises. */
typedef struct eamfe_barostat {
    double p0;       /* target pressure, eV/A^3 */
    double tau_p;    /* coupling time, ps (> 0) */
    double beta_T;   /* compressibility, A^3/eV: sets the relaxation rate, not the sampled distribution */
    double dt;       /* time between moves (the coupling interval), ps */
    int32_t aniso;   /* 0: isotropic; 1: each box edge on its own (orthorhombic) */
    int32_t pad_;
} eamfe_barostat;
int eamfe_barostat_step(eamfe_ctx* ctx, const eamfe_barostat* b, int64_t step, double w_eam, double* x_dev,
                        double* v_dev, double* mu_host, double* P_host);

/* Current box edges, L_host[n_rep][3] (Angstrom): those of eamfe_system_setup
 * until a barostat move changes them. */
int eamfe_get_boxes(const eamfe_ctx* ctx, double* L_host);

/* Per-atom spring constants for systems of several species (the paper's
 * remark on one spring constant per group of atoms, chosen from each
 * group's mean-squared displacement, Eq. msd): s_dev[N_tot] (device FP64,
 * copied) scales each atom's spring to k s_i, k its replica's spring
 * constant; this enters the spring force, U_E and so dH/dl of the FL,
 * harmonic and Einstein-RS paths.  NULL restores s_i = 1.  The Einstein
 * reference free energy is then the sum of eamfe_einstein_free_energy over
 * the groups, each with its own k s and atom count.  Reset by
 * eamfe_system_setup. */
int eamfe_set_spring_scale(eamfe_ctx* ctx, const double* s_dev);

/* Mean-squared displacement of each replica's atoms at x_dev (device SoA
 * [3][N_tot] FP64) from its lattice sites x0, with the replica's
 * centre-of-mass displacement removed (Eq. msd and the spring-constant
 * choice around it: k = 3 kB T / msd, averaged over an equilibrium run at the
 * size and temperature of the switching runs).  msd[n_rep] is a host array in
 * A^2.  Synchronises. */
int eamfe_msd(eamfe_ctx* ctx, const double* x_dev, double* msd);

/* Spring constant from a mean-squared displacement by equipartition
 * (Eq. msd): k = 3 kB T / msd, msd in A^2 (eamfe_msd, averaged), T in K;
 * returns eV/A^2, or 0 for msd <= 0. */
double eamfe_spring_constant(double msd, double T);

/* Copy the current Verlet rows (for inspection): nnb_dev[N_tot] row lengths,
 * nbr_dev[N_tot][cap] global atom ids in row order, -1 past each row's end
 * (may be NULL; cap >= the row capacity reported by eamfe_list_stats).
 * Device int32 arrays.  Synchronises. */
int eamfe_copy_lists(eamfe_ctx* ctx, int32_t* nnb_dev, int32_t* nbr_dev, int cap);

/* ---- potential --------------------------------------------------------- */

/* Tabulated EAM (the paper's "pair eam" input; Eq. H with U = EAM):
 *   U = sum_i F(rho_i) + 1/2 sum_{i != j} phi(r_ij),  rho_i = sum_{j != i} rho(r_ij),
 * pairs counted only for r < r_cut.  Host knot arrays: phi_knots, rho_knots
 * at r_k = k r_cut/(n_r-1), k = 0..n_r-1; F_knots at rho_k = k rho_max/(n_rho-1).
 * Each function is the natural cubic spline through its knots; outside the
 * table the last cubic piece is continued and EAMFE_ETABLE_RANGE is latched
 * when a density exceeds rho_max.  May be called again to replace the tables.
 * EAMFE_FP32 holds the pair and density-derivative tables in one block's LDS
 * (32 bytes per knot): n_r above the device's LDS per block / 32 (5120 on
 * gfx950) returns EAMFE_EINVAL and keeps the tables the context had.
 * EAMFE_FP64 has no such limit (its kernels copy the tables into LDS only
 * when they fit, else read them from global memory). */
int eam_setup(eamfe_ctx* ctx, int n_r, double r_cut, const double* phi_knots,
              const double* rho_knots, int n_rho, double rho_max, const double* F_knots);

/* ---- system ------------------------------------------------------------ */

/* Describe n_rep replicas (host array, 1 <= n_rep <= 8192) and their lattice
 * sites x0 (device, SoA [3][N_tot], copied).  N_tot = sum n_atoms < 2^28
 * (EAMFE_EINVAL otherwise).  Replaces any previous system. */
int eamfe_system_setup(eamfe_ctx* ctx, int n_rep, const eamfe_replica* reps, const double* x0_dev);

/* Build the Verlet lists at positions x (device SoA) with cutoff r_cut+skin:
 * cell binning with cells of edge >= (r_cut+skin)/2 and a 5 x 5 x 5 cell
 * stencil where a box holds at least five such cells per edge, all-pairs
 * otherwise.  max_neighbors bounds each atom's row
 * (rounded up to a multiple of 32): a row that does not fit is reported as
 * EAMFE_ENEIGH_OVERFLOW.  With max_neighbors = 0 the capacity is estimated
 * from the densest replica and enlarged until every row (and cell bin) of
 * this configuration fits.  EAMFE_EBOX if an edge <= 2(r_cut+skin). */
int neigh_build(eamfe_ctx* ctx, const double* x_dev, double skin, int max_neighbors);

/* ---- evaluation -------------------------------------------------------- */

/* EAM energy and forces at x (device SoA) using the current lists (rebuilt
 * first if any atom moved more than skin/2 since they were built).
 * f_dev: device SoA [3][N_tot] float64 (may be NULL); U_dev: device [n_rep]
 * float64 (may be NULL); e_atom_dev: device [N_tot] per-atom energy
 * F(rho_i) + 1/2 sum_j phi(r_ij) (may be NULL).  A row or cell-bin
 * overflow enlarges the lists and evaluates again.  Synchronises. */
int eam_forces(eamfe_ctx* ctx, const double* x_dev, double* f_dev, double* U_dev, double* e_atom_dev);

/* Initial velocities v = sqrt(kB T / m) z with z from Philox stream 1 at
 * step 0 (one counter per atom id within its replica); with fix_com the
 * replica's mean velocity is removed.  v_dev: device SoA. */
int eamfe_init_velocities(eamfe_ctx* ctx, double* v_dev, int fix_com);

/* Host lambda table of the protocol: lam_host[0..S] (S+1 values), *n_steps = S.
 * lam_host may be NULL to query S. */
int eamfe_lambda_schedule(const eamfe_protocol* p, double* lam_host, int64_t* n_steps);

/* Advance every replica through steps [step_begin, step_end) of the
 * protocol (0 <= step_begin < step_end <= S).  One step s:
 *   W += (l_{s+1} - l_s) dH/dl(x_s)                    (Eq. w_irr, left point)
 *   BAOAB: v += dt/2m F(x_s; l_{s+1}); x += dt/2 v;
 *          v = c1 v + sqrt((1-c1^2) kB T/m) (xi - <xi>); x += dt/2 v;
 *          v += dt/2m F(x_{s+1}; l_{s+1}),   c1 = exp(-dt/damp),
 *   with xi from Philox stream 0 keyed (seed; atom id, step s) and <xi> its
 *   replica mean when fix_com (else 0).
 * x_dev, v_dev: device SoA, updated in place.  The work carried between calls
 * restarts at 0 when step_begin == 0.  Optional device outputs (NULL to skip),
 * indexed by the global step s: dHdl_out[n_rep][S] = dH/dl(x_s),
 * W_out[n_rep][S] = W after step s's increment; lam_out[S+1] = the table.
 * Steps run in chunks (eamfe_set_chunk, default 1000).  For the EAM modes
 * the stream is synchronised after every chunk to read the latched status:
 * a neighbour-row or cell-bin overflow restores the state saved at the
 * chunk's start, enlarges the capacity and replays the chunk (the noise is
 * keyed by step, so the replay is the same trajectory).  With `sync` the
 * call also synchronises at its end and reports any other latched
 * condition. */
int run_switching(eamfe_ctx* ctx, const eamfe_protocol* p, int64_t step_begin, int64_t step_end,
                  double* x_dev, double* v_dev, double* lam_out, double* dHdl_out, double* W_out,
                  int sync);

/* One step s of the protocol (same arithmetic as run_switching) with the
 * work of each replica carried in W_dev[n_rep] (device, in/out) and
 * dH/dl(x_s) written to dHdl_dev[n_rep] (device, may be NULL). */
int switch_step(eamfe_ctx* ctx, const eamfe_protocol* p, int64_t step, double* x_dev, double* v_dev,
                double* W_dev, double* dHdl_dev);

/* Steps per chunk of run_switching (>= 1). */
int eamfe_set_chunk(eamfe_ctx* ctx, int64_t steps);

/* Number of chunk replays after capacity overflows so far. */
int eamfe_replays(const eamfe_ctx* ctx, int64_t* n);

/* Per-replica work after the last stepping call: host W_host[n_rep]. */
int eamfe_get_work(eamfe_ctx* ctx, double* W_host);

/* Checkpoint and resume.  Besides x, v and the step index (the caller's),
 * the state a run carries from one step to the next is each replica's
 * accumulated work and the positions at which the neighbour lists were last
 * built (the noise is a function of seed and step only).  get_state copies
 * the work to W_host[n_rep] (host), those positions to xref_dev (device SoA
 * [3][N_tot] FP64; ESTATE if no lists were built yet) and the lists' skin to
 * *skin; any pointer may be NULL.  set_state, on a context set up with the
 * same potential, replicas and launch shape, loads the work and builds the
 * lists at xref_dev with that skin.  run_switching from the saved step then
 * continues bitwise as the uninterrupted run would (a range starting at step
 * 0 clears the work instead).  Both synchronise. */
int eamfe_get_state(eamfe_ctx* ctx, double* W_host, double* xref_dev, double* skin);
int eamfe_set_state(eamfe_ctx* ctx, const double* W_host, const double* xref_dev, double skin);

/* ---- differentiation --------------------------------------------------- */

/* dU_EAM/dtheta at x, theta = the knot values (phi_k, rho_k, F_k) given to
 * eam_setup (n_r == n_rho required, and 32 (n_r - 1) bytes of histogram must
 * fit one block's LDS: at most 5121 knots on gfx950, else EAMFE_EINVAL
 * before any kernel runs).  U is linear in the phi and F knots and,
 * through rho_i, depends on the rho knots; the kernels bin (1, t, t^2, t^3)
 * of every spline evaluation per interval in 2^-32 fixed point
 * (deterministic), then apply the transpose of the natural-spline map.
 * Pair geometry and spline coordinates are float64 in both numeric forms
 * (in EAMFE_FP32 from the box coordinates); F'(rho_i) and rho_i come from
 * the form's density pass.
 * By Eq. dFdL with theta in the role of lambda, the average of this over the
 * H0 ensemble is dF0/dtheta.
 *   reduce == 0: dtheta_dev[r][f][k] += w[r] dU_r/dtheta_{f,k}   (device, [n_rep][3][n_r])
 *   reduce != 0: dtheta_dev[f][k]    += sum_r w[r] dU_r/dtheta_{f,k}  (device, [3][n_r])
 * f = 0 phi, 1 rho, 2 F.  w_host: host [n_rep] weights or NULL (all 1).
 * The caller zeroes dtheta_dev.  Synchronises. */
int eamfe_adjoint_theta(eamfe_ctx* ctx, const double* x_dev, const double* w_host, int reduce,
                        double* dtheta_dev);

/* eamfe_adjoint_theta for callers that cannot allocate device memory (code
 * under HIP graph capture, tight serving loops, harnesses that forbid it):
 * the same arguments, kernels and results, with the adjoint's per-call
 * scratch (its fixed-point coefficient bins and the knot transform's work
 * rows) in a fixed per-device region inside the library instead of the
 * context's workspace, so the call allocates nothing, also in a context
 * without a caller workspace (where the lists must then already fit: else
 * EAMFE_ENOMEM, nothing allocated).  The region holds 32 MiB:
 *   n_rep * 3 * (n_r - 1) * 32 bytes (rounded up to 256)
 *   + (reduce ? 1 : n_rep) * 3 * 2 * n_r * 8 bytes
 * must fit (116 replicas at 2000 knots with reduce = 0, 174 with
 * reduce = 1); larger calls return EAMFE_EINVAL and do nothing.  Every call
 * on one device uses that device's one region (cleared at each call): calls
 * that overlap in time on one device, from any contexts or streams, race. */
int eamfe_adjoint_theta_noalloc(eamfe_ctx* ctx, const double* x_dev, const double* w_host, int reduce,
                                double* dtheta_dev);

/* Sample dU/dtheta inside run_switching at every `every`-th step whose
 * lambda equals the protocol's start value (the H0 ensemble: lambda = 0 for
 * FL/HH, 1 for RS), accumulating as eamfe_adjoint_theta would into
 * dtheta_dev (device, kept by the caller until sampling is switched off with
 * every = 0).  Resets the sample count.  A run that samples with tables the
 * adjoint cannot take (see eamfe_adjoint_theta) returns EAMFE_EINVAL before
 * any step runs. */
int eamfe_set_adjoint_sampling(eamfe_ctx* ctx, int every, const double* w_host, int reduce, double* dtheta_dev);

/* Samples accumulated since the last eamfe_set_adjoint_sampling. */
int eamfe_adjoint_samples(const eamfe_ctx* ctx, int64_t* n);

/* ---- estimators (host, float64) ---------------------------------------- */

/* Einstein crystal F_E = 3 n_eff kB T ln(hbar w / kB T), w = sqrt(k/m). */
double eamfe_einstein_free_energy(double n_eff, double T, double k, double mass);

/* Fixed centre-of-mass term of Eq. cm: kB T ln[(N/V)(2 pi kB T/(N k))^(3/2)]. */
double eamfe_fixed_cm_correction(double N, double V, double T, double k);

/* Frenkel--Ladd: from n replicas' forward (H0 -> H_E) and backward works,
 * F0 = F_E(n_eff) + (mean W_bwd - mean W_fwd)/2 [+ delta F_CM(N, V, T, k) if add_cm]
 * (Eq. fl with the sign implied by Eq. W12, plus Eq. cm).  n_eff is the
 * number of oscillators of the Einstein crystal, the atom count N: with the
 * centre of mass held in the run (fix_com), Eq. cm alone accounts for the
 * constraint, and F_E(N) + Eq. cm is the free crystal's free energy.
 * Outputs: F0, the dissipation (Eq. Ediss) and the standard error of F0
 * (any may be NULL). */
int eamfe_fl_free_energy(int n, const double* W_fwd, const double* W_bwd, double n_eff, double N,
                         double V, double T, double k, double mass, int add_cm,
                         double* F0, double* E_diss, double* F0_err);

/* Jarzynski's equality (Eq. jarz): dF = -kB T ln(mean_i exp(-W_i / kB T))
 * over n realizations W[n] (host, eV) of one switching leg, taken as a
 * shifted exponential average so no exponential overflows.  dF_err (may be
 * NULL) is the first-order error, kB T s_e / (sqrt(n) e_mean), with e the
 * shifted exponentials and s_e their sample standard deviation (NaN for
 * n = 1).  EAMFE_EINVAL for n < 1, T <= 0 or NULL W. */
int eamfe_jarzynski(int n, const double* W, double T, double* dF, double* dF_err);

/* The works of the two switching legs from cumulative per-step work traces
 * W_trace[n_rep][stride] (host FP64, column s = the work after step s, as
 * run_switching writes them) of protocol p: the forward leg is steps
 * n_eq .. n_eq + n_sw - 1, the backward leg the n_sw steps after the first
 * hold.  W_fwd[r] = W(n_eq + n_sw - 1) - W(n_eq - 1) (the latter 0 when
 * n_eq = 0), W_bwd[r] likewise.  EAMFE_EINVAL if the trace is shorter than
 * the backward leg's end. */
int eamfe_switch_works(const eamfe_protocol* p, int n_rep, const double* W_trace, int64_t stride, double* W_fwd,
                       double* W_bwd);

/* Reversible scaling (Eq. rs): from one replica's cumulative work trace
 * W_trace[S] of an RS protocol and F0(T0), the free energy on n_T
 * temperatures T_grid in [T0, T0/lambda_f]:
 *   F(T) = F0(T0)/l + 3/2 n_eff kB T0 ln(l)/l + (W_{1->l} - W_{l->1})/(2l),  l = T0/T,
 * work between steps interpolated linearly. */
int eamfe_rs_free_energy(const eamfe_protocol* p, const double* W_trace, double F0_T0, double T0,
                         double n_eff, int n_T, const double* T_grid, double* F_out);

/* Eq. rs for a run with the centre of mass held (fix_com), from an F0(T0)
 * of the free crystal (eamfe_fl_free_energy with Eq. cm).  Such a run samples
 * the held system, N atoms with 3(N-1) momenta and the configurational
 * integral at one centre-of-mass position; Eq. rs maps that system's free
 * energy from T0 to T exactly with n_eff = N - 1 in its kinetic term.  The
 * free crystal differs from the held one by
 *   c(T) = -kB T ln(V/N) + 3 kB T ln Lambda(T),  Lambda = sqrt(2 pi hbar^2 / (m kB T)),
 * the convention under which F_E(N) + Eq. cm is the free crystal's value, so
 *   F(T) = rs_{N-1}(F0(T0) - c(T0)) + c(T),
 * rs the map of eamfe_rs_free_energy, N atoms, V the box volume, mass in amu.
 * EAMFE_EINVAL for N <= 1, V <= 0 or mass <= 0, or as eamfe_rs_free_energy. */
int eamfe_rs_free_energy_cm(const eamfe_protocol* p, const double* W_trace, double F0_T0, double T0,
                            double N, double V, double mass, int n_T, const double* T_grid, double* F_out);

#ifdef __cplusplus
}
#endif
#endif /* EAMFE_H */
