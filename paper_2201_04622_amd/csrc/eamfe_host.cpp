// Host side of the C ABI declared in include/eamfe.h: context and buffers,
// spline tables, replica/tile layout, lambda schedules, the stepping loop,
// the free-energy estimators and the barostat's per-replica coupling move.
// All per-atom arithmetic of the MD path runs in the kernels of
// eamfe_kernels.hip (and the rescaling kernel of eamfe_barostat.hip); this
// file only prepares tables, launches, and works on per-replica scalars.
#include "../../include/eamfe.h"
#include "eamfe_internal.h"

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <queue>
#include <string>
#include <vector>

using namespace eamfe;

// Scratch of eamfe_adjoint_theta_noalloc, for callers that cannot allocate:
// the adjoint's fixed-point coefficient bins, then the knot transform's work
// rows.  Each device holds its own copy from the library's load to the end
// of the process; host code reaches it only through the address
// hipGetSymbolAddress returns on that device (g_scratch_ptr), never through
// this name.
constexpr size_t kNoAllocScratchBytes = (size_t)32 << 20;
static __device__ __align__(256) unsigned char scratch[kNoAllocScratchBytes];
constexpr int kMaxDevices = 64;
static void* g_scratch_ptr[kMaxDevices] = {};
static std::mutex g_scratch_mu;

// Device address of this device's scratch (the device is current), once per device.
static int scratch_setup(int device)
{
    if (device < 0 || device >= kMaxDevices) return EAMFE_EDEVICE;
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (g_scratch_ptr[device]) return EAMFE_OK;
    void* p = nullptr;
    if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) return EAMFE_EDEVICE;
    g_scratch_ptr[device] = p;
    return EAMFE_OK;
}

namespace eamfe {
// eamfe_barostat.hip
hipError_t launch_rescale(double* x, double* v, const int32_t* rep_of, const double* mu, int N, hipStream_t s);
hipError_t launch_kinetic(const double* v, const RepDesc* reps, int n_rep, int N, double* out, hipStream_t s);
void barostat_gauss3(uint64_t seed, uint32_t atom, int64_t step, uint32_t stream, double z[3]);
}  // namespace eamfe

struct DevBuf {
    void* p = nullptr;
    size_t bytes = 0;
};

// Sizes that fix the layout of a context's device memory.
struct Shape {
    long N = 0;            // atoms
    long n_rep = 0;        // replicas
    long max_units = 0;    // work units at the finest launch shape (64/16 atoms per unit)
    long max_slices = 0;   // blocks of a staged pair launch, at most
    long n_r = 0, n_rho = 0;
    long cap = 0, n_cells = 0, ccap = 0;
    long lam_len = 0;      // entries of the lambda table
};

// Buffer groups of the arena, in layout order.  A group that changes size
// moves only the groups after it, and those hold contents that are rebuilt
// from host copies (tables, lambda table), rebuilt by the kernels (lists) or
// scratch (adjoint bins).
enum Group : int { G_CORE = 0, G_SYS, G_TAB, G_LIST, G_LAM, G_ADJ, G_COUNT };

struct eamfe_ctx {
    int device = 0;
    hipStream_t stream = nullptr;
    int precision = EAMFE_FP64;
    int deterministic = 1;   // FP32: 2^-32 fixed-point per-atom sums (shape-independent bits)
    int lanes = 4;
    int block = 256;
    int grid = 0;      // persistent pair-kernel blocks (0: every resident slot), a multiple of 8
    int n_cu = 256;
    int max_lds = 65536;   // LDS bytes one block may allocate
    int xcd = 1;
    std::string err;

    // potential
    bool have_pot = false;
    int n_r = 0, n_rho = 0;
    double r_cut = 0.0, rho_max = 0.0;
    std::vector<double> knots_phi, knots_rho, knots_F;
    std::vector<double> c_phi, c_rho, c_F;   // [n-1][4] float64
    DevBuf tab_pair, tab_rho, tab_F;

    // system
    int n_rep = 0;
    int N = 0;
    std::vector<eamfe_replica> reps_in;
    std::vector<RepDesc> reps;
    std::vector<Tile> tiles;   // work units in queue order
    int n_tiles = 0;           // work units
    int nq = 1;                // unit groups (one per XCD with affinity)
    int qoff[9] = {0};         // group q holds tiles[qoff[q] .. qoff[q+1])
    std::vector<int4> slices;  // per block of a staged pair launch: first unit, units, replica's first atom, atoms
    int max_rep_atoms = 0;
    DevBuf slices_d;
    DevBuf reps_d, tiles_d, rep_of_d, x0_d, xref_d, Pa_d, Pb_d, Qa_d, Qb_d, e_emb_d, xi_d;
    DevBuf noise_part_d, energy_part_d, U_rep_d, W_state_d;
    DevBuf iter_d, rebuild_d, flag_pre_d, status_d, row_acc_d, msd_d, kscale_d, vir_d, mu_d;
    bool has_kscale = false;   // per-atom spring scales set

    // neighbour lists
    bool have_list = false;
    double skin = 0.3;
    int cap = 0, ccap = 0, n_cells = 0;
    DevBuf nbr_d, nnb_d, cell_cnt_d, cell_atoms_d, cell_rep_d;
    // rows of replicas that fit one block's LDS come from k_rows_lds
    int lds_rows = 1;                       // 0: every replica through k_bin / k_list
    int n_lds = 0, n_global = 0, lds_atoms = 0, lds_cells = 0, lds_waves = 0;
    DevBuf lds_list_d;                      // [n_rep] those replicas, in order

    // graph replay of the middle iterations (0 = eager launches)
    int graph_iters = 0;
    hipStream_t gstream = nullptr;
    hipEvent_t ev_user = nullptr, ev_graph = nullptr;
    hipGraphExec_t gexec[2] = {nullptr, nullptr};

    // optional per-launch timing with HIP events on the context's stream
    int timing = 0;          // sample every timing-th iteration (0 = off)
    int timing_kinds = 7;    // kernels timed: bit 0 density, bit 1 force, bit 2 list rebuild
    int64_t timing_seen = 0; // iterations run since timing was switched on
    bool timing_now = false; // current iteration is sampled
    std::vector<hipEvent_t> ev_pool;
    size_t ev_used = 0;
    std::vector<int> ev_kind;   // 0 density, 1 force, 2 neighbour rebuild (one entry per event pair)

    // list statistics
    DevBuf stats_d;

    // autotuner scratch state
    DevBuf tune_x, tune_v, tune_w;

    // chunked stepping: checkpoint of (x, v, W) for replay after a list overflow
    int64_t chunk = 1000;
    int min_ccap = 0;
    int64_t replays = 0;
    DevBuf snap_P, snap_Q, snap_v, snap_w, snap_rows;

    // adjoint: densities, fixed-point bins, finish scratch, weights
    DevBuf rho_d, bins_d, adj_scratch_d, adj_w_d;
    // sampling of dU/dtheta inside run_switching (0 = off)
    int adj_every = 0;
    int adj_reduce = 0;
    double* adj_out = nullptr;
    std::vector<double> adj_w;
    int64_t adj_samples = 0;

    // lambda table
    DevBuf lam_d;

    // device memory: one arena holding every buffer above, laid out by `shape`
    Shape shape;
    char* arena = nullptr;
    size_t arena_bytes = 0;
    bool caller_ws = false;     // the arena is the caller's (eamfe_set_workspace): never allocate
    size_t need = 0;            // bytes the last call that ran out of workspace needed
    int64_t resume_step = -1;   // where an interrupted run_switching stopped (-1: none)
    int64_t device_allocs = 0;  // hipMalloc calls made by the library
    bool no_alloc = false;      // inside a call that must not allocate (as with a caller's workspace)
    long cap_min = 0;           // row capacity asked for after an overflow (kept across re-plans)

    long n_atoms_total() const { return N; }
    std::vector<double> lam_h;
    eamfe_protocol lam_key{};
    bool lam_valid = false;
};

namespace {

int fail(eamfe_ctx* c, int code, const std::string& msg)
{
    if (c) c->err = msg;
    return code;
}

#define HIPCHK(ctx, expr)                                                                      \
    do {                                                                                       \
        hipError_t e_ = (expr);                                                                \
        if (e_ != hipSuccess)                                                                  \
            return fail(ctx, e_ == hipErrorOutOfMemory ? EAMFE_ENOMEM : EAMFE_EDEVICE,        \
                        std::string(#expr) + ": " + hipGetErrorString(e_));                    \
    } while (0)

#define LCHK(ctx, expr)                                                                        \
    do {                                                                                       \
        int e_ = (expr);                                                                       \
        if (e_ != 0)                                                                           \
            return fail(ctx, EAMFE_EDEVICE, std::string(#expr) + ": " +                        \
                                                hipGetErrorString((hipError_t)e_));            \
    } while (0)

#define OK(expr)                        \
    do {                                \
        int r_ = (expr);                \
        if (r_ != EAMFE_OK) return r_;  \
    } while (0)

constexpr size_t kAlign = 256;

size_t align_up(size_t b) { return (b + kAlign - 1) / kAlign * kAlign; }

// Every device buffer of a context with the group it belongs to and its size
// under shape s, in layout order.
template <typename F>
void for_regions(eamfe_ctx* c, const Shape& s, F&& f)
{
    const size_t N = (size_t)s.N, R = (size_t)s.n_rep, U = (size_t)s.max_units, d = sizeof(double);
    const size_t real = c->precision == EAMFE_FP32 ? 4 : 8;
    if (N || s.n_r) {
        f(c->status_d, G_CORE, sizeof(int32_t));
        f(c->iter_d, G_CORE, sizeof(int64_t));
        f(c->stats_d, G_CORE, 2 * sizeof(unsigned long long));
    }
    if (N) {
        f(c->reps_d, G_SYS, R * sizeof(RepDesc));
        f(c->tiles_d, G_SYS, U * sizeof(Tile));
        f(c->slices_d, G_SYS, (size_t)s.max_slices * sizeof(int4));
        f(c->noise_part_d, G_SYS, U * 3 * d);
        f(c->energy_part_d, G_SYS, U * 3 * d);
        f(c->vir_d, G_SYS, U * 3 * d);
        f(c->rep_of_d, G_SYS, N * sizeof(int32_t));
        f(c->x0_d, G_SYS, 3 * N * d);
        f(c->xref_d, G_SYS, 3 * N * d);
        f(c->Pa_d, G_SYS, N * sizeof(double4));
        f(c->Pb_d, G_SYS, N * sizeof(double4));
        f(c->Qa_d, G_SYS, N * sizeof(uint4));
        f(c->Qb_d, G_SYS, N * sizeof(uint4));
        f(c->e_emb_d, G_SYS, N * d);
        f(c->xi_d, G_SYS, 3 * N * d);
        f(c->rho_d, G_SYS, N * d);
        f(c->kscale_d, G_SYS, N * d);
        f(c->U_rep_d, G_SYS, 2 * R * d);
        f(c->W_state_d, G_SYS, R * d);
        f(c->rebuild_d, G_SYS, R * sizeof(int32_t));
        f(c->flag_pre_d, G_SYS, (2 * R + 2) * sizeof(int32_t));
        f(c->row_acc_d, G_SYS, (R + 3) * d);
        f(c->msd_d, G_SYS, R * d);
        f(c->mu_d, G_SYS, 3 * R * d);
        f(c->adj_w_d, G_SYS, R * d);
        f(c->lds_list_d, G_SYS, R * sizeof(int32_t));
        f(c->tune_x, G_SYS, 3 * N * d);
        f(c->tune_v, G_SYS, 3 * N * d);
        f(c->tune_w, G_SYS, R * d);
        f(c->snap_P, G_SYS, N * sizeof(double4));
        f(c->snap_Q, G_SYS, N * sizeof(uint4));
        f(c->snap_v, G_SYS, 3 * N * d);
        f(c->snap_w, G_SYS, R * d);
        f(c->snap_rows, G_SYS, (R + 3) * d);
    }
    if (s.n_r) {
        f(c->tab_pair, G_TAB, 8 * (size_t)(s.n_r - 1) * real);
        f(c->tab_rho, G_TAB, 4 * (size_t)(s.n_r - 1) * real);
        f(c->tab_F, G_TAB, 4 * (size_t)(s.n_rho - 1) * real);
    }
    if (N && s.cap) {
        const size_t nc = (size_t)std::max(1L, s.n_cells);
        f(c->nbr_d, G_LIST, N * (size_t)s.cap * sizeof(int32_t));
        f(c->nnb_d, G_LIST, N * sizeof(int32_t));
        f(c->cell_cnt_d, G_LIST, nc * sizeof(int32_t));
        f(c->cell_atoms_d, G_LIST, nc * (size_t)s.ccap * sizeof(int32_t));
        f(c->cell_rep_d, G_LIST, nc * sizeof(int32_t));
    }
    if (s.lam_len) f(c->lam_d, G_LAM, (size_t)s.lam_len * d);
    if (N && s.n_r) {
        const size_t nb = (size_t)std::max(s.n_r, s.n_rho) - 1;
        f(c->bins_d, G_ADJ, R * 3 * nb * 4 * sizeof(unsigned long long));
        f(c->adj_scratch_d, G_ADJ, R * 3 * 2 * (nb + 1) * d);
    }
}

size_t layout_bytes(eamfe_ctx* c, const Shape& s)
{
    size_t off = 0;
    for_regions(c, s, [&](DevBuf&, int, size_t b) { off += align_up(b); });
    return off;
}

int upload_tables(eamfe_ctx* c);   // below
void drop_graphs(eamfe_ctx* c);     // below

// Make the arena hold the layout of shape s and point every buffer into it.
// Contents keep their offsets when the arena is replaced (the live layout is
// copied over); groups whose offset changes are rebuilt here (tables and the
// lambda table from their host copies) or by their owners (lists are planned
// and rebuilt by the caller that changed a group before them; adjoint bins
// are scratch).  With a caller's workspace that is too small nothing
// changes: EAMFE_ENOMEM, and `need` holds the bytes required.
int bind(eamfe_ctx* c, const Shape& s)
{
    const size_t need = layout_bytes(c, s);
    HIPCHK(c, hipStreamSynchronize(c->stream));   // no pass in flight uses the old layout
    if (need > c->arena_bytes) {
        if (c->caller_ws || c->no_alloc) {
            c->need = need;
            return fail(c, EAMFE_ENOMEM, "workspace of " + std::to_string(c->arena_bytes) + " bytes is too small: " +
                                             std::to_string(need) + " needed (eamfe_workspace_bytes)");
        }
        const size_t grow = need + need / 4;
        void* p = nullptr;
        ++c->device_allocs;
        const hipError_t e = hipMalloc(&p, grow);
        if (e != hipSuccess) return fail(c, EAMFE_ENOMEM, std::string("hipMalloc: ") + hipGetErrorString(e));
        if (c->arena) {
            const size_t used = layout_bytes(c, c->shape);
            HIPCHK(c, hipMemcpy(p, c->arena, used, hipMemcpyDeviceToDevice));
            (void)hipFree(c->arena);
        }
        c->arena = (char*)p;
        c->arena_bytes = grow;
    }
    size_t old_off[G_COUNT], new_off[G_COUNT], old_len[G_COUNT], new_len[G_COUNT];
    for (int g = 0; g < G_COUNT; ++g) old_off[g] = new_off[g] = old_len[g] = new_len[g] = 0;
    {
        size_t off = 0;
        int last = -1;
        for_regions(c, c->shape, [&](DevBuf&, int g, size_t b) {
            if (g != last) old_off[g] = off, last = g;
            old_len[g] += align_up(b);
            off += align_up(b);
        });
        off = 0;
        last = -1;
        for_regions(c, s, [&](DevBuf& buf, int g, size_t b) {
            if (g != last) new_off[g] = off, last = g;
            new_len[g] += align_up(b);
            buf.p = c->arena + off;
            buf.bytes = b;
            off += align_up(b);
        });
    }
    const Shape old = c->shape;
    c->shape = s;
    c->need = 0;
    drop_graphs(c);   // captured launches hold buffer addresses
    if (new_len[G_CORE] && !old_len[G_CORE]) HIPCHK(c, hipMemset(c->status_d.p, 0, new_len[G_CORE]));
    const bool tab_moved = old_off[G_TAB] != new_off[G_TAB] || old_len[G_TAB] != new_len[G_TAB];
    const bool lam_moved = old_off[G_LAM] != new_off[G_LAM] || old_len[G_LAM] != new_len[G_LAM];
    if (tab_moved && c->have_pot && s.n_r == old.n_r && s.n_rho == old.n_rho) OK(upload_tables(c));
    if (lam_moved && c->lam_valid && s.lam_len == old.lam_len)
        HIPCHK(c, hipMemcpy(c->lam_d.p, c->lam_h.data(), c->lam_h.size() * sizeof(double), hipMemcpyHostToDevice));
    return EAMFE_OK;
}


// Natural cubic spline on x_k = k h through y[0..n-1] -> [n-1][4] (a, b, c, d)
// with s(t) = a + t(b + t(c + t d)) on interval m, t = x/h - m.  The second
// derivatives solve the tridiagonal system M_{k-1} + 4 M_k + M_{k+1} =
// 6 (y_{k+1} - 2 y_k + y_{k-1}) / h^2 with M_0 = M_{n-1} = 0 (natural ends).
std::vector<double> natural_spline(const double* y, int n, double h)
{
    std::vector<double> M(n, 0.0), diag(n, 4.0), rhs(n, 0.0);
    for (int k = 1; k < n - 1; ++k) rhs[k] = 6.0 * (y[k + 1] - 2.0 * y[k] + y[k - 1]) / (h * h);
    // forward elimination (unit off-diagonals)
    for (int k = 2; k < n - 1; ++k) {
        const double w = 1.0 / diag[k - 1];
        diag[k] -= w;
        rhs[k] -= w * rhs[k - 1];
    }
    for (int k = n - 2; k >= 1; --k) M[k] = (rhs[k] - (k + 1 < n - 1 ? M[k + 1] : 0.0)) / diag[k];
    std::vector<double> c(4 * (size_t)(n - 1));
    for (int m = 0; m < n - 1; ++m) {
        c[4 * m + 0] = y[m];
        c[4 * m + 1] = (y[m + 1] - y[m]) - h * h * (2.0 * M[m] + M[m + 1]) / 6.0;
        c[4 * m + 2] = 0.5 * h * h * M[m];
        c[4 * m + 3] = h * h * (M[m + 1] - M[m]) / 6.0;
    }
    return c;
}

template <typename real>
int upload_tables_t(eamfe_ctx* c)
{
    const int mr = c->n_r - 1, mf = c->n_rho - 1;
    const double inv_h = (c->n_r - 1) / c->r_cut;
    std::vector<real> pair(8 * (size_t)mr), rho(4 * (size_t)mr), F(4 * (size_t)mf);
    for (int m = 0; m < mr; ++m) {
        for (int q = 0; q < 4; ++q) pair[8 * m + q] = (real)c->c_phi[4 * m + q];
        pair[8 * m + 4] = (real)(c->c_rho[4 * m + 1] * inv_h);
        pair[8 * m + 5] = (real)(2.0 * c->c_rho[4 * m + 2] * inv_h);
        pair[8 * m + 6] = (real)(3.0 * c->c_rho[4 * m + 3] * inv_h);
        pair[8 * m + 7] = (real)0;
        for (int q = 0; q < 4; ++q) rho[4 * m + q] = (real)c->c_rho[4 * m + q];
    }
    for (int m = 0; m < mf; ++m)
        for (int q = 0; q < 4; ++q) F[4 * m + q] = (real)c->c_F[4 * m + q];
    HIPCHK(c, hipMemcpy(c->tab_pair.p, pair.data(), pair.size() * sizeof(real), hipMemcpyHostToDevice));
    HIPCHK(c, hipMemcpy(c->tab_rho.p, rho.data(), rho.size() * sizeof(real), hipMemcpyHostToDevice));
    HIPCHK(c, hipMemcpy(c->tab_F.p, F.data(), F.size() * sizeof(real), hipMemcpyHostToDevice));
    return EAMFE_OK;
}

int upload_tables(eamfe_ctx* c)
{
    return c->precision == EAMFE_FP32 ? upload_tables_t<float>(c) : upload_tables_t<double>(c);
}

Tables tables_of(const eamfe_ctx* c)
{
    Tables t{};
    t.pair = c->tab_pair.p;
    t.rho = c->tab_rho.p;
    t.F = c->tab_F.p;
    t.n_r = c->n_r;
    t.n_rho = c->n_rho;
    t.r_cut = c->r_cut;
    t.rc2 = c->r_cut * c->r_cut;
    t.inv_h_r = (c->n_r - 1) / c->r_cut;
    t.inv_h_rho = (c->n_rho - 1) / c->rho_max;
    t.rho_max = c->rho_max;
    return t;
}

// Work-unit table for the current launch shape: every replica is cut into
// units of 64/lanes atoms (one wavefront's atoms), in replica-major order
// (consecutive wavefronts of a block share a replica's neighbourhoods in the
// CU's caches); unit slots (tile_base) follow the replica index.  With XCD affinity (and at least 8 replicas) replicas
// are binned greedily by atom count into 8 groups (group x is spread over the
// blocks on XCD x); otherwise one group.
// Blocks of the staged pair launches (each stages one replica's records in
// LDS): every replica of a unit group gets at least one block and the
// group's n_cu / nq blocks go to the replicas with the largest slices, whose
// units are then split into near-equal contiguous runs.  Block b serves
// group b % nq, so a replica's blocks share an XCD (and its L2) as its units
// do in the persistent form.
void build_slices(eamfe_ctx* c)
{
    std::vector<std::vector<int2>> per_group(c->nq);
    size_t most = 0;
    for (int x = 0; x < c->nq; ++x) {
        // the group's replicas: runs of units with one replica each
        std::vector<int2> runs;   // first unit, units
        for (int u = c->qoff[x]; u < c->qoff[x + 1];) {
            int e = u;
            while (e < c->qoff[x + 1] && c->tiles[e].rep == c->tiles[u].rep) ++e;
            runs.push_back(make_int2(u, e - u));
            u = e;
        }
        const int target = std::max((int)runs.size(), c->n_cu / c->nq);
        std::vector<int> nb(runs.size(), 1);
        // largest slice first: a max-heap of (units per block, run)
        std::priority_queue<std::pair<double, int>> heap;
        for (size_t k = 0; k < runs.size(); ++k) heap.push({(double)runs[k].y, (int)k});
        for (int left = target - (int)runs.size(); left > 0 && !heap.empty(); --left) {
            const int k = heap.top().second;
            heap.pop();
            if (nb[k] >= runs[k].y) continue;   // one unit per block at most
            ++nb[k];
            heap.push({(double)runs[k].y / nb[k], k});
        }
        for (size_t k = 0; k < runs.size(); ++k) {
            const int n = runs[k].y, m = nb[k];
            for (int j = 0, at = runs[k].x; j < m; ++j) {
                const int len = n / m + (j < n % m ? 1 : 0);
                per_group[x].push_back(make_int2(at, len));
                at += len;
            }
        }
        most = std::max(most, per_group[x].size());
    }
    c->slices.assign(most * c->nq, make_int4(0, 0, 0, 0));
    for (int x = 0; x < c->nq; ++x)
        for (size_t k = 0; k < per_group[x].size(); ++k) {
            const int2 u = per_group[x][k];
            const RepDesc& R = c->reps[c->tiles[u.x].rep];
            c->slices[k * c->nq + x] = make_int4(u.x, u.y, R.off, R.n);
        }
}

int build_tiles(eamfe_ctx* c)
{
    const int A = 64 / c->lanes;
    c->tiles.clear();
    std::vector<std::vector<Tile>> per(c->n_rep);
    int base = 0;
    for (int r = 0; r < c->n_rep; ++r) {
        RepDesc& R = c->reps[r];
        R.n_tiles = (R.n + A - 1) / A;
        R.tile_base = base;
        base += R.n_tiles;
        for (int t = 0; t < R.n_tiles; ++t) {
            Tile tl;
            tl.rep = r;
            tl.first = R.off + t * A;
            tl.count = std::min(A, R.n - t * A);
            tl.idx = t;
            per[r].push_back(tl);
        }
    }
    c->n_tiles = base;
    c->max_rep_atoms = 0;
    for (const auto& R : c->reps) c->max_rep_atoms = std::max(c->max_rep_atoms, R.n);
    for (int q = 0; q < 9; ++q) c->qoff[q] = 0;
    if (c->xcd && c->n_rep >= 8) {
        std::vector<int> order(c->n_rep);
        for (int r = 0; r < c->n_rep; ++r) order[r] = r;
        std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return c->reps[a].n > c->reps[b].n; });
        std::vector<long> load(8, 0);
        std::vector<std::vector<int>> bins(8);
        for (int r : order) {
            const int x = (int)(std::min_element(load.begin(), load.end()) - load.begin());
            load[x] += c->reps[r].n;
            bins[x].push_back(r);
        }
        for (int x = 0; x < 8; ++x) {
            std::sort(bins[x].begin(), bins[x].end());
            for (int r : bins[x]) c->tiles.insert(c->tiles.end(), per[r].begin(), per[r].end());
            c->qoff[x + 1] = (int)c->tiles.size();
        }
        c->nq = 8;
    } else {
        for (auto& v : per) c->tiles.insert(c->tiles.end(), v.begin(), v.end());
        c->qoff[1] = (int)c->tiles.size();
        c->nq = 1;
    }
    if ((long)c->tiles.size() > c->shape.max_units) return fail(c, EAMFE_EINVAL, "internal: unit table overflow");
    if (!c->tiles.empty())
        HIPCHK(c, hipMemcpy(c->tiles_d.p, c->tiles.data(), c->tiles.size() * sizeof(Tile), hipMemcpyHostToDevice));
    build_slices(c);
    if ((long)c->slices.size() > c->shape.max_slices) return fail(c, EAMFE_EINVAL, "internal: slice table overflow");
    if (!c->slices.empty())
        HIPCHK(c, hipMemcpy(c->slices_d.p, c->slices.data(), c->slices.size() * sizeof(int4), hipMemcpyHostToDevice));
    HIPCHK(c, hipMemcpy(c->reps_d.p, c->reps.data(), c->reps.size() * sizeof(RepDesc), hipMemcpyHostToDevice));
    return EAMFE_OK;
}

int upload_reps(eamfe_ctx* c)
{
    HIPCHK(c, hipMemcpyAsync(c->reps_d.p, c->reps.data(), c->reps.size() * sizeof(RepDesc), hipMemcpyHostToDevice,
                             c->stream));
    // the host vector may change before the copy runs: wait for it
    HIPCHK(c, hipStreamSynchronize(c->stream));
    return EAMFE_OK;
}

double4* PA(eamfe_ctx* c) { return (double4*)c->Pa_d.p; }
double4* PB(eamfe_ctx* c) { return (double4*)c->Pb_d.p; }
uint4* QA(eamfe_ctx* c) { return (uint4*)c->Qa_d.p; }
uint4* QB(eamfe_ctx* c) { return (uint4*)c->Qb_d.p; }
uint4* Q_of(eamfe_ctx* c, const double4* P) { return P == PA(c) ? QA(c) : QB(c); }

NeighArgs neigh_args(eamfe_ctx* c, const double4* P)
{
    NeighArgs a{};
    a.tiles = (const Tile*)c->tiles_d.p;
    a.reps = (const RepDesc*)c->reps_d.p;
    a.rep_of = (const int32_t*)c->rep_of_d.p;
    a.cell_rep = (const int32_t*)c->cell_rep_d.p;
    a.P = P;
    a.Q = Q_of(c, P);
    a.n_rep = c->n_rep;
    a.xref = (double*)c->xref_d.p;
    a.cell_cnt = (int32_t*)c->cell_cnt_d.p;
    a.cell_atoms = (int32_t*)c->cell_atoms_d.p;
    a.nbr = (int32_t*)c->nbr_d.p;
    a.nnb = (int32_t*)c->nnb_d.p;
    a.rebuild = (int32_t*)c->rebuild_d.p;
    a.flag_pre = (int32_t*)c->flag_pre_d.p;
    a.status = (int32_t*)c->status_d.p;
    a.N = c->N;
    a.n_cells = c->n_cells;
    a.ccap = c->ccap;
    a.cap = c->cap;
    a.chunk = std::max(512, c->ccap);
    a.rl2 = (c->r_cut + c->skin) * (c->r_cut + c->skin);
    {
        // candidate test in single precision on folded coordinates: widen the
        // radius by far more than its rounding so no pair within r_cut + skin is lost
        double Lmax = 0.0;
        for (const auto& R : c->reps) Lmax = std::max({Lmax, R.L[0], R.L[1], R.L[2]});
        const double margin = std::max(1e-3, 64.0 * Lmax * 1.2e-7);
        a.rl2_f = (float)((c->r_cut + c->skin + margin) * (c->r_cut + c->skin + margin));
    }
    a.half_skin2 = 0.25 * c->skin * c->skin;
    a.lds_list = (const int32_t*)c->lds_list_d.p;
    a.n_lds = c->n_lds;
    a.n_global = c->n_global;
    a.lds_atoms = c->lds_atoms;
    a.lds_cells = c->lds_cells;
    a.lds_waves = c->lds_waves;
    a.lds_grid = c->n_cu;
    return a;
}

StepArgs step_args(eamfe_ctx* c)
{
    StepArgs a{};
    a.tiles = (const Tile*)c->tiles_d.p;
    a.reps = (const RepDesc*)c->reps_d.p;
    a.x0 = (const double*)c->x0_d.p;
    a.kscale = c->has_kscale ? (const double*)c->kscale_d.p : nullptr;
    a.xref = (const double*)c->xref_d.p;
    a.nbr = (const int32_t*)c->nbr_d.p;
    a.nnb = (const int32_t*)c->nnb_d.p;
    a.cap = c->cap;
    a.e_emb = (double*)c->e_emb_d.p;
    a.xi = (double*)c->xi_d.p;
    a.noise_part = (double*)c->noise_part_d.p;
    a.energy_part = (double*)c->energy_part_d.p;
    a.U_rep = (double*)c->U_rep_d.p;
    a.rebuild = (int32_t*)c->rebuild_d.p;
    a.cell_cnt = (int32_t*)c->cell_cnt_d.p;
    a.flag_pre = (int32_t*)c->flag_pre_d.p;
    a.row_acc = (double*)c->row_acc_d.p;
    a.status = (int32_t*)c->status_d.p;
    a.iter = (int64_t*)c->iter_d.p;
    a.W_state = (double*)c->W_state_d.p;
    a.tab = tables_of(c);
    a.N = c->N;
    a.n_tiles = c->n_tiles;
    a.n_rep = c->n_rep;
    a.grid_blocks = c->grid;
    a.n_cu = c->n_cu;
    a.nq = c->nq;
    for (int q = 0; q < 9; ++q) a.qoff[q] = c->qoff[q];
    // FP32 form: stage each block's replica records in LDS when they fit
    // beside the pair table (and no persistent grid was asked for)
    a.slices = (const int4*)c->slices_d.p;
    a.stage_atoms = c->max_rep_atoms;
    const long lds_force = 32L * c->n_r + 16L * c->max_rep_atoms;
    a.slice_grid = (c->precision == EAMFE_FP32 && c->have_pot && c->grid == 0 && lds_force <= c->max_lds)
                       ? (int)c->slices.size()
                       : 0;
    a.half_skin2 = 0.25 * c->skin * c->skin;
    a.fix = c->deterministic && c->precision == EAMFE_FP32;
    return a;
}

// Neighbour-list geometry for the current system and skin.  max_neighbors
// > 0 fixes the row capacity (rounded up to a multiple of 32); 0 takes an
// estimate from the densest replica, at least the capacity an earlier
// overflow asked for (cap_min).  Nothing changes if the lists do not fit the
// workspace.
int plan_lists(eamfe_ctx* c, double skin, int max_neighbors)
{
    const double rl = c->r_cut + skin;
    double dens_max = 0.0, cellvol_max = 0.0;
    int n_cells = 0;
    std::vector<int32_t> cell_rep;
    std::vector<RepDesc> reps = c->reps;
    for (int r = 0; r < c->n_rep; ++r) {
        const RepDesc& R = reps[r];
        for (int d = 0; d < 3; ++d)
            if (!(R.L[d] > 2.0 * rl))
                return fail(c, EAMFE_EBOX, "box edge " + std::to_string(R.L[d]) + " of replica " +
                                               std::to_string(r) + " is not larger than 2 (r_cut + skin)");
    }
    // cells of edge >= rl / 2: a 5 x 5 x 5 stencil holds every pair within rl,
    // and five or more cells per edge keep its cells distinct; replicas small
    // enough for one block's LDS (allow_lds) get their rows from k_rows_lds
    // and no global cells
    auto classify = [&](bool allow_lds) {
        dens_max = cellvol_max = 0.0;
        n_cells = 0;
        cell_rep.clear();
        for (int r = 0; r < c->n_rep; ++r) {
            RepDesc& R = reps[r];
            const double V = R.L[0] * R.L[1] * R.L[2];
            dens_max = std::max(dens_max, R.n / V);
            int nc[3];
            bool cells = true;
            for (int d = 0; d < 3; ++d) {
                nc[d] = (int)std::floor(2.0 * R.L[d] / rl);
                if (nc[d] < 5) cells = false;
            }
            for (int d = 0; d < 3; ++d) R.nc[d] = cells ? nc[d] : 0;
            R.lds = allow_lds && R.n <= kRowsAtomsMax && (long)R.nc[0] * R.nc[1] * R.nc[2] <= kRowsCellsMax;
            R.cell_base = n_cells;
            if (cells && !R.lds) {
                const int k = nc[0] * nc[1] * nc[2];
                for (int q = 0; q < k; ++q) cell_rep.push_back(r);
                n_cells += k;
                cellvol_max = std::max(cellvol_max, V / k * (R.n / V));
            }
        }
    };
    classify(c->lds_rows != 0);
    // mean occupancy of the fullest cells, with room for clustering (set below, after the builders are chosen)
    int ccap = 0;
    int cap;
    if (max_neighbors > 0) {
        cap = (max_neighbors + 31) / 32 * 32;   // rows are read four slots at a time, 16-byte aligned
    } else {
        const double nmean = 4.0 / 3.0 * M_PI * rl * rl * rl * dens_max;
        cap = std::max((int)(std::ceil((nmean * 2.0 + 32.0) / 32.0) * 32.0), (int)c->cap_min);
    }
    // the LDS builder's block: records, ids and cell starts of its largest
    // replica and a row buffer per wavefront; as many wavefronts as fit
    int lds_atoms = 0, lds_cells = 0, lds_waves = 0;
    for (const RepDesc& R : reps)
        if (R.lds) {
            lds_atoms = std::max(lds_atoms, R.n);
            lds_cells = std::max(lds_cells, R.nc[0] * R.nc[1] * R.nc[2]);
        }
    if (lds_atoms)
        for (int wv : {16, 8, 4})
            if (rows_lds_bytes(lds_atoms, lds_cells, cap, wv) + 1024 <= (size_t)c->max_lds) {   // + static shared words
                lds_waves = wv;
                break;
            }
    if (lds_atoms && !lds_waves) {   // not even four wavefronts fit: every replica through k_bin / k_list
        classify(false);
        lds_atoms = lds_cells = 0;
    }
    std::vector<int32_t> lds_list;
    for (int r = 0; r < c->n_rep; ++r)
        if (reps[r].lds) lds_list.push_back(r);
    ccap = std::max({32, c->min_ccap, (int)(std::ceil(cellvol_max * 4.0 / 32.0) * 32.0) + 32});
    Shape s2 = c->shape;
    s2.cap = cap;
    s2.n_cells = n_cells;
    s2.ccap = ccap;
    OK(bind(c, s2));
    c->n_lds = (int)lds_list.size();
    c->n_global = c->n_rep - c->n_lds;
    c->lds_atoms = lds_atoms;
    c->lds_cells = lds_cells;
    c->lds_waves = lds_waves;
    if (!lds_list.empty())
        HIPCHK(c, hipMemcpy(c->lds_list_d.p, lds_list.data(), lds_list.size() * sizeof(int32_t),
                            hipMemcpyHostToDevice));
    c->reps = reps;
    c->ccap = ccap;
    c->cap = cap;
    c->n_cells = n_cells;
    c->skin = skin;
    HIPCHK(c, hipMemsetAsync(c->cell_cnt_d.p, 0, (size_t)std::max(1, n_cells) * sizeof(int32_t), c->stream));
    HIPCHK(c, hipMemsetAsync(c->nnb_d.p, 0, (size_t)c->N * sizeof(int32_t), c->stream));
    if (n_cells)
        HIPCHK(c, hipMemcpy(c->cell_rep_d.p, cell_rep.data(), cell_rep.size() * sizeof(int32_t),
                            hipMemcpyHostToDevice));
    OK(upload_reps(c));
    return EAMFE_OK;
}

// Row or bin overflow seen (status bits st): ask for larger rows or bins and
// plan the lists again (EAMFE_ENOMEM if they do not fit the workspace).
int grow_lists(eamfe_ctx* c, int st)
{
    const int new_cap = (st & ST_NEIGH_OVERFLOW) ? (int)(std::ceil(c->cap * 1.5 / 32.0) * 32.0) : c->cap;
    if (st & ST_CELL_OVERFLOW) c->min_ccap = (int)(std::ceil(c->ccap * 1.5 / 32.0) * 32.0);
    c->cap_min = std::max<long>(c->cap_min, new_cap);
    return plan_lists(c, c->skin, new_cap);
}

int status_code(int st)
{
    if (st & ST_NEIGH_OVERFLOW) return EAMFE_ENEIGH_OVERFLOW;
    if (st & ST_CELL_OVERFLOW) return EAMFE_ECELL_OVERFLOW;
    if (st & ST_NONFINITE) return EAMFE_ENONFINITE;
    if (st & ST_TABLE_RANGE) return EAMFE_ETABLE_RANGE;
    return EAMFE_OK;
}

int read_status(eamfe_ctx* c)
{
    HIPCHK(c, hipStreamSynchronize(c->stream));
    if (!c->status_d.p) return EAMFE_OK;   // no device state yet
    int st = 0;
    HIPCHK(c, hipMemcpy(&st, c->status_d.p, sizeof(int), hipMemcpyDeviceToHost));
    if (st) {
        HIPCHK(c, hipMemset(c->status_d.p, 0, sizeof(int)));
        const int code = status_code(st);
        const char* what = code == EAMFE_ENEIGH_OVERFLOW ? "neighbour row overflow (raise max_neighbors)"
                           : code == EAMFE_ECELL_OVERFLOW ? "cell bin overflow"
                           : code == EAMFE_ENONFINITE     ? "non-finite position, force or energy"
                                                          : "density beyond rho_max";
        return fail(c, code, what);
    }
    return EAMFE_OK;
}

__global__ void k_set_i64(int64_t* p, int64_t v) { *p = v; }

int set_iter(eamfe_ctx* c, int64_t v)
{
    hipLaunchKernelGGL(k_set_i64, dim3(1), dim3(1), 0, c->stream, (int64_t*)c->iter_d.p, v);
    HIPCHK(c, hipGetLastError());
    return EAMFE_OK;
}

__global__ void k_fill_i32(int32_t* p, int n, int32_t v)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = v;
}

int set_rebuild_all(eamfe_ctx* c)
{
    hipLaunchKernelGGL(k_fill_i32, dim3((c->n_rep + 255) / 256), dim3(256), 0, c->stream, (int32_t*)c->rebuild_d.p,
                       c->n_rep, 1);
    HIPCHK(c, hipGetLastError());
    return EAMFE_OK;
}

bool proto_equal(const eamfe_protocol& a, const eamfe_protocol& b)
{
    return a.mode == b.mode && a.function == b.function && a.n_eq == b.n_eq && a.n_sw == b.n_sw &&
           a.n_hold == b.n_hold && a.n_hold2 == b.n_hold2 && a.lambda_f == b.lambda_f;
}

double lambda_fl(int function, double tau)
{
    if (function == 1) return tau;
    // 9th-order smooth step with zero slope at both ends (Sec. fl_lammps, function 2)
    const double t2 = tau * tau, t4 = t2 * t2, t5 = t4 * tau;
    return t5 * (126.0 + tau * (-420.0 + tau * (540.0 + tau * (-315.0 + tau * 70.0))));
}

double lambda_rs(double lf, double tau) { return 1.0 / (1.0 + tau * (1.0 / lf - 1.0)); }

int check_protocol(const eamfe_protocol* p)
{
    if (!p) return EAMFE_EINVAL;
    if (p->mode < 0 || p->mode > 3) return EAMFE_EINVAL;
    if (p->n_eq < 0 || p->n_sw < 1 || p->n_hold < 0 || p->n_hold2 < 0) return EAMFE_EINVAL;
    if ((p->mode == EAMFE_MODE_FL || p->mode == EAMFE_MODE_HH) && p->function != 1 && p->function != 2)
        return EAMFE_EINVAL;
    if ((p->mode == EAMFE_MODE_RS || p->mode == EAMFE_MODE_EIN_RS) && !(p->lambda_f > 0.0)) return EAMFE_EINVAL;
    if (!(p->dt > 0.0) || p->damp < 0.0) return EAMFE_EINVAL;
    return EAMFE_OK;
}

int ensure_lambda(eamfe_ctx* c, const eamfe_protocol* p, int64_t* S_out)
{
    int64_t S = 0;
    OK(eamfe_lambda_schedule(p, nullptr, &S));
    if (!c->lam_valid || !proto_equal(c->lam_key, *p)) {
        if (S + 1 > c->shape.lam_len) {   // a longer table than any before: a larger region
            Shape s2 = c->shape;
            s2.lam_len = S + 1;
            c->lam_valid = false;
            OK(bind(c, s2));
        }
        c->lam_h.assign(S + 1, 0.0);
        OK(eamfe_lambda_schedule(p, c->lam_h.data(), &S));
        HIPCHK(c, hipStreamSynchronize(c->stream));   // earlier passes may still read the old table
        HIPCHK(c, hipMemcpy(c->lam_d.p, c->lam_h.data(), (S + 1) * sizeof(double), hipMemcpyHostToDevice));
        c->lam_key = *p;
        c->lam_valid = true;
    }
    *S_out = S;
    return EAMFE_OK;
}

// Per-replica thermostat amplitude for the protocol's damping.
int set_thermostat(eamfe_ctx* c, const eamfe_protocol* p, double* c1_out)
{
    const double c1 = p->damp > 0.0 ? std::exp(-p->dt / p->damp) : 1.0;
    bool changed = false;
    for (auto& R : c->reps) {
        const double c2 = std::sqrt((1.0 - c1 * c1) * kB * R.T * R.inv_m);
        if (c2 != R.c2) {
            R.c2 = c2;
            changed = true;
        }
    }
    if (changed) OK(upload_reps(c));
    *c1_out = c1;
    return EAMFE_OK;
}

// Lists valid for packed positions P: plan them if needed, else flag the
// replicas in which some atom moved more than skin/2 since the last build.
int ensure_lists(eamfe_ctx* c, double skin, const double4* P)
{
    if (!c->have_list || skin != c->skin) {
        OK(plan_lists(c, skin, c->have_list ? c->cap : 0));
        c->have_list = true;
        OK(set_rebuild_all(c));
    } else {
        NeighArgs na = neigh_args(c, P);
        LCHK(c, launch_check_displacement(na, c->stream));
    }
    return EAMFE_OK;
}


// Pack caller SoA positions into the A buffers (both numeric forms).
int pack(eamfe_ctx* c, const double* x)
{
    LCHK(c, launch_pack(PA(c), QA(c), x, (const int32_t*)c->rep_of_d.p, (const RepDesc*)c->reps_d.p, c->N,
                        c->stream));
    return EAMFE_OK;
}

// The adjoint's tables: equal knot counts, and each block's histogram of
// four fixed-point words per interval (32 bytes) within one block's LDS.
int check_adjoint_tables(eamfe_ctx* c, const char* who)
{
    if (c->n_r != c->n_rho)
        return fail(c, EAMFE_EINVAL, std::string(who) + ": phi/rho and F tables must have equal knot counts");
    const long need = 32L * (std::max(c->n_r, c->n_rho) - 1);
    if (need > c->max_lds)
        return fail(c, EAMFE_EINVAL, std::string(who) + ": tables of " + std::to_string(c->n_r) +
                                         " knots need " + std::to_string(need) + " bytes of LDS per block, more than " +
                                         std::to_string(c->max_lds) + " (at most " +
                                         std::to_string(c->max_lds / 32 + 1) + " knots)");
    return EAMFE_OK;
}

// dU/dtheta at the packed positions P (density pass already run with
// rho_out, so F' and rho are current): bins -> knot gradients into out.
// bins: n_rep * 3 * nb * 4 fixed-point words; fin: the knot transform's
// work rows, (reduce ? 1 : n_rep) * 3 * 2 * (nb + 1) doubles.
int adjoint_at(eamfe_ctx* c, const double4* P, const double* w_host, int reduce, double* out,
               unsigned long long* bins_p, double* fin_p)
{
    OK(check_adjoint_tables(c, "adjoint"));
    const int nb = std::max(c->n_r, c->n_rho) - 1;
    const size_t bins = (size_t)c->n_rep * 3 * nb * 4;
    LCHK(c, launch_fill_u64(bins_p, bins, 0ull, c->stream));   // a fill kernel: capturable, unlike a memset
    AdjointArgs a{};
    a.reps = (const RepDesc*)c->reps_d.p;
    a.P = P;
    a.Q = Q_of(c, P);
    a.nbr = (const int32_t*)c->nbr_d.p;
    a.nnb = (const int32_t*)c->nnb_d.p;
    a.cap = c->cap;
    a.rho = (const double*)c->rho_d.p;
    a.bins = bins_p;
    a.nb = nb;
    a.tab = tables_of(c);
    a.N = c->N;
    a.n_rep = c->n_rep;
    a.tile_atoms = 64 / c->lanes;
    a.n_units = c->n_tiles;
    const int grid = std::max(1, std::min(c->n_tiles, 2 * c->n_cu));
    LCHK(c, launch_adjoint(a, c->precision, grid, c->stream));
    const double* wd = nullptr;
    if (w_host) {
        HIPCHK(c, hipMemcpyAsync(c->adj_w_d.p, w_host, (size_t)c->n_rep * sizeof(double), hipMemcpyHostToDevice,
                                 c->stream));
        HIPCHK(c, hipStreamSynchronize(c->stream));   // the host array may go away
        wd = (const double*)c->adj_w_d.p;
    }
    LCHK(c, launch_adjoint_finish(a, wd, reduce, out, fin_p, c->stream));
    return EAMFE_OK;
}

// Timing events of a sampled launch (kind: 0 density, 1 force, 2 lists).
// mark records one on the stream (end = 0 start, 1 stop), around the list
// pass's kernels; stamps hands out a pair for a pair kernel to stamp with
// its own start and end (null pair: this launch is not sampled).  They are
// read only after the stream has been synchronised, so they are recorded
// without the system-scope fence (no cache writeback and invalidation
// between the sampled kernel and the next).
int next_event(eamfe_ctx* c, hipEvent_t* e)
{
    if (c->ev_used == c->ev_pool.size()) {
        hipEvent_t n;
        HIPCHK(c, hipEventCreateWithFlags(&n, hipEventDisableSystemFence));
        c->ev_pool.push_back(n);
    }
    *e = c->ev_pool[c->ev_used++];
    return EAMFE_OK;
}

bool sampled(const eamfe_ctx* c, int kind)
{
    return c->timing && c->timing_now && (c->timing_kinds & (1 << kind));
}

int mark(eamfe_ctx* c, int kind, int end)
{
    if (!sampled(c, kind)) return EAMFE_OK;
    if (!end) c->ev_kind.push_back(kind);
    hipEvent_t e;
    OK(next_event(c, &e));
    HIPCHK(c, hipEventRecord(e, c->stream));
    return EAMFE_OK;
}

int stamps(eamfe_ctx* c, int kind, hipEvent_t* t0, hipEvent_t* t1)
{
    *t0 = *t1 = nullptr;
    if (!sampled(c, kind)) return EAMFE_OK;
    c->ev_kind.push_back(kind);
    OK(next_event(c, t0));
    return next_event(c, t1);
}

// Iterations it_first .. it_last of a protocol starting from packed
// positions *cur (one of the two internal buffers); on return *cur is the
// buffer holding the final positions.
// One MD iteration on stream st: list upkeep (whose first kernel finishes
// the previous iteration's force pass), density pass, force pass.  Without
// EAM there is no list pass and the force pass is finished at once; with it
// the caller finishes the last iteration's force pass.
// finish_prev: the density pass finishes the force pass before it (an extra
// block, off the path of the list pass).
int one_iteration(eamfe_ctx* c, StepArgs& a, double4* cur, double4* nxt, bool has_eam, hipStream_t st, bool sample,
                  bool finish_prev)
{
    // sampled: the first iteration after timing was switched on, then every
    // timing-th one, so any range of at least one iteration has a sample
    c->timing_now = c->timing > 0 && c->timing_seen % c->timing == 0;
    if (c->timing > 0) ++c->timing_seen;
    if (has_eam) {
        NeighArgs na = neigh_args(c, cur);
        OK(mark(c, 2, 0));
        LCHK(c, launch_neigh_rebuild(na, a, c->lanes, c->block, st));
        OK(mark(c, 2, 1));
    }
    a.P = cur;
    a.Pn = nxt;
    a.Q = Q_of(c, cur);
    a.Qn = Q_of(c, nxt);
    a.rho_out = sample ? (double*)c->rho_d.p : nullptr;
    a.finish_prev = finish_prev ? 1 : 0;
    hipEvent_t t0, t1;
    OK(stamps(c, 0, &t0, &t1));
    LCHK(c, launch_density(a, c->precision, c->lanes, c->block, st, t0, t1));
    a.finish_prev = 0;
    if (sample) {
        OK(adjoint_at(c, cur, c->adj_w.empty() ? nullptr : c->adj_w.data(), c->adj_reduce, c->adj_out,
                      (unsigned long long*)c->bins_d.p, (double*)c->adj_scratch_d.p));
        ++c->adj_samples;
    }
    OK(stamps(c, 1, &t0, &t1));
    LCHK(c, launch_force(a, c->precision, c->lanes, c->block, st, t0, t1));
    if (!has_eam) LCHK(c, launch_finish(a, st));
    return EAMFE_OK;
}

void drop_graphs(eamfe_ctx* c)
{
    for (int k = 0; k < 2; ++k) {
        if (c->gexec[k]) (void)hipGraphExecDestroy(c->gexec[k]);
        c->gexec[k] = nullptr;
    }
}

// Capture `iters` (even) middle iterations starting from buffer `start` into a
// graph on the internal stream; the kernels read the step from the device
// counter, so one graph serves every middle stretch of a run.
int capture_middle(eamfe_ctx* c, const StepArgs& a0, double4* start, bool has_eam, int iters, hipGraphExec_t* out)
{
    StepArgs a = a0;
    const int timing = c->timing;
    c->timing = 0;                   // no event records inside a graph
    a.it_first = -1;                 // the closing kick of the previous step always applies
    a.it_last = INT64_MAX;           // and a new step always starts
    HIPCHK(c, hipStreamBeginCapture(c->gstream, hipStreamCaptureModeThreadLocal));
    double4* cur = start;
    double4* nxt = cur == PA(c) ? PB(c) : PA(c);
    int rc = EAMFE_OK;
    for (int k = 0; k < iters && rc == EAMFE_OK; ++k) {
        a.it_k = k;   // step = the counter at the replay's start + k
        rc = one_iteration(c, a, cur, nxt, has_eam, c->gstream, false, has_eam);
        std::swap(cur, nxt);
    }
    if (rc == EAMFE_OK) rc = launch_advance_iter((int64_t*)c->iter_d.p, iters, c->gstream) ? EAMFE_EDEVICE : EAMFE_OK;
    c->timing = timing;
    hipGraph_t g = nullptr;
    const hipError_t e = hipStreamEndCapture(c->gstream, &g);
    if (rc) {
        if (g) (void)hipGraphDestroy(g);
        return rc;
    }
    if (e != hipSuccess) return fail(c, EAMFE_EDEVICE, std::string("hipStreamEndCapture: ") + hipGetErrorString(e));
    const hipError_t e2 = hipGraphInstantiate(out, g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    if (e2 != hipSuccess) return fail(c, EAMFE_EDEVICE, std::string("hipGraphInstantiate: ") + hipGetErrorString(e2));
    return EAMFE_OK;
}

// Iterations it_first .. it_last of a protocol starting from packed
// positions *cur (one of the two internal buffers); on return *cur is the
// buffer holding the final positions.  The first and last iterations carry
// the open/close flags and run eagerly; with graphs enabled the middle ones
// replay a captured graph of c->graph_iters iterations.
int iterate(eamfe_ctx* c, StepArgs a, double4** cur_io, bool has_eam, int64_t it_first, int64_t it_last)
{
    double4* cur = *cur_io;
    double4* nxt = cur == PA(c) ? PB(c) : PA(c);
    a.it_first = it_first;
    a.it_last = it_last;
    a.step_kernel = 1;
    a.has_eam = has_eam ? 1 : 0;
    OK(set_iter(c, it_first));
    int64_t base = it_first;   // the device step counter
    const bool graphs = c->graph_iters > 0 && !c->timing && c->adj_every == 0 && c->gstream;
    int64_t it = it_first;
    while (it <= it_last) {
        const bool middle = it > it_first && it < it_last;
        if (graphs && middle && it_last - it >= c->graph_iters) {
            if (base != it) {   // a replay's steps count from the counter
                OK(set_iter(c, it));
                base = it;
            }
            const int k = cur == PA(c) ? 0 : 1;
            if (!c->gexec[k]) OK(capture_middle(c, a, cur, has_eam, c->graph_iters, &c->gexec[k]));
            HIPCHK(c, hipEventRecord(c->ev_user, c->stream));
            HIPCHK(c, hipStreamWaitEvent(c->gstream, c->ev_user, 0));
            const int64_t reps = (it_last - it) / c->graph_iters;
            for (int64_t q = 0; q < reps; ++q) HIPCHK(c, hipGraphLaunch(c->gexec[k], c->gstream));
            HIPCHK(c, hipEventRecord(c->ev_graph, c->gstream));
            HIPCHK(c, hipStreamWaitEvent(c->stream, c->ev_graph, 0));
            it += reps * c->graph_iters;   // graph_iters is even: the buffers are back where they were
            base += reps * c->graph_iters;   // each replay advanced the counter
            continue;
        }
        const bool sample = has_eam && c->adj_every > 0 && it < it_last && it % c->adj_every == 0 &&
                            c->lam_valid && c->lam_h[it] == c->lam_h[0];
        a.it_k = it - base;
        OK(one_iteration(c, a, cur, nxt, has_eam, c->stream, sample, has_eam && it > it_first));
        std::swap(cur, nxt);
        ++it;
    }
    if (has_eam && it > it_first) {   // the last force pass
        a.it_k = (it - 1) - base;
        LCHK(c, launch_finish(a, c->stream));
    }
    *cur_io = cur;
    return EAMFE_OK;
}

bool ready(eamfe_ctx* c, bool need_pot);

// dU/dtheta at positions x.  The adjoint's bins and knot-transform rows are
// the context's own (static_base null), or at static_base and static_base +
// fin_off.  The context's are looked up only after the lists are in place:
// planning the lists can move the adjoint group of the arena.
int adjoint_theta_with(eamfe_ctx* c, const double* x, const double* w_host, int reduce, double* dtheta,
                       char* static_base, size_t fin_off)
{
    OK(check_adjoint_tables(c, "adjoint_theta"));   // before any kernel runs
    OK(pack(c, x));
    OK(ensure_lists(c, c->have_list ? c->skin : 0.3, PA(c)));
    NeighArgs na = neigh_args(c, PA(c));
    LCHK(c, launch_neigh_rebuild(na, step_args(c), c->lanes, c->block, c->stream));
    StepArgs a = step_args(c);
    a.P = PA(c);
    a.Q = QA(c);
    a.has_eam = 1;
    a.step_kernel = 0;
    a.rho_out = (double*)c->rho_d.p;
    LCHK(c, launch_density(a, c->precision, c->lanes, c->block, c->stream));
    unsigned long long* bins = static_base ? (unsigned long long*)static_base : (unsigned long long*)c->bins_d.p;
    double* fin = static_base ? (double*)(static_base + fin_off) : (double*)c->adj_scratch_d.p;
    OK(adjoint_at(c, PA(c), w_host, reduce, dtheta, bins, fin));
    return read_status(c);
}

bool ready(eamfe_ctx* c, bool need_pot)
{
    if (!c) return false;
    if (need_pot && !c->have_pot) {
        c->err = "eam_setup has not been called";
        return false;
    }
    if (c->n_rep == 0) {
        c->err = "eamfe_system_setup has not been called";
        return false;
    }
    return true;
}

}  // namespace

// ===========================================================================
// C ABI
// ===========================================================================
extern "C" {

int eamfe_create(eamfe_ctx** out, int device, void* hip_stream, int precision, int deterministic)
{
    if (!out || (precision != EAMFE_FP64 && precision != EAMFE_FP32) || (deterministic != 0 && deterministic != 1))
        return EAMFE_EINVAL;
    *out = nullptr;
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || device < 0 || device >= ndev) return EAMFE_EDEVICE;
    if (hipSetDevice(device) != hipSuccess) return EAMFE_EDEVICE;
    eamfe_ctx* c = new (std::nothrow) eamfe_ctx();
    if (!c) return EAMFE_ENOMEM;
    c->device = device;
    c->stream = (hipStream_t)hip_stream;
    c->precision = precision;
    c->deterministic = deterministic;
    if (scratch_setup(device) != EAMFE_OK) {
        delete c;
        return EAMFE_EDEVICE;
    }
    {
        int cus = 0;
        if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, device) == hipSuccess && cus > 0)
            c->n_cu = cus;
        int lds = 0;
        if (hipDeviceGetAttribute(&lds, hipDeviceAttributeMaxSharedMemoryPerBlock, device) == hipSuccess && lds > 0)
            c->max_lds = lds;
    }
    *out = c;   // no device memory yet: the first setup call lays out the arena
    return EAMFE_OK;
}

int eamfe_destroy(eamfe_ctx* c)
{
    if (!c) return EAMFE_OK;
    (void)hipSetDevice(c->device);
    if (c->stream) (void)hipStreamSynchronize(c->stream);
    else (void)hipDeviceSynchronize();
    for (hipEvent_t e : c->ev_pool) (void)hipEventDestroy(e);
    drop_graphs(c);
    if (c->ev_user) (void)hipEventDestroy(c->ev_user);
    if (c->ev_graph) (void)hipEventDestroy(c->ev_graph);
    if (c->gstream) (void)hipStreamDestroy(c->gstream);
    if (c->arena && !c->caller_ws) (void)hipFree(c->arena);   // never the caller's workspace
    delete c;
    return EAMFE_OK;
}

int eamfe_workspace_bytes(const eamfe_ctx* c, size_t* bytes)
{
    if (!c || !bytes) return EAMFE_EINVAL;
    const size_t cur = layout_bytes(const_cast<eamfe_ctx*>(c), c->shape);
    *bytes = std::max(cur, c->need);
    return EAMFE_OK;
}

int eamfe_set_workspace(eamfe_ctx* c, void* dev, size_t bytes)
{
    if (!c || (bytes && !dev)) return EAMFE_EINVAL;
    if ((uintptr_t)dev % kAlign) return fail(c, EAMFE_EINVAL, "set_workspace: the workspace must be 256-byte aligned");
    const size_t used = layout_bytes(c, c->shape);
    if (bytes < used) {
        c->need = std::max(c->need, used);
        return fail(c, EAMFE_ENOMEM, "set_workspace: " + std::to_string(used) + " bytes needed");
    }
    (void)hipSetDevice(c->device);
    HIPCHK(c, hipStreamSynchronize(c->stream));
    // every live buffer keeps its offset: one copy moves them all
    if (c->arena && used && (char*)dev != c->arena)
        HIPCHK(c, hipMemcpy(dev, c->arena, used, hipMemcpyDeviceToDevice));
    if (c->arena && !c->caller_ws) (void)hipFree(c->arena);
    c->arena = (char*)dev;
    c->arena_bytes = bytes;
    c->caller_ws = true;
    size_t off = 0;
    for_regions(c, c->shape, [&](DevBuf& b, int, size_t n) {
        b.p = c->arena + off;
        b.bytes = n;
        off += align_up(n);
    });
    drop_graphs(c);
    return EAMFE_OK;
}

int eamfe_resume_step(const eamfe_ctx* c, int64_t* step)
{
    if (!c || !step) return EAMFE_EINVAL;
    *step = c->resume_step;
    return EAMFE_OK;
}

int eamfe_device_allocations(const eamfe_ctx* c, int64_t* n)
{
    if (!c || !n) return EAMFE_EINVAL;
    *n = c->device_allocs;
    return EAMFE_OK;
}

const char* eamfe_last_error(const eamfe_ctx* c) { return c ? c->err.c_str() : "null context"; }

int eamfe_set_stream(eamfe_ctx* c, void* s)
{
    if (!c) return EAMFE_EINVAL;
    c->stream = (hipStream_t)s;
    return EAMFE_OK;
}

int eamfe_set_launch(eamfe_ctx* c, int lanes, int block)
{
    if (!c) return EAMFE_EINVAL;
    if (lanes && lanes != 1 && lanes != 2 && lanes != 4 && lanes != 8 && lanes != 16)
        return fail(c, EAMFE_EINVAL, "lanes_per_atom must be 1, 2, 4, 8 or 16");
    if (block && (block < 64 || block > 1024 || block % 64))
        return fail(c, EAMFE_EINVAL, "block_threads must be a multiple of 64 in [64, 1024]");
    if (lanes) c->lanes = lanes;
    if (block) c->block = block;
    if (c->n_rep) {
        (void)hipSetDevice(c->device);
        HIPCHK(c, hipStreamSynchronize(c->stream));
        return build_tiles(c);
    }
    return EAMFE_OK;
}

int eamfe_set_graph(eamfe_ctx* c, int iters)
{
    if (!c || iters < 0) return EAMFE_EINVAL;
    (void)hipSetDevice(c->device);
    drop_graphs(c);
    c->graph_iters = (iters + 1) / 2 * 2;
    if (c->graph_iters && !c->gstream) {
        HIPCHK(c, hipStreamCreateWithFlags(&c->gstream, hipStreamNonBlocking));
        HIPCHK(c, hipEventCreateWithFlags(&c->ev_user, hipEventDisableTiming));
        HIPCHK(c, hipEventCreateWithFlags(&c->ev_graph, hipEventDisableTiming));
    }
    return EAMFE_OK;
}

int eamfe_set_grid(eamfe_ctx* c, int blocks)
{
    if (!c || blocks < 0) return EAMFE_EINVAL;
    c->grid = (blocks + 7) / 8 * 8;
    return EAMFE_OK;
}

int eamfe_get_grid(const eamfe_ctx* c, int* blocks)
{
    if (!c || !blocks) return EAMFE_EINVAL;
    *blocks = c->grid;
    return EAMFE_OK;
}

int eamfe_get_launch(const eamfe_ctx* c, int* lanes, int* block)
{
    if (!c) return EAMFE_EINVAL;
    if (lanes) *lanes = c->lanes;
    if (block) *block = c->block;
    return EAMFE_OK;
}

int eamfe_set_list_builder(eamfe_ctx* c, int lds)
{
    if (!c || (lds != 0 && lds != 1)) return EAMFE_EINVAL;
    if (c->lds_rows != lds) {
        c->lds_rows = lds;
        c->have_list = false;   // planned and built again by the next pass
    }
    return EAMFE_OK;
}

int eamfe_get_list_builder(const eamfe_ctx* c, int* lds)
{
    if (!c || !lds) return EAMFE_EINVAL;
    *lds = c->lds_rows;
    return EAMFE_OK;
}

int eamfe_set_xcd_affinity(eamfe_ctx* c, int on)
{
    if (!c) return EAMFE_EINVAL;
    c->xcd = on ? 1 : 0;
    if (c->n_rep) {
        (void)hipSetDevice(c->device);
        HIPCHK(c, hipStreamSynchronize(c->stream));
        return build_tiles(c);
    }
    return EAMFE_OK;
}

int eamfe_check(eamfe_ctx* c)
{
    if (!c) return EAMFE_EINVAL;
    (void)hipSetDevice(c->device);
    return read_status(c);
}

int eam_setup(eamfe_ctx* c, int n_r, double r_cut, const double* phi, const double* rho, int n_rho, double rho_max,
              const double* F)
{
    if (!c) return EAMFE_EINVAL;
    if (n_r < 3 || n_rho < 3 || !(r_cut > 0.0) || !(rho_max > 0.0) || !phi || !rho || !F)
        return fail(c, EAMFE_EINVAL, "eam_setup: bad table description");
    // the FP32 pair kernels hold the pair table and the density-derivative
    // table in one block's LDS: 16 bytes per interval each, plus a padding
    // interval per table
    if (c->precision == EAMFE_FP32 && 32L * n_r > c->max_lds)
        return fail(c, EAMFE_EINVAL, "eam_setup: FP32 tables of " + std::to_string(n_r) + " knots need " +
                                         std::to_string(32L * n_r) + " bytes of LDS per block, more than " +
                                         std::to_string(c->max_lds) + " (at most " + std::to_string(c->max_lds / 32) +
                                         " knots in EAMFE_FP32; EAMFE_FP64 reads its tables from global memory)");
    (void)hipSetDevice(c->device);
    HIPCHK(c, hipStreamSynchronize(c->stream));
    Shape s2 = c->shape;
    s2.n_r = n_r;
    s2.n_rho = n_rho;
    OK(bind(c, s2));   // nothing changes if the tables do not fit
    c->n_r = n_r;
    c->n_rho = n_rho;
    c->r_cut = r_cut;
    c->rho_max = rho_max;
    c->knots_phi.assign(phi, phi + n_r);
    c->knots_rho.assign(rho, rho + n_r);
    c->knots_F.assign(F, F + n_rho);
    c->c_phi = natural_spline(phi, n_r, r_cut / (n_r - 1));
    c->c_rho = natural_spline(rho, n_r, r_cut / (n_r - 1));
    c->c_F = natural_spline(F, n_rho, rho_max / (n_rho - 1));
    OK(upload_tables(c));
    c->have_pot = true;
    c->have_list = false;   // the cutoff may have changed
    return EAMFE_OK;
}

int eamfe_system_setup(eamfe_ctx* c, int n_rep, const eamfe_replica* in, const double* x0_dev)
{
    if (!c) return EAMFE_EINVAL;
    if (n_rep < 1 || !in || !x0_dev) return fail(c, EAMFE_EINVAL, "system_setup: bad arguments");
    if (n_rep > kMaxRepsList)
        return fail(c, EAMFE_EINVAL, "system_setup: at most " + std::to_string(kMaxRepsList) + " replicas");
    (void)hipSetDevice(c->device);
    HIPCHK(c, hipStreamSynchronize(c->stream));
    long N = 0;
    for (int r = 0; r < n_rep; ++r) {
        const eamfe_replica& q = in[r];
        if (q.n_atoms < 1 || !(q.mass > 0.0) || !(q.T >= 0.0) || !(q.box[0] > 0 && q.box[1] > 0 && q.box[2] > 0))
            return fail(c, EAMFE_EINVAL, "replica " + std::to_string(r) + ": bad description");
        N += q.n_atoms;
    }
    if (N >= (1L << 28)) return fail(c, EAMFE_EINVAL, "too many atoms (at most 2^28 - 1)");
    Shape s2 = c->shape;
    s2.N = N;
    s2.n_rep = n_rep;
    s2.max_units = 0;   // units of 64/16 atoms, the finest launch shape
    for (int r = 0; r < n_rep; ++r) s2.max_units += (in[r].n_atoms + 3) / 4;
    s2.max_slices = 8L * std::max<long>(n_rep, c->n_cu);
    s2.cap = s2.n_cells = s2.ccap = 0;   // lists are planned for the new system
    OK(bind(c, s2));   // nothing changes if the system does not fit
    c->have_list = false;
    c->cap_min = 0;
    c->min_ccap = 0;
    c->n_rep = n_rep;
    c->N = (int)N;
    c->reps_in.assign(in, in + n_rep);
    c->reps.assign(n_rep, RepDesc{});
    std::vector<int32_t> rep_of(N);
    int off = 0;
    for (int r = 0; r < n_rep; ++r) {
        RepDesc& R = c->reps[r];
        const eamfe_replica& q = in[r];
        R.off = off;
        R.n = q.n_atoms;
        for (int d = 0; d < 3; ++d) {
            R.L[d] = q.box[d];
            R.invL[d] = 1.0 / q.box[d];
        }
        R.T = q.T;
        R.k = q.k;
        R.k2 = q.k2;
        R.mass = q.mass;
        R.inv_m = 1.0 / (q.mass * mvv2e);
        R.sig_v = std::sqrt(kB * q.T * R.inv_m);
        R.c2 = 0.0;
        R.seed = q.seed;
        for (int i = 0; i < q.n_atoms; ++i) rep_of[off + i] = r;
        off += q.n_atoms;
    }
    const size_t v3 = 3 * (size_t)N * sizeof(double);
    HIPCHK(c, hipMemcpy(c->x0_d.p, x0_dev, v3, hipMemcpyDeviceToDevice));
    HIPCHK(c, hipMemcpy(c->xref_d.p, x0_dev, v3, hipMemcpyDeviceToDevice));
    HIPCHK(c, hipMemset(c->xi_d.p, 0, v3));
    HIPCHK(c, hipMemset(c->Pa_d.p, 0, (size_t)N * sizeof(double4)));
    HIPCHK(c, hipMemset(c->Pb_d.p, 0, (size_t)N * sizeof(double4)));
    HIPCHK(c, hipMemset(c->Qa_d.p, 0, (size_t)N * sizeof(uint4)));
    HIPCHK(c, hipMemset(c->Qb_d.p, 0, (size_t)N * sizeof(uint4)));
    HIPCHK(c, hipMemset(c->e_emb_d.p, 0, (size_t)N * sizeof(double)));
    HIPCHK(c, hipMemcpy(c->rep_of_d.p, rep_of.data(), (size_t)N * sizeof(int32_t), hipMemcpyHostToDevice));
    HIPCHK(c, hipMemset(c->U_rep_d.p, 0, (size_t)n_rep * 2 * sizeof(double)));
    HIPCHK(c, hipMemset(c->W_state_d.p, 0, (size_t)n_rep * sizeof(double)));
    HIPCHK(c, hipMemset(c->rebuild_d.p, 0, (size_t)n_rep * sizeof(int32_t)));
    HIPCHK(c, hipMemset(c->flag_pre_d.p, 0, (size_t)(2 * n_rep + 2) * sizeof(int32_t)));
    HIPCHK(c, hipMemset(c->row_acc_d.p, 0, (size_t)(n_rep + 3) * sizeof(double)));
    c->have_list = false;
    c->has_kscale = false;
    return build_tiles(c);
}

int neigh_build(eamfe_ctx* c, const double* x, double skin, int max_neighbors)
{
    if (!ready(c, true)) return c ? EAMFE_ESTATE : EAMFE_EINVAL;
    if (!x || !(skin >= 0.0) || max_neighbors < 0) return fail(c, EAMFE_EINVAL, "neigh_build: bad arguments");
    (void)hipSetDevice(c->device);
    HIPCHK(c, hipStreamSynchronize(c->stream));
    OK(plan_lists(c, skin, max_neighbors));
    c->have_list = true;
    OK(pack(c, x));
    for (int attempt = 0;; ++attempt) {
        OK(set_rebuild_all(c));
        NeighArgs na = neigh_args(c, PA(c));
        LCHK(c, launch_neigh_rebuild(na, step_args(c), c->lanes, c->block, c->stream));
        // the flags and bin counters are cleared by the next density pass; clear them here too
        hipLaunchKernelGGL(k_fill_i32, dim3((c->n_rep + 255) / 256), dim3(256), 0, c->stream,
                           (int32_t*)c->rebuild_d.p, c->n_rep, 0);
        HIPCHK(c, hipGetLastError());
        if (c->n_cells > 0) {
            hipLaunchKernelGGL(k_fill_i32, dim3((c->n_cells + 255) / 256), dim3(256), 0, c->stream,
                               (int32_t*)c->cell_cnt_d.p, c->n_cells, 0);
            HIPCHK(c, hipGetLastError());
        }
        if (max_neighbors > 0 || attempt >= 6) break;
        // automatic capacity: enlarge rows or bins until this configuration fits
        HIPCHK(c, hipStreamSynchronize(c->stream));
        int st = 0;
        HIPCHK(c, hipMemcpy(&st, c->status_d.p, sizeof(int), hipMemcpyDeviceToHost));
        if (!(st & (ST_NEIGH_OVERFLOW | ST_CELL_OVERFLOW))) break;
        HIPCHK(c, hipMemset(c->status_d.p, 0, sizeof(int)));
        OK(grow_lists(c, st));
    }
    return read_status(c);
}

int eam_forces(eamfe_ctx* c, const double* x, double* f, double* U, double* e_atom)
{
    if (!ready(c, true)) return c ? EAMFE_ESTATE : EAMFE_EINVAL;
    if (!x) return fail(c, EAMFE_EINVAL, "eam_forces: null positions");
    (void)hipSetDevice(c->device);
    OK(pack(c, x));
    OK(ensure_lists(c, c->have_list ? c->skin : 0.3, PA(c)));
    for (int attempt = 0;; ++attempt) {
        NeighArgs na = neigh_args(c, PA(c));
        LCHK(c, launch_neigh_rebuild(na, step_args(c), c->lanes, c->block, c->stream));
        StepArgs a = step_args(c);
        a.P = PA(c);
        a.Pn = nullptr;
        a.Q = QA(c);
        a.Qn = nullptr;
        a.v = nullptr;
        a.has_eam = 1;
        a.step_kernel = 0;
        a.mode = EAMFE_MODE_FL;
        a.f_out = f;
        a.e_atom_out = e_atom;
        LCHK(c, launch_density(a, c->precision, c->lanes, c->block, c->stream));
        LCHK(c, launch_force(a, c->precision, c->lanes, c->block, c->stream));
        LCHK(c, launch_finish(a, c->stream));
        HIPCHK(c, hipStreamSynchronize(c->stream));
        int st = 0;
        HIPCHK(c, hipMemcpy(&st, c->status_d.p, sizeof(int), hipMemcpyDeviceToHost));
        if (!(st & (ST_NEIGH_OVERFLOW | ST_CELL_OVERFLOW)) || attempt >= 6) break;
        // rows or bins too small for this configuration: enlarge and evaluate again
        HIPCHK(c, hipMemset(c->status_d.p, 0, sizeof(int)));
        OK(grow_lists(c, st));
        OK(set_rebuild_all(c));
        ++c->replays;
    }
    if (U)
        HIPCHK(c, hipMemcpy2DAsync(U, sizeof(double), c->U_rep_d.p, 2 * sizeof(double), sizeof(double), c->n_rep,
                                   hipMemcpyDeviceToDevice, c->stream));
    return read_status(c);
}

int eamfe_init_velocities(eamfe_ctx* c, double* v, int fix_com)
{
    if (!ready(c, false)) return c ? EAMFE_ESTATE : EAMFE_EINVAL;
    if (!v) return fail(c, EAMFE_EINVAL, "init_velocities: null v");
    (void)hipSetDevice(c->device);
    StepArgs a = step_args(c);
    a.v = v;
    LCHK(c, launch_init_velocities(a, c->n_rep, fix_com, c->stream));
    return EAMFE_OK;
}

int eamfe_lambda_schedule(const eamfe_protocol* p, double* lam, int64_t* n_steps)
{
    if (check_protocol(p)) return EAMFE_EINVAL;
    const int64_t S = (int64_t)p->n_eq + 2 * (int64_t)p->n_sw + p->n_hold + p->n_hold2;
    if (n_steps) *n_steps = S;
    if (!lam) return EAMFE_OK;
    const bool rs = p->mode == EAMFE_MODE_RS || p->mode == EAMFE_MODE_EIN_RS;
    const double start = rs ? 1.0 : 0.0;
    auto f = [&](double tau) { return rs ? lambda_rs(p->lambda_f, tau) : lambda_fl(p->function, tau); };
    int64_t s = 0;
    for (int64_t q = 0; q <= p->n_eq; ++q) lam[s++] = start;                // equilibrate at the start point
    for (int64_t q = 1; q <= p->n_sw; ++q) lam[s++] = f((double)q / p->n_sw);  // forward
    const double end = lam[s - 1];
    for (int64_t q = 1; q <= p->n_hold; ++q) lam[s++] = end;                // hold at the end point
    for (int64_t q = 1; q <= p->n_sw; ++q) lam[s++] = f(1.0 - (double)q / p->n_sw);  // backward (time reverse)
    for (int64_t q = 1; q <= p->n_hold2; ++q) lam[s++] = start;
    return s == S + 1 ? EAMFE_OK : EAMFE_EINVAL;
}

}  // extern "C"

namespace {

// Steps [s0, s1) from caller positions x (SoA, packed on entry, unpacked on
// exit) and velocities v.  Steps run in chunks; after each chunk the
// latched status is read.  A neighbour-row or cell overflow (possible when a
// crystal collapses into dense clusters) restores the chunk's starting
// state, enlarges the capacity and replays the chunk; the noise is a
// function of (seed, atom, step), so the replay is the trajectory the run
// would have had.
int run_range(eamfe_ctx* c, const eamfe_protocol* p, int64_t S, int64_t s0, int64_t s1, double* x, double* v,
              double* dHdl_out, double* W_out, int64_t stride, int64_t trace_off, double c1, bool has_eam)
{
    if (has_eam && c->adj_every > 0) OK(check_adjoint_tables(c, "adjoint sampling"));   // before any step runs
    drop_graphs(c);   // captured kernel arguments belong to one call (pointers, protocol, shapes)
    OK(pack(c, x));
    double4* cur = PA(c);
    c->resume_step = s0;   // nothing has run if the lists do not fit
    if (has_eam) OK(ensure_lists(c, p->skin, cur));
    c->resume_step = -1;
    const size_t v3 = 3 * (size_t)c->N * sizeof(double);
    const size_t p4 = (size_t)c->N * sizeof(double4);
    const size_t wb = (size_t)c->n_rep * sizeof(double);
    const size_t q4 = (size_t)c->N * sizeof(uint4);
    for (int64_t b = s0; b < s1; b += c->chunk) {
        const int64_t e = std::min(s1, b + c->chunk);
        if (has_eam) {
            HIPCHK(c, hipMemcpyAsync(c->snap_P.p, cur, p4, hipMemcpyDeviceToDevice, c->stream));
            HIPCHK(c, hipMemcpyAsync(c->snap_Q.p, Q_of(c, cur), q4, hipMemcpyDeviceToDevice, c->stream));
            HIPCHK(c, hipMemcpyAsync(c->snap_v.p, v, v3, hipMemcpyDeviceToDevice, c->stream));
            HIPCHK(c, hipMemcpyAsync(c->snap_w.p, c->W_state_d.p, wb, hipMemcpyDeviceToDevice, c->stream));
            HIPCHK(c, hipMemcpyAsync(c->snap_rows.p, c->row_acc_d.p, wb + 3 * sizeof(double), hipMemcpyDeviceToDevice,
                                     c->stream));
        }
        for (int attempt = 0;; ++attempt) {
            StepArgs a = step_args(c);
            a.v = v;
            a.lam = (const double*)c->lam_d.p;
            a.dHdl_out = dHdl_out;
            a.W_out = W_out;
            a.S = stride;
            a.trace_off = trace_off;
            a.mode = p->mode;
            a.fix_com = p->fix_com ? 1 : 0;
            a.dt = p->dt;
            a.c1 = c1;
            double4* start = cur;
            OK(iterate(c, a, &cur, has_eam, b, e));
            if (!has_eam) break;
            HIPCHK(c, hipStreamSynchronize(c->stream));
            int st = 0;
            HIPCHK(c, hipMemcpy(&st, c->status_d.p, sizeof(int), hipMemcpyDeviceToHost));
            if (!(st & (ST_NEIGH_OVERFLOW | ST_CELL_OVERFLOW))) break;
            if (attempt >= 6) return read_status(c);
            HIPCHK(c, hipMemset(c->status_d.p, 0, sizeof(int)));
            drop_graphs(c);
            // back to the chunk's start, then larger rows or bins
            cur = start;
            HIPCHK(c, hipMemcpyAsync(cur, c->snap_P.p, p4, hipMemcpyDeviceToDevice, c->stream));
            HIPCHK(c, hipMemcpyAsync(Q_of(c, cur), c->snap_Q.p, q4, hipMemcpyDeviceToDevice, c->stream));
            HIPCHK(c, hipMemcpyAsync(v, c->snap_v.p, v3, hipMemcpyDeviceToDevice, c->stream));
            HIPCHK(c, hipMemcpyAsync(c->W_state_d.p, c->snap_w.p, wb, hipMemcpyDeviceToDevice, c->stream));
            HIPCHK(c, hipMemcpyAsync(c->row_acc_d.p, c->snap_rows.p, wb + 3 * sizeof(double), hipMemcpyDeviceToDevice,
                                     c->stream));
            ++c->replays;
            const int g = grow_lists(c, st);
            if (g == EAMFE_ENOMEM) {
                // the workspace is too small for the larger lists: hand the
                // chunk's starting state back (x, v; the work is held) and
                // stop there; the caller enlarges the workspace and resumes at
                // step b, where the lists are planned and built again exactly
                // as a replay here would have built them
                LCHK(c, launch_unpack(x, cur, c->N, c->stream));
                HIPCHK(c, hipStreamSynchronize(c->stream));
                c->have_list = false;
                c->resume_step = b;
                return g;
            }
            OK(g);
            OK(set_rebuild_all(c));
        }
    }
    LCHK(c, launch_unpack(x, cur, c->N, c->stream));
    return EAMFE_OK;
}

}  // namespace

extern "C" {

int run_switching(eamfe_ctx* c, const eamfe_protocol* p, int64_t s0, int64_t s1, double* x, double* v,
                  double* lam_out, double* dHdl_out, double* W_out, int sync)
{
    const bool has_eam = p && (p->mode == EAMFE_MODE_FL || p->mode == EAMFE_MODE_RS);
    if (!ready(c, has_eam)) return c ? EAMFE_ESTATE : EAMFE_EINVAL;
    if (check_protocol(p)) return fail(c, EAMFE_EINVAL, "run_switching: bad protocol");
    if (!x || !v) return fail(c, EAMFE_EINVAL, "run_switching: null x or v");
    (void)hipSetDevice(c->device);
    int64_t S = 0;
    c->resume_step = s0;   // nothing has run if the lambda table does not fit
    OK(ensure_lambda(c, p, &S));
    c->resume_step = -1;
    if (s0 < 0 || s1 <= s0 || s1 > S) return fail(c, EAMFE_EINVAL, "run_switching: bad step range");
    double c1 = 1.0;
    OK(set_thermostat(c, p, &c1));
    if (lam_out)
        HIPCHK(c, hipMemcpyAsync(lam_out, c->lam_d.p, (S + 1) * sizeof(double), hipMemcpyDeviceToDevice, c->stream));
    if (s0 == 0) HIPCHK(c, hipMemsetAsync(c->W_state_d.p, 0, (size_t)c->n_rep * sizeof(double), c->stream));
    OK(run_range(c, p, S, s0, s1, x, v, dHdl_out, W_out, S, 0, c1, has_eam));
    if (sync) return read_status(c);
    return EAMFE_OK;
}

int eamfe_set_chunk(eamfe_ctx* c, int64_t steps)
{
    if (!c || steps < 1) return EAMFE_EINVAL;
    c->chunk = steps;
    return EAMFE_OK;
}

int eamfe_replays(const eamfe_ctx* c, int64_t* n)
{
    if (!c || !n) return EAMFE_EINVAL;
    *n = c->replays;
    return EAMFE_OK;
}

int switch_step(eamfe_ctx* c, const eamfe_protocol* p, int64_t step, double* x, double* v, double* W, double* dHdl)
{
    const bool has_eam = p && (p->mode == EAMFE_MODE_FL || p->mode == EAMFE_MODE_RS);
    if (!ready(c, has_eam)) return c ? EAMFE_ESTATE : EAMFE_EINVAL;
    if (check_protocol(p) || !x || !v || !W) return fail(c, EAMFE_EINVAL, "switch_step: bad arguments");
    (void)hipSetDevice(c->device);
    int64_t S = 0;
    OK(ensure_lambda(c, p, &S));
    if (step < 0 || step >= S) return fail(c, EAMFE_EINVAL, "switch_step: step out of range");
    double c1 = 1.0;
    OK(set_thermostat(c, p, &c1));
    HIPCHK(c, hipMemcpyAsync(c->W_state_d.p, W, (size_t)c->n_rep * sizeof(double), hipMemcpyDeviceToDevice,
                             c->stream));
    // one-step trace: column (step - step) of a [n_rep][1] array
    OK(run_range(c, p, S, step, step + 1, x, v, dHdl, nullptr, 1, step, c1, has_eam));
    HIPCHK(c, hipMemcpyAsync(W, c->W_state_d.p, (size_t)c->n_rep * sizeof(double), hipMemcpyDeviceToDevice,
                             c->stream));
    return read_status(c);
}

int eamfe_get_work(eamfe_ctx* c, double* W)
{
    if (!ready(c, false) || !W) return c ? EAMFE_EINVAL : EAMFE_EINVAL;
    (void)hipSetDevice(c->device);
    HIPCHK(c, hipStreamSynchronize(c->stream));
    HIPCHK(c, hipMemcpy(W, c->W_state_d.p, (size_t)c->n_rep * sizeof(double), hipMemcpyDeviceToHost));
    return EAMFE_OK;
}

int eamfe_get_state(eamfe_ctx* c, double* W, double* xref, double* skin)
{
    if (!ready(c, false)) return c ? EAMFE_ESTATE : EAMFE_EINVAL;
    (void)hipSetDevice(c->device);
    HIPCHK(c, hipStreamSynchronize(c->stream));
    if (W) HIPCHK(c, hipMemcpy(W, c->W_state_d.p, (size_t)c->n_rep * sizeof(double), hipMemcpyDeviceToHost));
    if (xref) {
        if (!c->have_list) return fail(c, EAMFE_ESTATE, "get_state: no neighbour lists have been built");
        HIPCHK(c, hipMemcpy(xref, c->xref_d.p, (size_t)3 * c->N * sizeof(double), hipMemcpyDeviceToDevice));
    }
    if (skin) *skin = c->have_list ? c->skin : 0.0;
    return EAMFE_OK;
}

int eamfe_set_state(eamfe_ctx* c, const double* W, const double* xref, double skin)
{
    if (!ready(c, false)) return c ? EAMFE_ESTATE : EAMFE_EINVAL;
    (void)hipSetDevice(c->device);
    if (W) {
        HIPCHK(c, hipStreamSynchronize(c->stream));
        HIPCHK(c, hipMemcpy(c->W_state_d.p, W, (size_t)c->n_rep * sizeof(double), hipMemcpyHostToDevice));
    }
    if (xref) OK(neigh_build(c, xref, skin, 0));   // the rows a build at those positions gives
    return EAMFE_OK;
}

int eamfe_adjoint_theta(eamfe_ctx* c, const double* x, const double* w_host, int reduce, double* dtheta)
{
    if (!ready(c, true)) return c ? EAMFE_ESTATE : EAMFE_EINVAL;
    if (!x || !dtheta) return fail(c, EAMFE_EINVAL, "adjoint_theta: null argument");
    (void)hipSetDevice(c->device);
    return adjoint_theta_with(c, x, w_host, reduce, dtheta, nullptr, 0);
}

int eamfe_adjoint_theta_noalloc(eamfe_ctx* c, const double* x, const double* w_host, int reduce, double* dtheta)
{
    if (!ready(c, true)) return c ? EAMFE_ESTATE : EAMFE_EINVAL;
    if (!x || !dtheta) return fail(c, EAMFE_EINVAL, "adjoint_theta_noalloc: null argument");
    if (c->device < 0 || c->device >= kMaxDevices || !g_scratch_ptr[c->device])
        return fail(c, EAMFE_EDEVICE, "adjoint_theta_noalloc: no scratch address for this device");
    const size_t nb = (size_t)std::max(c->n_r, c->n_rho) - 1;
    const size_t bins = (size_t)c->n_rep * 3 * nb * 4 * sizeof(unsigned long long);
    const size_t fin = (size_t)(reduce ? 1 : c->n_rep) * 3 * 2 * (nb + 1) * sizeof(double);
    const size_t fin_off = (bins + 255) / 256 * 256;
    if (fin_off + fin > kNoAllocScratchBytes)
        return fail(c, EAMFE_EINVAL, "adjoint_theta_noalloc: needs " + std::to_string(fin_off + fin) +
                                         " bytes of scratch, more than its fixed " +
                                         std::to_string(kNoAllocScratchBytes) + " (fewer replicas or reduce = 1)");
    (void)hipSetDevice(c->device);
    char* base = (char*)g_scratch_ptr[c->device];
    c->no_alloc = true;   // the arena must already hold the lists: report EAMFE_ENOMEM rather than grow it
    const int rc = adjoint_theta_with(c, x, w_host, reduce, dtheta, base, fin_off);
    c->no_alloc = false;
    return rc;
}

int eamfe_set_adjoint_sampling(eamfe_ctx* c, int every, const double* w_host, int reduce, double* dtheta)
{
    if (!c || every < 0 || (every > 0 && !dtheta)) return EAMFE_EINVAL;
    c->adj_every = every;
    c->adj_reduce = reduce ? 1 : 0;
    c->adj_out = dtheta;
    if (w_host && c->n_rep) c->adj_w.assign(w_host, w_host + c->n_rep);
    else c->adj_w.clear();
    c->adj_samples = 0;
    return EAMFE_OK;
}

int eamfe_adjoint_samples(const eamfe_ctx* c, int64_t* n)
{
    if (!c || !n) return EAMFE_EINVAL;
    *n = c->adj_samples;
    return EAMFE_OK;
}

int eamfe_set_kernel_timing(eamfe_ctx* c, int stride, int kinds)
{
    if (!c || stride < 0 || kinds < 0 || kinds > 7) return EAMFE_EINVAL;
    c->timing = stride;
    c->timing_kinds = kinds ? kinds : 7;
    c->timing_seen = 0;
    c->ev_used = 0;
    c->ev_kind.clear();
    return EAMFE_OK;
}

int eamfe_kernel_timing(eamfe_ctx* c, double* ms_total, int64_t* launches)
{
    if (!c) return EAMFE_EINVAL;
    (void)hipSetDevice(c->device);
    HIPCHK(c, hipStreamSynchronize(c->stream));
    double t[3] = {0.0, 0.0, 0.0};
    int64_t n[3] = {0, 0, 0};
    for (size_t q = 0; q < c->ev_kind.size(); ++q) {
        float ms = 0.0f;
        HIPCHK(c, hipEventElapsedTime(&ms, c->ev_pool[2 * q], c->ev_pool[2 * q + 1]));
        t[c->ev_kind[q]] += ms;
        n[c->ev_kind[q]] += 1;
    }
    for (int k = 0; k < 3; ++k) {
        if (ms_total) ms_total[k] = t[k];
        if (launches) launches[k] = n[k];
    }
    c->ev_used = 0;
    c->ev_kind.clear();
    return EAMFE_OK;
}

int eamfe_autotune(eamfe_ctx* c, const eamfe_protocol* p, int64_t step, const double* x, const double* v,
                   int trial_steps, int* lanes_out, int* block_out, double* ms_per_step)
{
    const bool has_eam = p && (p->mode == EAMFE_MODE_FL || p->mode == EAMFE_MODE_RS);
    if (!ready(c, has_eam)) return c ? EAMFE_ESTATE : EAMFE_EINVAL;
    if (check_protocol(p) || !x || !v || trial_steps < 1) return fail(c, EAMFE_EINVAL, "autotune: bad arguments");
    (void)hipSetDevice(c->device);
    int64_t S = 0;
    OK(ensure_lambda(c, p, &S));
    if (step < 0 || step >= S) return fail(c, EAMFE_EINVAL, "autotune: step out of range");
    const int64_t s1 = std::min<int64_t>(S, step + 2 + trial_steps);
    const int64_t s2 = std::min<int64_t>(S, step + 2 + std::max<int64_t>(trial_steps, 100));
    const size_t v3 = 3 * (size_t)c->N * sizeof(double);
    HIPCHK(c, hipMemcpyAsync(c->tune_w.p, c->W_state_d.p, (size_t)c->n_rep * sizeof(double),
                             hipMemcpyDeviceToDevice, c->stream));
    const int timing = c->timing;
    c->timing = 0;
    const int lanes0 = c->lanes, block0 = c->block, grid0 = c->grid;
    int best_l = lanes0, best_b = block0, best_g = grid0;
    double best = 1e300;
    hipEvent_t e0, e1;
    HIPCHK(c, hipEventCreate(&e0));
    HIPCHK(c, hipEventCreate(&e1));
    int rc = EAMFE_OK;
    const int lanes_c[] = {1, 2, 4, 8, 16};
    const int block_c[] = {64, 128, 256, 512, 640, 768, 1024};
    const int grid_c[] = {0, c->n_cu, 2 * c->n_cu, 4 * c->n_cu};
    struct Cand {
        double per;
        int L, B, G;
    };
    std::vector<Cand> cands;   // every timed shape
    for (int L : lanes_c) {
        for (int B : block_c) {
          for (int G : grid_c) {
            if (B / L < 4) continue;   // at least four atoms per block
            c->lanes = L;
            c->block = B;
            c->grid = (G + 7) / 8 * 8;
            if ((rc = build_tiles(c))) goto done;
            if (hipMemcpyAsync(c->tune_x.p, x, v3, hipMemcpyDeviceToDevice, c->stream) ||
                hipMemcpyAsync(c->tune_v.p, v, v3, hipMemcpyDeviceToDevice, c->stream)) {
                rc = fail(c, EAMFE_EDEVICE, "autotune: copy failed");
                goto done;
            }
            if ((rc = run_switching(c, p, step, step + 2 <= s1 - 1 ? step + 2 : s1, (double*)c->tune_x.p,
                                    (double*)c->tune_v.p, nullptr, nullptr, nullptr, 0)))
                goto done;
            if (step + 2 < s1) {
                (void)hipEventRecord(e0, c->stream);
                if ((rc = run_switching(c, p, step + 2, s1, (double*)c->tune_x.p, (double*)c->tune_v.p, nullptr,
                                        nullptr, nullptr, 0)))
                    goto done;
                (void)hipEventRecord(e1, c->stream);
                (void)hipEventSynchronize(e1);
                float ms = 0.0f;
                (void)hipEventElapsedTime(&ms, e0, e1);
                const double per = ms / (double)(s1 - step - 2);
                cands.push_back({per, L, B, c->grid});
                if (per < best) {
                    best = per;
                    best_l = L;
                    best_b = B;
                    best_g = c->grid;
                }
            }
          }
        }
    }
    // second round: shapes within 4 % of the fastest trade places from run to
    // run on timing noise, so the (at most four) fastest within that margin are
    // timed again over three times the steps, and the fastest of that round wins
    if (!rc && cands.size() > 1) {
        std::sort(cands.begin(), cands.end(), [](const Cand& u, const Cand& w) { return u.per < w.per; });
        const int64_t s3 = std::min<int64_t>(S, step + 2 + 3 * (int64_t)trial_steps);
        if (step + 2 < s3) {
            double best2 = 1e300;
            for (size_t q = 0; q < cands.size() && q < 4 && cands[q].per <= cands[0].per * 1.04; ++q) {
                c->lanes = cands[q].L;
                c->block = cands[q].B;
                c->grid = cands[q].G;
                if ((rc = build_tiles(c))) goto done;
                if (hipMemcpyAsync(c->tune_x.p, x, v3, hipMemcpyDeviceToDevice, c->stream) ||
                    hipMemcpyAsync(c->tune_v.p, v, v3, hipMemcpyDeviceToDevice, c->stream)) {
                    rc = fail(c, EAMFE_EDEVICE, "autotune: copy failed");
                    goto done;
                }
                if ((rc = run_switching(c, p, step, step + 2, (double*)c->tune_x.p, (double*)c->tune_v.p, nullptr,
                                        nullptr, nullptr, 0)))
                    goto done;
                (void)hipEventRecord(e0, c->stream);
                if ((rc = run_switching(c, p, step + 2, s3, (double*)c->tune_x.p, (double*)c->tune_v.p, nullptr,
                                        nullptr, nullptr, 0)))
                    goto done;
                (void)hipEventRecord(e1, c->stream);
                (void)hipEventSynchronize(e1);
                float ms = 0.0f;
                (void)hipEventElapsedTime(&ms, e0, e1);
                const double per = ms / (double)(s3 - step - 2);
                if (per < best2) {
                    best2 = per;
                    best = per;
                    best_l = cands[q].L;
                    best_b = cands[q].B;
                    best_g = cands[q].G;
                }
            }
        }
    }
    // at the chosen shape, the list builder: rows from LDS or from global memory
    // (identical rows; the faster depends on how many atoms a step rebuilds, so
    // this trial spans at least 100 steps, to s2)
    if (!rc && has_eam && step + 2 < s2) {
        c->lanes = best_l;
        c->block = best_b;
        c->grid = best_g;
        if ((rc = build_tiles(c))) goto done;
        const int lds0 = c->lds_rows;
        double t_b[2] = {1e300, 1e300};
        for (int lds = 0; lds < 2; ++lds) {
            c->lds_rows = lds;
            c->have_list = false;
            if (hipMemcpyAsync(c->tune_x.p, x, v3, hipMemcpyDeviceToDevice, c->stream) ||
                hipMemcpyAsync(c->tune_v.p, v, v3, hipMemcpyDeviceToDevice, c->stream)) {
                rc = fail(c, EAMFE_EDEVICE, "autotune: copy failed");
                break;
            }
            if ((rc = run_switching(c, p, step, step + 2, (double*)c->tune_x.p, (double*)c->tune_v.p, nullptr,
                                    nullptr, nullptr, 0)))
                break;
            (void)hipEventRecord(e0, c->stream);
            if ((rc = run_switching(c, p, step + 2, s2, (double*)c->tune_x.p, (double*)c->tune_v.p, nullptr, nullptr,
                                    nullptr, 0)))
                break;
            (void)hipEventRecord(e1, c->stream);
            (void)hipEventSynchronize(e1);
            float ms = 0.0f;
            (void)hipEventElapsedTime(&ms, e0, e1);
            t_b[lds] = ms / (double)(s2 - step - 2);
        }
        c->lds_rows = rc ? lds0 : (t_b[1] <= t_b[0] ? 1 : 0);
    }
done:
    // the lists now follow a trial's positions: plan and build them again at
    // the caller's (at the chosen shape and builder), as a pass would on
    // finding none, so the caller's next pass starts from valid lists
    c->have_list = false;
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    c->timing = timing;
    c->lanes = rc ? lanes0 : best_l;
    c->block = rc ? block0 : best_b;
    c->grid = rc ? grid0 : best_g;
    {
        const int r2 = build_tiles(c);
        if (!rc) rc = r2;
    }
    if (!rc && has_eam) rc = neigh_build(c, x, p->skin, 0);
    (void)hipMemcpyAsync(c->W_state_d.p, c->tune_w.p, (size_t)c->n_rep * sizeof(double), hipMemcpyDeviceToDevice,
                         c->stream);
    (void)hipStreamSynchronize(c->stream);
    if (rc) return rc;
    if (lanes_out) *lanes_out = best_l;
    if (block_out) *block_out = best_b;
    if (ms_per_step) *ms_per_step = best;
    return read_status(c);
}

int eamfe_copy_lists(eamfe_ctx* c, int32_t* nnb_dev, int32_t* nbr_dev, int cap)
{
    if (!c || !nnb_dev) return EAMFE_EINVAL;
    if (!c->have_list) return fail(c, EAMFE_ESTATE, "no neighbour lists");
    if (nbr_dev && cap < c->cap) return fail(c, EAMFE_EINVAL, "copy_lists: capacity smaller than the rows'");
    (void)hipSetDevice(c->device);
    HIPCHK(c, hipMemcpyAsync(nnb_dev, c->nnb_d.p, (size_t)c->N * sizeof(int32_t), hipMemcpyDeviceToDevice,
                             c->stream));
    if (nbr_dev)
        LCHK(c, launch_rows_rowmajor((const int32_t*)c->nbr_d.p, (const int32_t*)c->nnb_d.p, c->N, c->cap, nbr_dev,
                                     cap, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    return EAMFE_OK;
}

__global__ void k_list_stats(const int32_t* nnb, int n, unsigned long long* out)
{
    unsigned long long s = 0, mx = 0;
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
        s += (unsigned long long)nnb[i];
        mx = nnb[i] > (int)mx ? (unsigned long long)nnb[i] : mx;
    }
    atomicAdd(&out[0], s);
    atomicMax(&out[1], mx);
}

int eamfe_row_history(eamfe_ctx* c, double* mean_len, int64_t* passes, int reset)
{
    if (!ready(c, false)) return c ? EAMFE_ESTATE : EAMFE_EINVAL;
    (void)hipSetDevice(c->device);
    std::vector<double> h(c->n_rep + 1);
    HIPCHK(c, hipMemcpyAsync(h.data(), c->row_acc_d.p, h.size() * sizeof(double), hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    double sum = 0.0;
    for (int r = 0; r < c->n_rep; ++r) sum += h[r];
    const double n = h[c->n_rep];
    if (mean_len) *mean_len = n > 0.0 ? sum / (n * c->N) : 0.0;
    if (passes) *passes = (int64_t)n;
    if (reset) HIPCHK(c, hipMemsetAsync(c->row_acc_d.p, 0, (h.size() + 2) * sizeof(double), c->stream));
    return EAMFE_OK;
}

int eamfe_list_rebuilds(eamfe_ctx* c, int64_t* replica_rebuilds, int64_t* atoms_rebuilt)
{
    if (!ready(c, false)) return c ? EAMFE_ESTATE : EAMFE_EINVAL;
    (void)hipSetDevice(c->device);
    double h[2];
    HIPCHK(c, hipMemcpyAsync(h, (const double*)c->row_acc_d.p + c->n_rep + 1, sizeof(h), hipMemcpyDeviceToHost,
                             c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    if (replica_rebuilds) *replica_rebuilds = (int64_t)h[0];
    if (atoms_rebuilt) *atoms_rebuilt = (int64_t)h[1];
    return EAMFE_OK;
}

int eamfe_pressure(eamfe_ctx* c, const double* x, const double* v, double* P)
{
    if (!ready(c, true)) return c ? EAMFE_ESTATE : EAMFE_EINVAL;
    if (!x || !P) return fail(c, EAMFE_EINVAL, "pressure: null argument");
    (void)hipSetDevice(c->device);
    OK(pack(c, x));
    OK(ensure_lists(c, c->have_list ? c->skin : 0.3, PA(c)));
    for (int attempt = 0;; ++attempt) {
        NeighArgs na = neigh_args(c, PA(c));
        LCHK(c, launch_neigh_rebuild(na, step_args(c), c->lanes, c->block, c->stream));
        StepArgs a = step_args(c);
        a.P = PA(c);
        a.Pn = nullptr;
        a.Q = QA(c);
        a.Qn = nullptr;
        a.v = const_cast<double*>(v);
        a.has_eam = 1;
        a.step_kernel = 0;
        a.mode = EAMFE_MODE_FL;
        a.vir_part = (double*)c->vir_d.p;
        LCHK(c, launch_density(a, c->precision, c->lanes, c->block, c->stream));
        LCHK(c, launch_force(a, c->precision, c->lanes, c->block, c->stream));
        LCHK(c, launch_finish(a, c->stream));
        HIPCHK(c, hipStreamSynchronize(c->stream));
        int st = 0;
        HIPCHK(c, hipMemcpy(&st, c->status_d.p, sizeof(int), hipMemcpyDeviceToHost));
        if (!(st & (ST_NEIGH_OVERFLOW | ST_CELL_OVERFLOW)) || attempt >= 6) break;
        HIPCHK(c, hipMemset(c->status_d.p, 0, sizeof(int)));
        OK(grow_lists(c, st));
        OK(set_rebuild_all(c));
        ++c->replays;
    }
    std::vector<double> part((size_t)c->n_tiles * 3);
    HIPCHK(c, hipMemcpy(part.data(), c->vir_d.p, part.size() * sizeof(double), hipMemcpyDeviceToHost));
    for (int r = 0; r < c->n_rep; ++r) {   // each replica's units in order
        const RepDesc& R = c->reps[r];
        const double V = R.L[0] * R.L[1] * R.L[2];
        for (int k = 0; k < 3; ++k) {
            double s = 0.0;
            for (int t = 0; t < R.n_tiles; ++t) s += part[(size_t)(R.tile_base + t) * 3 + k];
            P[3 * r + k] = s / V;
        }
    }
    return read_status(c);
}

int eamfe_barostat_step(eamfe_ctx* c, const eamfe_barostat* b, int64_t step, double w_eam, double* x, double* v,
                        double* mu_out, double* P_out)
{
    if (!ready(c, true)) return c ? EAMFE_ESTATE : EAMFE_EINVAL;
    if (!b || !x || !v) return fail(c, EAMFE_EINVAL, "barostat_step: null argument");
    if (!(b->tau_p > 0.0) || !(b->beta_T >= 0.0) || !(b->dt >= 0.0) || !std::isfinite(b->p0) ||
        !std::isfinite(w_eam) || (b->aniso != 0 && b->aniso != 1))
        return fail(c, EAMFE_EINVAL,
                    "barostat_step: need tau_p > 0, beta_T >= 0, dt >= 0, finite p0 and w_eam, aniso 0 or 1");
    (void)hipSetDevice(c->device);
    // configurational pressure tensor of U_EAM at x (virial only), then the
    // kinetic part from the velocities: P_aa = (sum m v_a^2 + w_eam W_aa) / V
    // is the internal pressure of H = w_eam U_EAM along axis a
    std::vector<double> Pc((size_t)c->n_rep * 3);
    OK(eamfe_pressure(c, x, nullptr, Pc.data()));
    // each replica's sum of v_a^2 per axis on the device (three numbers per
    // replica cross to the host, not the velocities)
    std::vector<double> kin((size_t)c->n_rep * 3);
    LCHK(c, launch_kinetic(v, (const RepDesc*)c->reps_d.p, c->n_rep, c->N, (double*)c->mu_d.p, c->stream));
    HIPCHK(c, hipMemcpyAsync(kin.data(), c->mu_d.p, kin.size() * sizeof(double), hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    const double rl = c->r_cut + c->skin;
    std::vector<double> mu((size_t)c->n_rep * 3), Pint((size_t)c->n_rep * 3);
    for (int r = 0; r < c->n_rep; ++r) {
        const RepDesc& R = c->reps[r];
        const double V = R.L[0] * R.L[1] * R.L[2];
        const double kT = kB * R.T;
        double Paa[3];
        for (int d = 0; d < 3; ++d) {
            const double mv2 = kin[3 * (size_t)r + d];
            Paa[d] = (mv2 * R.mass * mvv2e + w_eam * Pc[3 * r + d] * V) / V;
            Pint[3 * r + d] = Paa[d];
        }
        double z[3];
        barostat_gauss3(R.seed, 0u, step, 3u, z);
        if (b->aniso) {
            // each edge on its own: eps_a = ln L_a with its own diagonal pressure
            const double amp = std::sqrt(2.0 * kT * b->beta_T * b->dt / (3.0 * V * b->tau_p));
            for (int d = 0; d < 3; ++d)
                mu[3 * r + d] = std::exp(-(b->beta_T / (3.0 * b->tau_p)) * (b->p0 - Paa[d] - kT / V) * b->dt +
                                         amp * z[d]);
        } else {
            const double P = (Paa[0] + Paa[1] + Paa[2]) / 3.0;
            const double deps = -(b->beta_T / b->tau_p) * (b->p0 - P - kT / V) * b->dt +
                                std::sqrt(2.0 * kT * b->beta_T * b->dt / (V * b->tau_p)) * z[0];
            mu[3 * r] = mu[3 * r + 1] = mu[3 * r + 2] = std::exp(deps / 3.0);
        }
        for (int d = 0; d < 3; ++d)
            if (!(R.L[d] * mu[3 * r + d] > 2.0 * rl))
                return fail(c, EAMFE_EBOX, "barostat_step: box edge of replica " + std::to_string(r) +
                                               " would fall to 2 (r_cut + skin) or below");
    }
    for (int r = 0; r < c->n_rep; ++r) {
        RepDesc& R = c->reps[r];
        for (int d = 0; d < 3; ++d) {
            R.L[d] *= mu[3 * r + d];
            R.invL[d] = 1.0 / R.L[d];
        }
    }
    HIPCHK(c, hipMemcpy(c->mu_d.p, mu.data(), mu.size() * sizeof(double), hipMemcpyHostToDevice));
    LCHK(c, launch_rescale(x, v, (const int32_t*)c->rep_of_d.p, (const double*)c->mu_d.p, c->N, c->stream));
    OK(upload_reps(c));
    drop_graphs(c);
    c->have_list = false;   // cells and rows are planned again for the new boxes by the next pass
    HIPCHK(c, hipStreamSynchronize(c->stream));
    if (mu_out) std::copy(mu.begin(), mu.end(), mu_out);
    if (P_out) std::copy(Pint.begin(), Pint.end(), P_out);
    return EAMFE_OK;
}

int eamfe_get_boxes(const eamfe_ctx* c, double* L)
{
    if (!c || !L) return EAMFE_EINVAL;
    for (int r = 0; r < c->n_rep; ++r)
        for (int d = 0; d < 3; ++d) L[3 * r + d] = c->reps[r].L[d];
    return EAMFE_OK;
}

int eamfe_set_spring_scale(eamfe_ctx* c, const double* s)
{
    if (!ready(c, false)) return c ? EAMFE_ESTATE : EAMFE_EINVAL;
    (void)hipSetDevice(c->device);
    drop_graphs(c);   // captured launches hold the old argument
    if (!s) {
        c->has_kscale = false;
        return EAMFE_OK;
    }
    HIPCHK(c, hipMemcpyAsync(c->kscale_d.p, s, (size_t)c->N * sizeof(double), hipMemcpyDeviceToDevice, c->stream));
    c->has_kscale = true;
    return EAMFE_OK;
}

int eamfe_msd(eamfe_ctx* c, const double* x, double* msd)
{
    if (!ready(c, false)) return c ? EAMFE_ESTATE : EAMFE_EINVAL;
    if (!x || !msd) return fail(c, EAMFE_EINVAL, "msd: null argument");
    (void)hipSetDevice(c->device);
    LCHK(c, launch_msd(x, (const double*)c->x0_d.p, (const RepDesc*)c->reps_d.p, c->n_rep, c->N, (double*)c->msd_d.p,
                       c->stream));
    HIPCHK(c, hipMemcpyAsync(msd, c->msd_d.p, (size_t)c->n_rep * sizeof(double), hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    return EAMFE_OK;
}

int eamfe_list_stats(eamfe_ctx* c, double* mean_len, int* max_len, int* capacity)
{
    if (!c) return EAMFE_EINVAL;
    if (!c->have_list) return fail(c, EAMFE_ESTATE, "no neighbour lists");
    (void)hipSetDevice(c->device);
    HIPCHK(c, hipMemsetAsync(c->stats_d.p, 0, 2 * sizeof(unsigned long long), c->stream));
    hipLaunchKernelGGL(k_list_stats, dim3(256), dim3(256), 0, c->stream, (const int32_t*)c->nnb_d.p, c->N,
                       (unsigned long long*)c->stats_d.p);
    HIPCHK(c, hipGetLastError());
    unsigned long long h[2];
    HIPCHK(c, hipMemcpyAsync(h, c->stats_d.p, sizeof(h), hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    if (mean_len) *mean_len = (double)h[0] / c->N;
    if (max_len) *max_len = (int)h[1];
    if (capacity) *capacity = c->cap;
    return EAMFE_OK;
}

// ---- estimators -------------------------------------------------------------
double eamfe_spring_constant(double msd, double T)
{
    return msd > 0.0 ? 3.0 * kB * T / msd : 0.0;
}

double eamfe_einstein_free_energy(double n_eff, double T, double k, double mass)
{
    const double omega = std::sqrt(k / (mass * mvv2e));
    return 3.0 * n_eff * kB * T * std::log(hbar * omega / (kB * T));
}

double eamfe_fixed_cm_correction(double N, double V, double T, double k)
{
    return kB * T * std::log(N / V * std::pow(2.0 * M_PI * kB * T / (N * k), 1.5));
}

int eamfe_fl_free_energy(int n, const double* Wf, const double* Wb, double n_eff, double N, double V, double T,
                         double k, double mass, int add_cm, double* F0, double* Ediss, double* err)
{
    if (n < 1 || !Wf || !Wb) return EAMFE_EINVAL;
    double mf = 0.0, mb = 0.0;
    for (int i = 0; i < n; ++i) {
        mf += Wf[i];
        mb += Wb[i];
    }
    mf /= n;
    mb /= n;
    // Eq. W12 with 1 = H0 and 2 = H_E: F_E - F0 = (W_fwd - W_bwd)/2
    const double dF = 0.5 * (mf - mb);
    double F = eamfe_einstein_free_energy(n_eff, T, k, mass) - dF;
    if (add_cm) F += eamfe_fixed_cm_correction(N, V, T, k);
    if (F0) *F0 = F;
    if (Ediss) *Ediss = 0.5 * (mf + mb);
    if (err) {
        double var = 0.0;
        for (int i = 0; i < n; ++i) {
            const double d = 0.5 * (Wf[i] - Wb[i]) - dF;
            var += d * d;
        }
        *err = n > 1 ? std::sqrt(var / (n - 1) / n) : NAN;
    }
    return EAMFE_OK;
}

int eamfe_jarzynski(int n, const double* W, double T, double* dF, double* err)
{
    if (n < 1 || !W || !(T > 0.0)) return EAMFE_EINVAL;
    const double b = 1.0 / (kB * T);
    double m = -INFINITY;   // shift: the largest exponent
    for (int i = 0; i < n; ++i) m = std::max(m, -b * W[i]);
    double s = 0.0;
    for (int i = 0; i < n; ++i) s += std::exp(-b * W[i] - m);
    const double mean = s / n;
    if (dF) *dF = -(m + std::log(mean)) / b;
    if (err) {
        double var = 0.0;
        for (int i = 0; i < n; ++i) {
            const double d = std::exp(-b * W[i] - m) - mean;
            var += d * d;
        }
        *err = n > 1 ? std::sqrt(var / (n - 1)) / (std::sqrt((double)n) * mean * b) : NAN;
    }
    return EAMFE_OK;
}

int eamfe_switch_works(const eamfe_protocol* p, int n_rep, const double* W, int64_t stride, double* Wf, double* Wb)
{
    if (check_protocol(p) || n_rep < 1 || !W || !Wf || !Wb || p->n_sw < 1) return EAMFE_EINVAL;
    const int64_t e0 = p->n_eq, e1 = p->n_eq + p->n_sw;
    const int64_t b0 = e1 + p->n_hold, b1 = b0 + p->n_sw;
    if (stride < b1) return EAMFE_EINVAL;
    for (int r = 0; r < n_rep; ++r) {
        const double* w = W + (size_t)r * stride;
        Wf[r] = w[e1 - 1] - (e0 > 0 ? w[e0 - 1] : 0.0);
        Wb[r] = w[b1 - 1] - w[b0 - 1];
    }
    return EAMFE_OK;
}

int eamfe_rs_free_energy(const eamfe_protocol* p, const double* W, double F0_T0, double T0, double n_eff, int n_T,
                         const double* T_grid, double* F_out)
{
    if (check_protocol(p) || !W || n_T < 1 || !T_grid || !F_out) return EAMFE_EINVAL;
    const int64_t n_eq = p->n_eq, n_sw = p->n_sw, b0 = p->n_eq + p->n_sw + p->n_hold;
    const double Tf = T0 / p->lambda_f;
    // cumulative work after q forward (backward) steps, q = 0..n_sw
    auto fwd = [&](int64_t q) { return q == 0 ? 0.0 : W[n_eq + q - 1] - (n_eq ? W[n_eq - 1] : 0.0); };
    auto bwd = [&](int64_t q) { return q == 0 ? 0.0 : W[b0 + q - 1] - W[b0 - 1]; };
    auto interp = [&](auto&& g, double pos) {
        if (pos <= 0.0) return g(0);
        if (pos >= (double)n_sw) return g(n_sw);
        const int64_t q = (int64_t)std::floor(pos);
        const double w = pos - q;
        return (1.0 - w) * g(q) + w * g(q + 1);
    };
    const double wb_total = bwd(n_sw);
    for (int k = 0; k < n_T; ++k) {
        const double T = T_grid[k];
        if (!(T >= T0 * (1 - 1e-12) && T <= Tf * (1 + 1e-12))) return EAMFE_EINVAL;
        const double lam = T0 / T;
        const double tau = (T - T0) / (Tf - T0);
        const double w1 = interp(fwd, tau * n_sw);                         // W_{1 -> lambda}
        const double w2 = wb_total - interp(bwd, (1.0 - tau) * n_sw);      // W_{lambda -> 1}
        F_out[k] = F0_T0 / lam + 1.5 * n_eff * kB * T0 * std::log(lam) / lam + (w1 - w2) / (2.0 * lam);
    }
    return EAMFE_OK;
}

int eamfe_rs_free_energy_cm(const eamfe_protocol* p, const double* W, double F0_T0, double T0, double N, double V,
                            double mass, int n_T, const double* T_grid, double* F_out)
{
    if (!(N > 1.0) || !(V > 0.0) || !(mass > 0.0)) return EAMFE_EINVAL;
    // c(T): free crystal minus the crystal with its centre of mass held
    auto c_of = [&](double T) {
        const double kT = kB * T;
        const double lam_dB = std::sqrt(2.0 * M_PI * hbar * hbar / (mass * mvv2e * kT));
        return -kT * std::log(V / N) + 3.0 * kT * std::log(lam_dB);
    };
    const int st = eamfe_rs_free_energy(p, W, F0_T0 - c_of(T0), T0, N - 1.0, n_T, T_grid, F_out);
    if (st != EAMFE_OK) return st;
    for (int q = 0; q < n_T; ++q) F_out[q] += c_of(T_grid[q]);
    return EAMFE_OK;
}

}  // extern "C"
