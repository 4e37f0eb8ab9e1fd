// engine.hip -- host side of the DPD engine: parameter checks, workspace
// layout, launch sequences and the C ABI declared in include/dpd.h.
//
// A handle holds one system or a batch of independent replicas.  The replicas'
// particles, cells and tiles are concatenated (replica r owns a contiguous
// range of each), so the per-step kernels (cell-count scan, scatter, pair
// kernel) cover the whole batch in one launch each.  A single system is the
// one-replica case and uses the kernels that take its parameters by value.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <algorithm>
#include <cstring>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "../../include/dpd.h"
#include "kernels.h"

using namespace dpd;

// Device scratch of dpd_forces_noalloc: the workspace of a one-system handle,
// for callers that cannot allocate device memory.  Every device the library
// runs on holds its own copy until the process ends.  In host code the name
// is not a device address: the address comes from hipGetSymbolAddress, per
// device (noalloc_scratch below).
constexpr size_t kNoAllocScratchBytes = size_t(32) << 20;
static __device__ __align__(256) unsigned char scratch[kNoAllocScratchBytes];

namespace {

thread_local std::string g_last_error = "no error";

struct Layout {
    size_t off_Sx, off_Sv, off_SF, off_Sid;
    size_t off_Ax, off_Au, off_Aid, off_Bx, off_Bu, off_Bid;
    size_t off_key, off_rank, off_src, off_count, off_cs;
    size_t off_scan, off_red, off_Fs, off_binacc, off_status, off_ovf;
    size_t off_count2, off_xref, off_rec, off_flags;  // second counter array; Verlet skin
    size_t off_reps, off_tile_rep, off_stepb;         // batch tables, graph step
    size_t off_Tx, off_Tv, off_TF, off_Tid;           // state saved by the tuner
    size_t off_posid, off_posid2;                     // input index by id (far bonds), per buffer
    size_t total;
};

// One replica: its parameters and derived launch constants.
struct Rep {
    dpd_params p;
    DevParams P;
};

// The whole handle: replicas, totals and the workspace layout.
struct Derived {
    std::vector<Rep> reps;
    long long N = 0, cells = 0, tiles = 0;
    long long tiles_alloc = 0;  // capacity of the per-tile arrays
    int n_scan_blocks = 0;      // chunks of the cell-count scan
    int bin_M_max = 0;
    bool skin = false;
    bool far_bond = false;  // some replica's bond can reach beyond the cell stencil
    Layout lay;
};

size_t align256(size_t x) { return (x + 255) & ~size_t(255); }

constexpr uint64_t kProfEvery = 8;  // pair launches per profiled launch

std::string fmt(const char* f, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, f);
    vsnprintf(buf, sizeof buf, f, ap);
    va_end(ap);
    return buf;
}

// Tile tx x ty cells (clamped so that a tile and its halo do not wrap onto
// themselves: side <= n_c - 2) and the constants the pair kernel derives from it.
void set_tiling(DevParams& P, int tx, int ty) {
    P.tile_x = std::max(1, std::min(tx, P.nc - 2));
    P.tile_y = std::max(1, std::min(ty, P.nc - 2));
    P.ntx = (P.nc + P.tile_x - 1) / P.tile_x;
    P.nty = (P.nc + P.tile_y - 1) / P.tile_y;
    const int w_full = P.tile_x + 2, w_last = (P.nc - (P.ntx - 1) * P.tile_x) + 2;
    P.wmul_full = (65536 + w_full - 1) / w_full;
    P.wmul_last = (65536 + w_last - 1) / w_last;
    // (tile + 1/2) / ntx lies at least 1/(2 ntx) >= 2^-17 from an integer, far
    // beyond the 2^-21 error of the product for tile < 2^31
    P.inv_ntx = 1.0 / (double)P.ntx;
}

// A tile schedule: the same tile sides for every replica (tx, ty >= 1), or
// each replica's own default tile scaled by f (tx == 0); and the tile order.
struct Sched {
    int tx, ty;
    double f;
    int order;
};

// The schedules the tuner times.
const Sched kCandidates[] = {
    {0, 0, 1.0, 0}, {0, 0, 0.85, 0}, {0, 0, 0.7, 0}, {0, 0, 0.55, 0},
    {8, 7, 0.0, 0}, {8, 8, 0.0, 0}, {6, 6, 0.0, 0}, {4, 4, 0.0, 0},
};

// Finer tilings the tuner may give single replicas of a batch whose tiles
// still overflow under the candidates above (dense clusters).
const Sched kRefine[] = {{0, 0, 0.4, 0}, {0, 0, 0.3, 0}};

// Default tile of a system, scaled by f.  Without a skin the sides shrink as
// 1 / (particles per cell): a tile then keeps about as many pairs as 8 x 7
// cells at one particle per cell (the kept pairs of a tile grow as its
// particles times the density, and must fit the pair list in LDS).  With a
// skin they shrink as 1 / sqrt(particles per cell), which keeps the staged
// particles (the records hold the pairs to r_c + skin).
void default_tile(const dpd_params& p, const DevParams& P, double f, int* tx, int* ty) {
    const double cell_n = std::max((double)P.N / ((double)P.nc * P.nc), 1.0 / 16.0);
    const double sc = p.skin > 0.0f ? std::sqrt(cell_n) : cell_n;
    *tx = std::max(1, std::min(kTileMax, (int)std::lround(kTileX * f / sc)));
    *ty = std::max(1, std::min(kTileMax, (int)std::lround(kTileY * f / sc)));
}

void apply_tiling(Rep& r, const Sched& s) {
    int tx = s.tx, ty = s.ty;
    if (tx <= 0) default_tile(r.p, r.P, s.f, &tx, &ty);
    set_tiling(r.P, tx, ty);
}

long long tiles_with(Rep r, const Sched& s) {
    apply_tiling(r, s);
    return (long long)r.P.ntx * r.P.nty;
}

// Validate the parameters of one system and derive its launch constants.
int derive_one(const dpd_params* p, DevParams& P, std::string* err) {
    if (!p) { *err = "params is NULL"; return DPD_EINVAL; }
    if (p->n_agents < 1 || p->n_agents > (int64_t(1) << 29)) {
        *err = fmt("n_agents = %lld outside [1, 2^29]", (long long)p->n_agents);
        return DPD_EINVAL;
    }
    auto finite = [](double v) { return std::isfinite(v); };
    if (!finite(p->L) || !finite(p->r_c) || !(p->r_c > 0.0) || !(p->L > 0.0)) {
        *err = "L and r_c must be finite and positive";
        return DPD_EINVAL;
    }
    if ((double)(float)p->L != p->L) {
        *err = fmt("L = %.17g is not exactly representable in FP32", p->L);
        return DPD_EINVAL;
    }
    if (!std::isfinite((double)p->skin) || p->skin < 0.0f || (double)p->skin > 0.5 * p->L) {
        *err = "skin must be finite, >= 0 and below L / 2";
        return DPD_EINVAL;
    }
    // smallest cell width: the cutoff plus the skin.  A bond that can reach
    // beyond the 3 x 3 stencil (1.25 bond_l, a quarter of stretch to spare,
    // wider than a cell) has its partner read by id instead.
    const double width = p->r_c + (double)p->skin;
    const double ncd = std::floor(p->L / width);
    if (!(ncd >= 3.0)) {
        *err = "L must be at least 3 (r_c + skin) (n_c >= 3)";
        return DPD_EINVAL;
    }
    if (ncd > 46340.0) { *err = "too many cells (n_c^2 must fit in int32)"; return DPD_EINVAL; }
    if (p->skin > 0.0f && 1.25 * p->bond_l > width) {
        *err = "a Verlet skin needs 1.25 bond_l <= r_c + skin (the bond within the cell stencil)";
        return DPD_EINVAL;
    }
    const double vals[] = {p->A, p->gamma, p->kT, p->kappa, p->bond_l, p->gamma_s};
    for (double v : vals)
        if (!finite(v) || v < 0.0) {
            *err = "A, gamma, kT, kappa, bond_l, gamma_s must be finite and >= 0";
            return DPD_EINVAL;
        }
    if (!finite(p->f_sp)) { *err = "f_sp must be finite"; return DPD_EINVAL; }
    if (!finite(p->mass) || !(p->mass > 0.0) || !finite(p->dt) || !(p->dt > 0.0)) {
        *err = "mass and dt must be finite and positive";
        return DPD_EINVAL;
    }
    if (p->noise_kind != 0 && p->noise_kind != 1) { *err = "noise_kind must be 0 or 1"; return DPD_EINVAL; }
    if (p->rng_kind != 0 && p->rng_kind != 1) { *err = "rng_kind must be 0 or 1"; return DPD_EINVAL; }
    if (p->sp_split != 0 && p->sp_split != 1) { *err = "sp_split must be 0 or 1"; return DPD_EINVAL; }
    if (p->bin_M_max < 0 || p->bin_M_max > 8192) { *err = "bin_M_max must be in [0, 8192]"; return DPD_EINVAL; }
    if (p->tile < 0 || p->tile > kTileMax) { *err = fmt("tile must be in [0, %d]", kTileMax); return DPD_EINVAL; }
    if (!std::isfinite((double)p->w_exp) || p->w_exp < 0.0f || p->w_exp > 8.0f) {
        *err = "w_exp must be in [0, 8] (0: 2)";
        return DPD_EINVAL;
    }

    P = DevParams{};
    P.N = (int)(2 * p->n_agents);
    P.nc = (int)ncd;
    P.n_cells = P.nc * P.nc;
    int tx = p->tile, ty = p->tile;
    if (!p->tile) default_tile(*p, P, 1.0, &tx, &ty);
    set_tiling(P, tx, ty);
    P.noise_kind = p->noise_kind;
    P.rng_kind = p->rng_kind;
    P.L = (float)p->L;
    P.halfL = (float)(0.5 * p->L);
    P.rc = (float)p->r_c;
    P.rc2 = (float)(p->r_c * p->r_c);
    P.inv_rc = (float)(1.0 / p->r_c);
    P.A = (float)p->A;
    P.gamma = (float)p->gamma;
    P.sigma_rdt = (float)(std::sqrt(2.0 * p->gamma * p->kT) / std::sqrt(p->dt));
    P.kappa = (float)p->kappa;
    P.bond_l = (float)p->bond_l;
    {
        const double l2 = (double)P.bond_l * (double)P.bond_l;
        P.bond_l2_hi = (float)l2;
        P.bond_l2_lo = (float)(l2 - (double)P.bond_l2_hi);
    }
    P.sp_head = (float)(p->sp_split == 0 ? 0.5 * p->f_sp : p->f_sp);
    P.sp_tail = (float)(p->sp_split == 0 ? 0.5 * p->f_sp : 0.0);
    P.gamma_s = (float)p->gamma_s;
    P.h = (float)(p->dt / (2.0 * p->mass));
    P.L_d = p->L;
    P.dt_d = p->dt;
    P.inv_w = (double)P.nc / p->L;
    P.skin_on = p->skin > 0.0f ? 1 : 0;
    {
        // pairs listed up to r_c + skin (rounded up); a rebuild once some particle
        // is more than skin / 2 from its rebuild position (rounded down)
        const double lr = p->r_c + (double)p->skin;
        P.list_rc2 = (float)(lr * lr * (1.0 + 1e-6));
        const double hs = 0.5 * (double)p->skin;
        P.half_skin2 = (float)(hs * hs * (1.0 - 1e-6));
    }
    P.seed_lo = (uint32_t)(p->seed & 0xffffffffu);
    P.seed_hi = (uint32_t)(p->seed >> 32);
    P.mass_d = p->mass;
    P.w_half = p->w_exp > 0.0f ? 0.5f * p->w_exp : 1.0f;
    P.far_bond = (1.25 * p->bond_l > width) ? 1 : 0;
    return DPD_OK;
}

// Offsets of every replica in the concatenated particle, cell and tile arrays.
void assign_offsets(Derived* d) {
    long long pb = 0, cb = 0, tb = 0;
    for (Rep& r : d->reps) {
        r.P.pbase = (int)pb;
        r.P.cbase = (int)cb;
        r.P.tbase = (int)tb;
        pb += r.P.N;
        cb += r.P.n_cells;
        tb += (long long)r.P.ntx * r.P.nty;
    }
    d->N = pb;
    d->cells = cb;
    d->tiles = tb;
}

// Validate n_rep parameter sets and lay out the workspace for them.
int derive(const dpd_params* p, int n_rep, Derived* d, std::string* err) {
    if (!p) { *err = "params is NULL"; return DPD_EINVAL; }
    if (n_rep < 1 || n_rep > 65536) { *err = fmt("n_rep = %d outside [1, 65536]", n_rep); return DPD_EINVAL; }
    d->reps.assign(n_rep, Rep{});
    int bin_M_max = 0;
    for (int r = 0; r < n_rep; ++r) {
        std::string e;
        int rc = derive_one(p + r, d->reps[r].P, &e);
        if (rc) {
            *err = n_rep > 1 ? fmt("replica %d: %s", r, e.c_str()) : e;
            return rc;
        }
        d->reps[r].p = p[r];
        bin_M_max = std::max(bin_M_max, p[r].bin_M_max ? p[r].bin_M_max : 256);
        if (n_rep > 1 && p[r].skin > 0.0f) {
            *err = "a batch of replicas runs without a Verlet skin (skin must be 0)";
            return DPD_EINVAL;
        }
    }
    d->skin = d->reps[0].P.skin_on != 0;
    d->far_bond = false;
    for (const Rep& r : d->reps) d->far_bond |= r.P.far_bond != 0;
    assign_offsets(d);
    if (d->N > (int64_t(1) << 30) || d->cells > 2147483647LL) {
        *err = "the batch holds more than 2^30 particles or 2^31 cells";
        return DPD_EINVAL;
    }
    // the per-tile arrays hold the tiles of any schedule the tuner may choose
    long long ta = 0;
    for (const Rep& r : d->reps) {
        long long t = (long long)r.P.ntx * r.P.nty;
        for (const Sched& c : kCandidates) t = std::max(t, tiles_with(r, c));
        if (d->reps.size() > 1)
            for (const Sched& c : kRefine) t = std::max(t, tiles_with(r, c));
        ta += t;
    }
    if (d->skin) ta = d->tiles;  // the skin keeps the tiling it was created with
    d->tiles_alloc = ta;
    const long long scan_tile = (long long)kScanThreads * 4 * scan_rows(d->cells);
    d->n_scan_blocks = (int)((d->cells + scan_tile - 1) / scan_tile);
    d->bin_M_max = bin_M_max;

    const size_t N = (size_t)d->N, C = (size_t)d->cells, T = (size_t)d->tiles_alloc;
    Layout& L = d->lay;
    size_t o = 0;
    auto take = [&](size_t bytes) { size_t r = o; o = align256(o + bytes); return r; };
    L.off_Sx = take(N * 8);
    L.off_Sv = take(N * 8);
    L.off_SF = take(N * 8);
    L.off_Sid = take(N * 4);
    L.off_Ax = take(N * 8);
    L.off_Au = take(N * 8);
    L.off_Aid = take(N * 4);
    L.off_Bx = take(N * 8);
    L.off_Bu = take(N * 8);
    L.off_Bid = take(N * 4);
    L.off_key = take(N * 4);
    L.off_rank = take(N * 4);
    L.off_src = take(N * 4);
    L.off_count = take(C * 4);
    L.off_count2 = take(C * 4);
    L.off_cs = take((C + 1) * 4);
    L.off_red = take((T + kRedParts) * 3 * 8);  // per tile, then per part
    L.off_Fs = take(N * 8);
    L.off_binacc = take((size_t)d->bin_M_max * d->bin_M_max * 3 * 8);
    L.off_status = take(16);
    L.off_ovf = take((T + 1) * 4);
    L.off_scan = take(((size_t)d->n_scan_blocks + 1) * 8);  // chunk descriptors, ticket counter
    L.off_flags = take(64);  // two displacement flags (by step parity), rebuild count
    L.off_stepb = take(64);
    L.off_reps = take((size_t)n_rep * sizeof(DevParams));
    L.off_tile_rep = take(n_rep > 1 ? T * 4 : 4);
    if (d->skin) {
        L.off_xref = take(N * 8);
        L.off_rec = take(T * kRecStride);
        L.off_Tx = L.off_Tv = L.off_TF = L.off_Tid = 0;
    } else {
        L.off_xref = L.off_rec = 0;
        L.off_Tx = take(N * 8);
        L.off_Tv = take(N * 8);
        L.off_TF = take(N * 8);
        L.off_Tid = take(N * 4);
    }
    L.off_posid = d->far_bond ? take(N * 4) : 0;
    L.off_posid2 = d->far_bond ? take(N * 4) : 0;
    L.total = o;
    return DPD_OK;
}

inline int grid_for(long long n, int block = kBlock) { return (int)((n + block - 1) / block); }

// A captured chunk of steps, replayed by dpd_step.
struct Graph {
    int K;
    bool reduce_last;
    hipGraphExec_t exec;
};

}  // namespace

struct dpd_handle {
    Derived d;
    int R;  // replicas
    hipStream_t stream;
    char* ws;
    float2 *Sx, *Sv, *SF, *Ax, *Au, *Bx, *Bu, *Fs;
    int *Sid, *Aid, *Bid, *key, *rank, *src, *count, *cs;
    float2 *Tx, *Tv, *TF;
    int* Tid;
    unsigned* status;
    int* ovf;  // [0]: count of tiles left to the overflow kernel, then their indices
    unsigned long long* scan_desc;  // per chunk of the cell scan, then its ticket counter
    // second counter array (see counter_of); Verlet skin: rebuild positions,
    // tile records, flags
    int* count2;
    float2* xref;
    unsigned char* rec;
    int* flags;
    double* red;
    long long* binacc;
    DevParams* reps_dev;  // parameters of every replica (batch)
    int* tile_rep;        // replica of every tile (batch)
    unsigned* stepb;      // step before a replayed chunk
    int* posid;           // input index by id (far bonds), or null: for buffers A and the
                          // inputs of the calls that bin S
    int* posid2;          // the same for buffers B
    int tile_order;       // 0: bands of tiles per XCD; 1: launch order
    int64_t step;
    bool have_state;
    // the last dpd_step also made the next step's half kick and drift (and its
    // cell counts); the next dpd_step starts from these buffers
    bool prepared;
    float2 *prep_x, *prep_u;
    int* prep_id;
    std::string err;
    bool profiling;
    std::vector<hipEvent_t> ev_start, ev_stop;
    size_t ev_used;
    double prof_ms;
    int64_t prof_n;
    uint64_t prof_seq;
    // steps replayed from captured graphs, in chunks of graph_chunk steps
    int graph_chunk;
    hipStream_t cap_stream;
    std::vector<Graph> graphs;
};

namespace {

int fail(dpd_handle* h, int code, const std::string& msg) {
    if (h) h->err = msg;
    g_last_error = msg;
    return code;
}

#define HIPCHK(h, expr)                                                              \
    do {                                                                             \
        hipError_t e_ = (expr);                                                      \
        if (e_ != hipSuccess)                                                        \
            return fail((h), DPD_EHIP, fmt("%s: %s", #expr, hipGetErrorString(e_))); \
    } while (0)

#define LAUNCHCHK(h)                                                                       \
    do {                                                                                   \
        hipError_t e_ = hipGetLastError();                                                 \
        if (e_ != hipSuccess)                                                              \
            return fail((h), DPD_EHIP, fmt("kernel launch: %s", hipGetErrorString(e_)));  \
    } while (0)

const DevParams& P0(const dpd_handle* h) { return h->d.reps[0].P; }

void drop_graphs(dpd_handle* h) {
    if (h->graphs.empty()) return;
    (void)hipStreamSynchronize(h->stream);  // no replay may still be in flight
    for (Graph& g : h->graphs) (void)hipGraphExecDestroy(g.exec);
    h->graphs.clear();
}

// Upload the replica table and the tile -> replica map (batches only).
int upload_tables(dpd_handle* h) {
    if (h->R == 1) return DPD_OK;
    std::vector<DevParams> P(h->R);
    std::vector<int> tr((size_t)h->d.tiles);
    for (int r = 0; r < h->R; ++r) {
        P[r] = h->d.reps[r].P;
        const long long t0 = P[r].tbase, nt = (long long)P[r].ntx * P[r].nty;
        for (long long t = 0; t < nt; ++t) tr[(size_t)(t0 + t)] = r;
    }
    HIPCHK(h, hipMemcpyAsync(h->reps_dev, P.data(), P.size() * sizeof(DevParams),
                             hipMemcpyHostToDevice, h->stream));
    HIPCHK(h, hipMemcpyAsync(h->tile_rep, tr.data(), tr.size() * 4, hipMemcpyHostToDevice,
                             h->stream));
    HIPCHK(h, hipStreamSynchronize(h->stream));  // the host vectors go out of scope
    return DPD_OK;
}

// cell_start from count (count cleared) and the slot -> input map.  Within a
// cell the slots are in arrival order; the pair kernel places each cell's
// members by id itself.  With id_of_input != NULL every cell is also ordered by
// id here (only for the state loaded with a given force, which no pair kernel
// passes through before it is stored).  With pos != NULL (far bonds) the map
// from id to input index of the binned buffers is written there; the stepping
// path passes NULL, since its buffers carry maps written by the kernels that
// wrote them (pos_of_buffer).
int bin_from_counts(dpd_handle* h, int* count, bool clear, const int* rebuild, int* moved_clear,
                    const int* id_of_input, const int* ids_in, int* pos) {
    const int G = h->d.n_scan_blocks;
    const int C = (int)h->d.cells, N = (int)h->d.N;
    auto scan = scan_rows(C) == 1 ? k_scan<1> : k_scan<4>;
    hipLaunchKernelGGL(scan, dim3(G), dim3(kScanThreads), 0, h->stream, count, C, clear ? 1 : 0,
                       h->cs, h->scan_desc,
                       h->scan_desc + G, h->status, h->ovf, rebuild, moved_clear, h->flags + 2);
    hipLaunchKernelGGL(k_scatter, dim3(std::min(grid_for(N), 4096)), dim3(kBlock), 0, h->stream,
                       N, (const int*)h->key, (const int*)h->rank, (const int*)h->cs, h->src,
                       rebuild);
    if (id_of_input)
        hipLaunchKernelGGL(k_cell_sort, dim3(grid_for(C)), dim3(kBlock), 0, h->stream, C,
                           (const int*)h->cs, h->src, id_of_input);
    if (pos)  // bonds beyond the stencil: where every id sits in the input
        hipLaunchKernelGGL(k_pos_of_id, dim3(std::min(grid_for(N), 4096)), dim3(kBlock), 0, h->stream,
                           N, ids_in, h->R > 1 ? (const DevParams*)h->reps_dev : nullptr, h->R,
                           pos, rebuild);
    LAUNCHCHK(h);
    return DPD_OK;
}

// Per-cell counter array of step s.  With a Verlet skin the two arrays
// alternate by step parity: step s fills the one for the keys of x_{s+1} while
// the other, consumed by the binning of step s, is cleared tile by tile.
int* counter_of(dpd_handle* h, int64_t s) {
    return (s & 1) ? h->count2 : h->count;
}

// Without a skin each array belongs to one of the ping-pong position buffers:
// the launch that writes positions into A fills `count`, into B `count2`.  A
// step's binning consumes the array of its input buffer without clearing it;
// its pair launch clears that array tile by tile while it fills the other.
// Whenever no step is prepared both arrays are zero.
int* counter_of_buffer(dpd_handle* h, const float2* x) {
    return x == h->Ax ? h->count : h->count2;
}

// Far bonds: the id -> index map of stepping buffers A or B (null without far
// bonds).  Whatever writes one of these buffers on the stepping path
// (k_kick_drift, the pair kernels) writes its map too, so the stepping
// binnings build none.
int* pos_of_buffer(dpd_handle* h, const float2* x) {
    return x == h->Ax ? h->posid : h->posid2;
}

template <int MODE, bool SKIN, bool BATCH>
void launch_pair_kernel(dpd_handle* h, const PairArgs& b, int reduce) {
    const int G = (int)h->d.tiles;
    hipLaunchKernelGGL((k_pair<MODE, SKIN, BATCH>), dim3(G), dim3(kWave), 0, h->stream, P0(h), b,
                       reduce);
}

template <int MODE, bool BATCH>
void launch_overflow(dpd_handle* h, const PairArgs& b, int reduce) {
    // tiles over an LDS capacity (dense clusters), if any
    const int Go = (int)std::min<long long>(h->d.tiles, 512);
    if (h->d.skin)  // tile records of a skin hold the small capacities only
        hipLaunchKernelGGL((k_pair_overflow<MODE, BATCH, false>), dim3(Go), dim3(kWave), 0, h->stream,
                           P0(h), b, reduce);
    else
        hipLaunchKernelGGL((k_pair_overflow<MODE, BATCH, true>), dim3(Go), dim3(kWave), 0, h->stream,
                           P0(h), b, reduce);
}

int launch_pair(dpd_handle* h, int mode, const PairArgs& a, bool reduce) {
    size_t ev = 0;
    // with profiling on, every kProfEvery-th launch is bracketed by events (an
    // event record between two kernels costs a few microseconds of GPU time)
    const bool timed = h->profiling && (h->prof_seq++ % kProfEvery == 0);
    if (timed) {
        if (h->ev_used == h->ev_start.size()) {
            hipEvent_t e0, e1;
            HIPCHK(h, hipEventCreate(&e0));
            HIPCHK(h, hipEventCreate(&e1));
            h->ev_start.push_back(e0);
            h->ev_stop.push_back(e1);
        }
        ev = h->ev_used++;
        HIPCHK(h, hipEventRecord(h->ev_start[ev], h->stream));
    }
    PairArgs b = a;
    b.ovf_count = h->ovf;
    b.ovf_list = h->ovf + 1;
    b.reps = h->reps_dev;
    b.tile_rep = h->tile_rep;
    b.nt_total = (int)h->d.tiles;
    b.tile_order = h->tile_order;
    if (!b.pos_of_id) b.pos_of_id = h->posid;
    const int red = reduce ? 1 : 0;
    const bool batch = h->R > 1;
    // the Verlet-skin variant of the kernel only where a skin is set (a force
    // evaluation alone keeps no record)
    const bool skin = h->d.skin && mode != MODE_FORCES;
    if (batch) {
        if (mode == MODE_STEP) launch_pair_kernel<MODE_STEP, false, true>(h, b, red);
        else if (mode == MODE_FINAL) launch_pair_kernel<MODE_FINAL, false, true>(h, b, red);
        else launch_pair_kernel<MODE_FORCES, false, true>(h, b, 0);
    } else if (mode == MODE_STEP && skin) {
        launch_pair_kernel<MODE_STEP, true, false>(h, b, red);
    } else if (mode == MODE_STEP) {
        launch_pair_kernel<MODE_STEP, false, false>(h, b, red);
    } else if (mode == MODE_FINAL && skin) {
        launch_pair_kernel<MODE_FINAL, true, false>(h, b, red);
    } else if (mode == MODE_FINAL) {
        launch_pair_kernel<MODE_FINAL, false, false>(h, b, red);
    } else {
        launch_pair_kernel<MODE_FORCES, false, false>(h, b, 0);
    }
    LAUNCHCHK(h);
    if (timed) {
        HIPCHK(h, hipEventRecord(h->ev_stop[ev], h->stream));
        if (h->ev_used >= 256) {  // fold the recorded pairs into the totals
            HIPCHK(h, hipEventSynchronize(h->ev_stop[ev]));
            for (size_t k = 0; k < h->ev_used; ++k) {
                float ms = 0.f;
                HIPCHK(h, hipEventElapsedTime(&ms, h->ev_start[k], h->ev_stop[k]));
                h->prof_ms += ms;
                h->prof_n += 1;
            }
            h->ev_used = 0;
        }
    }
    if (batch) {
        if (mode == MODE_STEP) launch_overflow<MODE_STEP, true>(h, b, red);
        else if (mode == MODE_FINAL) launch_overflow<MODE_FINAL, true>(h, b, red);
        else launch_overflow<MODE_FORCES, true>(h, b, 0);
    } else {
        if (mode == MODE_STEP) launch_overflow<MODE_STEP, false>(h, b, red);
        else if (mode == MODE_FINAL) launch_overflow<MODE_FINAL, false>(h, b, red);
        else launch_overflow<MODE_FORCES, false>(h, b, 0);
    }
    LAUNCHCHK(h);
    return DPD_OK;
}

// FP64 (P_x, P_y, KE) of every replica from the per-tile partials of the last
// pair launch, into out[3 r .. 3 r + 2].
int launch_reduce(dpd_handle* h, double* out) {
    if (h->R == 1) {
        const int parts = (int)std::min<long long>(kRedParts, h->d.tiles);
        double* part = h->red + 3 * (size_t)h->d.tiles_alloc;
        hipLaunchKernelGGL(k_reduce_part, dim3(parts), dim3(kBlock), 0, h->stream,
                           (const double*)h->red, (int)h->d.tiles, part);
        hipLaunchKernelGGL(k_reduce_final, dim3(1), dim3(kBlock), 0, h->stream, (const double*)part,
                           parts, h->d.reps[0].p.mass, out);
    } else {
        hipLaunchKernelGGL(k_reduce_reps, dim3(h->R), dim3(kBlock), 0, h->stream,
                           (const double*)h->red, (const DevParams*)h->reps_dev, out);
    }
    LAUNCHCHK(h);
    return DPD_OK;
}

int read_status(dpd_handle* h) {
    unsigned st[4] = {0, 0, 0, 0};
    HIPCHK(h, hipStreamSynchronize(h->stream));
    HIPCHK(h, hipMemcpy(st, h->status, sizeof st, hipMemcpyDeviceToHost));
    if (st[0]) {
        const unsigned zero[4] = {0, 0, 0, 0};
        HIPCHK(h, hipMemcpy(h->status, zero, sizeof zero, hipMemcpyHostToDevice));
    }
    if (st[0] & kStatusNonFinite)
        return fail(h, DPD_ENONFINITE, "a non-finite position, velocity or force appeared");
    if (st[0] & kStatusBond)
        return fail(h, DPD_EBOND, "a bonded partner was farther than one cell width");
    if (st[0] & kStatusRange)
        return fail(h, DPD_ERANGE, "a velocity exceeded the range of the binned field");
    if (st[0] & kStatusBinning)
        return fail(h, DPD_EHIP, "internal error: cell counts inconsistent with the particle count");
    if (st[0] & kStatusScan)
        return fail(h, DPD_EHIP, "internal error: the cell scan waited too long for a chunk's sum");
    return DPD_OK;
}

// Drop the prepared next step (its cell counts are cleared so that the next
// binning starts from zero).
int unprepare(dpd_handle* h) {
    if (!h->prepared) return DPD_OK;
    const long long C = h->d.cells;
    hipLaunchKernelGGL(k_fill_i32, dim3(grid_for(C)), dim3(kBlock), 0, h->stream, h->count, 0, C);
    hipLaunchKernelGGL(k_fill_i32, dim3(grid_for(C)), dim3(kBlock), 0, h->stream, h->count2, 0, C);
    LAUNCHCHK(h);
    h->prepared = false;
    return DPD_OK;
}

// First half kick and drift of a dpd_step call from the stored state, into the
// A buffers (with a skin this step rebuilds).
int kick_drift(dpd_handle* h) {
    int* count = h->d.skin ? counter_of(h, h->step) : counter_of_buffer(h, h->Ax);
    for (const Rep& r : h->d.reps) {
        const DevParams& P = r.P;
        const size_t pb = (size_t)P.pbase;
        hipLaunchKernelGGL(k_kick_drift, dim3(grid_for(P.N)), dim3(kBlock), 0, h->stream, P,
                           (const float2*)(h->Sx + pb), (const float2*)(h->Sv + pb),
                           (const float2*)(h->SF + pb), (const int*)(h->Sid + pb), h->Ax + pb,
                           h->Au + pb, h->Aid + pb, h->key + pb, h->rank + pb, count, h->status,
                           h->posid);
    }
    if (h->d.skin)
        hipLaunchKernelGGL(k_fill_i32, dim3(1), dim3(kBlock), 0, h->stream, h->flags + (h->step & 1),
                           1, 1LL);
    LAUNCHCHK(h);
    h->prepared = true;
    h->prep_x = h->Ax;
    h->prep_u = h->Au;
    h->prep_id = h->Aid;
    return DPD_OK;
}

// The arguments of the pair launch of step s = h->step + k of a run that
// starts from the prepared buffers (in, out alternate; the last step stores
// the state and prepares the next one).
PairArgs step_args(dpd_handle* h, int64_t k, bool last, float2* inx, float2* inu, int* inid,
                   float2* outx, float2* outu, int* outid) {
    const int64_t s = h->step + k;
    PairArgs a = {};
    a.cs = h->cs;
    a.src = h->src;
    a.xin = inx;
    a.uin = inu;
    a.idin = inid;
    a.status = h->status;
    a.red = h->red;
    a.step = (uint32_t)((uint64_t)s & 0xffffffffu);
    a.keyout = h->key;
    a.rankout = h->rank;
    if (h->d.skin) {
        a.count = counter_of(h, s);
        a.rebuild = h->flags + ((s - 1) & 1);
        a.rec = h->rec;
        a.xref = h->xref;
        a.moved = h->flags + (s & 1);
        a.count_clear = counter_of(h, s - 1);
    } else {
        a.count = counter_of_buffer(h, outx);
        a.count_clear = counter_of_buffer(h, inx);
        a.pos_of_id = pos_of_buffer(h, inx);
        a.pos_out = pos_of_buffer(h, outx);
    }
    if (last) {
        a.xout = h->Sx;
        a.uout = h->Sv;
        a.idout = h->Sid;
        a.Fout = h->SF;
        a.pxout = outx;
        a.puout = outu;
        a.pidout = outid;
    } else {
        a.xout = outx;
        a.uout = outu;
        a.idout = outid;
    }
    return a;
}

// n >= 1 steps from the prepared buffers, launched one by one.  Records of
// (P_x, P_y, KE) per replica are taken at the steps k0 + k that are multiples
// of reduce_every, into pk_out + 3 R *rec.
int run_steps(dpd_handle* h, int64_t n, int reduce_every, double* pk_out, int64_t k0, int64_t* rec) {
    float2 *inx = h->prep_x, *inu = h->prep_u;
    int* inid = h->prep_id;
    const bool in_a = (inx == h->Ax);
    float2* outx = in_a ? h->Bx : h->Ax;
    float2* outu = in_a ? h->Bu : h->Au;
    int* outid = in_a ? h->Bid : h->Aid;
    for (int64_t k = 1; k <= n; ++k) {
        // forces of step s = step + k: the binning consumes the keys of x_s
        // (counters of step s - 1) if this step rebuilds
        const int64_t s = h->step + k;
        const int* rebuild = h->d.skin ? h->flags + ((s - 1) & 1) : nullptr;
        int* moved = h->d.skin ? h->flags + (s & 1) : nullptr;
        int* counts = h->d.skin ? counter_of(h, s - 1) : counter_of_buffer(h, inx);
        int rc = bin_from_counts(h, counts, h->d.skin, rebuild, moved, nullptr, inid, nullptr);
        if (rc) return rc;
        const bool last = (k == n);
        const bool red = pk_out && reduce_every > 0 && ((k0 + k) % reduce_every == 0);
        const PairArgs a = step_args(h, k, last, inx, inu, inid, outx, outu, outid);
        rc = launch_pair(h, last ? MODE_FINAL : MODE_STEP, a, red);
        if (rc) return rc;
        if (red) {
            rc = launch_reduce(h, pk_out + 3 * (size_t)h->R * (size_t)(*rec));
            if (rc) return rc;
            ++*rec;
        }
        std::swap(inx, outx);
        std::swap(inu, outu);
        std::swap(inid, outid);
    }
    // the last launch left the next step's start in what is now `in`
    h->prep_x = inx;
    h->prep_u = inu;
    h->prep_id = inid;
    h->step += n;
    return DPD_OK;
}

// Capture K steps (K even, prepared buffers in A, step numbers read from
// *stepb) into a graph; with reduce_last the last pair launch also writes the
// per-tile partials of the FP64 sums.  The chunk ends with the next step
// prepared in A again and *stepb advanced by K.
int capture_chunk(dpd_handle* h, int K, bool reduce_last, hipGraphExec_t* out) {
    if (!h->cap_stream) HIPCHK(h, hipStreamCreateWithFlags(&h->cap_stream, hipStreamNonBlocking));
    hipStream_t user = h->stream;
    h->stream = h->cap_stream;
    hipGraph_t graph = nullptr;
    hipError_t e = hipStreamBeginCapture(h->cap_stream, hipStreamCaptureModeThreadLocal);
    if (e != hipSuccess) {
        h->stream = user;
        return fail(h, DPD_EHIP, fmt("hipStreamBeginCapture: %s", hipGetErrorString(e)));
    }
    int rc = DPD_OK;
    float2 *inx = h->Ax, *inu = h->Au, *outx = h->Bx, *outu = h->Bu;
    int *inid = h->Aid, *outid = h->Bid;
    for (int k = 1; k <= K && rc == DPD_OK; ++k) {
        rc = bin_from_counts(h, counter_of_buffer(h, inx), false, nullptr, nullptr, nullptr, inid, nullptr);
        if (rc) break;
        const bool last = (k == K);
        PairArgs a = step_args(h, k, last, inx, inu, inid, outx, outu, outid);
        a.step = (uint32_t)k;
        a.step_base = h->stepb;
        rc = launch_pair(h, last ? MODE_FINAL : MODE_STEP, a, last && reduce_last);
        std::swap(inx, outx);
        std::swap(inu, outu);
        std::swap(inid, outid);
    }
    if (rc == DPD_OK) {
        hipLaunchKernelGGL(k_add_u32, dim3(1), dim3(64), 0, h->cap_stream, h->stepb, (unsigned)K);
        e = hipGetLastError();
        if (e != hipSuccess) rc = fail(h, DPD_EHIP, fmt("kernel launch: %s", hipGetErrorString(e)));
    }
    e = hipStreamEndCapture(h->cap_stream, &graph);
    h->stream = user;
    if (rc) {
        if (graph) (void)hipGraphDestroy(graph);
        return rc;
    }
    if (e != hipSuccess) return fail(h, DPD_EHIP, fmt("hipStreamEndCapture: %s", hipGetErrorString(e)));
    e = hipGraphInstantiate(out, graph, nullptr, nullptr, 0);
    (void)hipGraphDestroy(graph);
    if (e != hipSuccess) return fail(h, DPD_EHIP, fmt("hipGraphInstantiate: %s", hipGetErrorString(e)));
    return DPD_OK;
}

// Copy the stored state (S) to the tuner's save area, or back.
int copy_state(dpd_handle* h, bool save) {
    const size_t N = (size_t)h->d.N;
    void* S[4] = {h->Sx, h->Sv, h->SF, h->Sid};
    void* T[4] = {h->Tx, h->Tv, h->TF, h->Tid};
    const size_t bytes[4] = {N * 8, N * 8, N * 8, N * 4};
    for (int k = 0; k < 4; ++k)
        HIPCHK(h, hipMemcpyAsync(save ? T[k] : S[k], save ? S[k] : T[k], bytes[k],
                                 hipMemcpyDeviceToDevice, h->stream));
    return DPD_OK;
}

// Bin the stored state S again (nothing prepared): after S was copied back
// from the tuner's save area, cell_start holds a later binning.  S is in the
// slot order of the binning of its own positions, which this repeats, so the
// cell list read with S (dpd_get_cells, the row binning of velocities) matches
// it again.
int rebin_stored(dpd_handle* h) {
    for (const Rep& r : h->d.reps) {
        const size_t pb = (size_t)r.P.pbase;
        hipLaunchKernelGGL(k_key_rank, dim3(grid_for(r.P.N)), dim3(kBlock), 0, h->stream, r.P,
                           (const float2*)h->Sx + pb, h->key + pb, h->rank + pb, h->count);
    }
    LAUNCHCHK(h);
    return bin_from_counts(h, h->count, true, nullptr, nullptr, nullptr, h->Sid, h->posid);
}

// The handle's replicas under schedule s (tile sides clamped per replica).
Derived with_schedule(const Derived& d, const Sched& s) {
    Derived nd = d;
    for (Rep& r : nd.reps) apply_tiling(r, s);
    assign_offsets(&nd);
    return nd;
}

// Apply a tile schedule to every replica.
int apply_schedule(dpd_handle* h, const Sched& s) {
    Derived nd = with_schedule(h->d, s);
    if (nd.tiles > h->d.tiles_alloc)
        return fail(h, DPD_EINVAL, fmt("tile %d x %d needs %lld tiles, the workspace holds %lld", s.tx,
                                       s.ty, nd.tiles, h->d.tiles_alloc));
    drop_graphs(h);
    h->d = nd;
    h->tile_order = s.order;
    return upload_tables(h);
}

}  // namespace

namespace {

// Device address of `scratch` on the current device, looked up once per
// device with that device current.
int noalloc_scratch(void** out) {
    constexpr int kMaxDevices = 64;
    static std::mutex mu;
    static void* ptr[kMaxDevices] = {};
    int dev = -1;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess)
        return fail(nullptr, DPD_EHIP, fmt("hipGetDevice: %s", hipGetErrorString(e)));
    if (dev < 0 || dev >= kMaxDevices)
        return fail(nullptr, DPD_EHIP, fmt("device %d outside [0, %d)", dev, kMaxDevices));
    std::lock_guard<std::mutex> lock(mu);
    if (!ptr[dev]) {
        void* p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p)
            return fail(nullptr, DPD_EHIP,
                        fmt("hipGetSymbolAddress(scratch): %s", hipGetErrorString(e)));
        ptr[dev] = p;
    }
    *out = ptr[dev];
    return DPD_OK;
}

}  // namespace

extern "C" {

int dpd_batch_workspace_bytes(const dpd_params* p, int32_t n_rep, size_t* bytes) {
    try {
        Derived d;
        std::string err;
        int rc = derive(p, n_rep, &d, &err);
        if (rc) return fail(nullptr, rc, err);
        if (!bytes) return fail(nullptr, DPD_EINVAL, "bytes is NULL");
        *bytes = d.lay.total;
        return DPD_OK;
    } catch (...) {
        return fail(nullptr, DPD_EINVAL, "internal error");
    }
}

int dpd_workspace_bytes(const dpd_params* p, size_t* bytes) {
    return dpd_batch_workspace_bytes(p, 1, bytes);
}

int64_t dpd_cells_per_side(const dpd_params* p) {
    DevParams P;
    std::string err;
    int rc = derive_one(p, P, &err);
    if (rc) return fail(nullptr, rc, err);
    return P.nc;
}

int dpd_create_batch(const dpd_params* p, int32_t n_rep, void* workspace, size_t bytes,
                     void* stream, dpd_handle** out) {
    try {
        if (!out) return fail(nullptr, DPD_EINVAL, "out is NULL");
        *out = nullptr;
        Derived d;
        std::string err;
        int rc = derive(p, n_rep, &d, &err);
        if (rc) return fail(nullptr, rc, err);
        if (!workspace || ((uintptr_t)workspace & 255u))
            return fail(nullptr, DPD_EWORKSPACE, "workspace is NULL or not 256-byte aligned");
        if (bytes < d.lay.total)
            return fail(nullptr, DPD_EWORKSPACE,
                        fmt("workspace has %zu bytes, needs %zu", bytes, d.lay.total));
        dpd_handle* h = new (std::nothrow) dpd_handle();
        if (!h) return fail(nullptr, DPD_EINVAL, "out of host memory");
        h->d = d;
        h->R = n_rep;
        h->stream = (hipStream_t)stream;
        h->ws = (char*)workspace;
        const Layout& L = d.lay;
        char* w = h->ws;
        h->Sx = (float2*)(w + L.off_Sx);
        h->Sv = (float2*)(w + L.off_Sv);
        h->SF = (float2*)(w + L.off_SF);
        h->Sid = (int*)(w + L.off_Sid);
        h->Ax = (float2*)(w + L.off_Ax);
        h->Au = (float2*)(w + L.off_Au);
        h->Aid = (int*)(w + L.off_Aid);
        h->Bx = (float2*)(w + L.off_Bx);
        h->Bu = (float2*)(w + L.off_Bu);
        h->Bid = (int*)(w + L.off_Bid);
        h->key = (int*)(w + L.off_key);
        h->rank = (int*)(w + L.off_rank);
        h->src = (int*)(w + L.off_src);
        h->count = (int*)(w + L.off_count);
        h->cs = (int*)(w + L.off_cs);
        h->red = (double*)(w + L.off_red);
        h->Fs = (float2*)(w + L.off_Fs);
        h->binacc = (long long*)(w + L.off_binacc);
        h->status = (unsigned*)(w + L.off_status);
        h->ovf = (int*)(w + L.off_ovf);
        h->scan_desc = (unsigned long long*)(w + L.off_scan);
        h->flags = (int*)(w + L.off_flags);
        h->stepb = (unsigned*)(w + L.off_stepb);
        h->reps_dev = (DevParams*)(w + L.off_reps);
        h->tile_rep = (int*)(w + L.off_tile_rep);
        h->count2 = (int*)(w + L.off_count2);
        h->xref = d.skin ? (float2*)(w + L.off_xref) : nullptr;
        h->rec = d.skin ? (unsigned char*)(w + L.off_rec) : nullptr;
        h->Tx = d.skin ? nullptr : (float2*)(w + L.off_Tx);
        h->Tv = d.skin ? nullptr : (float2*)(w + L.off_Tv);
        h->TF = d.skin ? nullptr : (float2*)(w + L.off_TF);
        h->Tid = d.skin ? nullptr : (int*)(w + L.off_Tid);
        h->posid = d.far_bond ? (int*)(w + L.off_posid) : nullptr;
        h->posid2 = d.far_bond ? (int*)(w + L.off_posid2) : nullptr;
        h->tile_order = 0;
        h->step = 0;
        h->have_state = false;
        h->prepared = false;
        h->prep_x = h->prep_u = nullptr;
        h->prep_id = nullptr;
        h->err = "no error";
        h->profiling = false;
        h->ev_used = 0;
        h->prof_ms = 0.0;
        h->prof_n = 0;
        h->prof_seq = 0;
        h->graph_chunk = 0;
        h->cap_stream = nullptr;
        // clear the counters the kernels rely on
        const long long C = d.cells;
        hipLaunchKernelGGL(k_fill_i32, dim3(grid_for(C)), dim3(kBlock), 0, h->stream, h->count, 0, C);
        hipLaunchKernelGGL(k_fill_i32, dim3(grid_for(C)), dim3(kBlock), 0, h->stream, h->count2, 0, C);
        hipLaunchKernelGGL(k_fill_i32, dim3(1), dim3(kBlock), 0, h->stream, (int*)h->status, 0, 4LL);
        hipLaunchKernelGGL(k_fill_i32, dim3(1), dim3(kBlock), 0, h->stream, h->ovf, 0, 1LL);
        hipLaunchKernelGGL(k_fill_i32, dim3(1), dim3(kBlock), 0, h->stream, h->flags, 0, 16LL);
        const long long scan_words = 2LL * (d.n_scan_blocks + 1);
        hipLaunchKernelGGL(k_fill_i32, dim3(grid_for(scan_words)), dim3(kBlock), 0, h->stream,
                           (int*)h->scan_desc, 0, scan_words);
        if (d.skin) {
            // no tile record is valid before the first rebuild
            const long long words = d.tiles_alloc * (long long)(kRecStride / 4);
            hipLaunchKernelGGL(k_fill_i32, dim3(grid_for(words)), dim3(kBlock), 0, h->stream,
                               (int*)h->rec, 0, words);
        }
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) {
            std::string m = fmt("kernel launch: %s", hipGetErrorString(e));
            delete h;
            return fail(nullptr, DPD_EHIP, m);
        }
        rc = upload_tables(h);
        if (rc) {
            std::string m = h->err;
            delete h;
            return fail(nullptr, rc, m);
        }
        *out = h;
        return DPD_OK;
    } catch (...) {
        return fail(nullptr, DPD_EINVAL, "internal error");
    }
}

int dpd_create(const dpd_params* p, void* workspace, size_t bytes, void* stream,
               dpd_handle** out) {
    return dpd_create_batch(p, 1, workspace, bytes, stream, out);
}

void dpd_destroy(dpd_handle* h) {
    if (!h) return;
    drop_graphs(h);
    if (h->cap_stream) (void)hipStreamDestroy(h->cap_stream);
    for (auto e : h->ev_start) (void)hipEventDestroy(e);
    for (auto e : h->ev_stop) (void)hipEventDestroy(e);
    delete h;
}

const char* dpd_last_error(const dpd_handle* h) {
    return h ? h->err.c_str() : g_last_error.c_str();
}

int dpd_set_state(dpd_handle* h, const float* x, const float* v, int64_t step, const float* F) {
    if (!h) return fail(nullptr, DPD_EINVAL, "handle is NULL");
    if (!x || !v) return fail(h, DPD_EINVAL, "x and v must not be NULL");
    try {
        int rc0 = unprepare(h);
        if (rc0) return rc0;
        for (const Rep& r : h->d.reps) {
            const DevParams& P = r.P;
            const size_t pb = (size_t)P.pbase;
            hipLaunchKernelGGL(k_load_input, dim3(grid_for(P.N)), dim3(kBlock), 0, h->stream, P,
                               (const float2*)x + pb, (const float2*)v + pb, h->Ax + pb, h->Au + pb,
                               h->Aid + pb, h->key + pb, h->rank + pb, h->count, h->status);
        }
        LAUNCHCHK(h);
        int rc = bin_from_counts(h, h->count, true, nullptr, nullptr, F ? h->Aid : nullptr, h->Aid, h->posid);
        if (rc) return rc;
        if (F) {
            for (const Rep& r : h->d.reps) {
                const size_t pb = (size_t)r.P.pbase;
                hipLaunchKernelGGL(k_gather_state, dim3(grid_for(r.P.N)), dim3(kBlock), 0, h->stream,
                                   r.P.N, (const int*)h->src + pb, (const float2*)h->Ax,
                                   (const float2*)h->Au, (const int*)h->Aid, (const float2*)F + pb,
                                   h->Sx + pb, h->Sv + pb, h->Sid + pb, h->SF + pb, h->status);
            }
            LAUNCHCHK(h);
        } else {
            PairArgs a = {};
            a.cs = h->cs;
            a.src = h->src;
            a.xin = h->Ax;
            a.uin = h->Au;
            a.idin = h->Aid;
            a.xout = h->Sx;
            a.uout = h->Sv;
            a.idout = h->Sid;
            a.Fout = h->SF;
            a.status = h->status;
            a.step = (uint32_t)((uint64_t)step & 0xffffffffu);
            rc = launch_pair(h, MODE_FORCES, a, false);
            if (rc) return rc;
        }
        h->step = step;
        h->have_state = true;
        return DPD_OK;
    } catch (...) {
        return fail(h, DPD_EINVAL, "internal error");
    }
}

int dpd_step(dpd_handle* h, int32_t n_steps, int32_t reduce_every, double* pk_out) {
    if (!h) return fail(nullptr, DPD_EINVAL, "handle is NULL");
    if (!h->have_state) return fail(h, DPD_ESTATE, "dpd_step before dpd_set_state");
    if (n_steps < 0) return fail(h, DPD_EINVAL, "n_steps < 0");
    if (reduce_every < 0) return fail(h, DPD_EINVAL, "reduce_every < 0");
    if (n_steps == 0) return DPD_OK;
    try {
        double* pk = reduce_every > 0 ? pk_out : nullptr;
        int rc;
        if (!h->prepared) {
            // first half kick + drift from the stored state
            rc = kick_drift(h);
            if (rc) return rc;
        }
        int64_t done = 0, rec = 0;
        const int K = h->graph_chunk;
        const bool graphs = K > 0 && !h->d.skin && !h->profiling &&
                            (pk == nullptr || reduce_every % K == 0);
        if (graphs && n_steps > K && h->prep_x != h->Ax && pk == nullptr) {
            // a captured chunk starts from the A buffers
            rc = run_steps(h, 1, 0, nullptr, 0, &rec);
            if (rc) return rc;
            done = 1;
        }
        if (graphs && h->prep_x == h->Ax && n_steps - done >= K) {
            const int64_t chunks = (n_steps - done) / K;
            hipLaunchKernelGGL(k_fill_i32, dim3(1), dim3(64), 0, h->stream, (int*)h->stepb,
                               (int)(uint32_t)((uint64_t)h->step & 0xffffffffu), 1LL);
            LAUNCHCHK(h);
            for (int64_t c = 0; c < chunks; ++c) {
                const bool red = pk && ((done + K) % reduce_every == 0);
                hipGraphExec_t exec = nullptr;
                for (const Graph& g : h->graphs)
                    if (g.K == K && g.reduce_last == red) exec = g.exec;
                if (!exec) {
                    rc = capture_chunk(h, K, red, &exec);
                    if (rc) return rc;
                    h->graphs.push_back(Graph{K, red, exec});
                }
                HIPCHK(h, hipGraphLaunch(exec, h->stream));
                h->step += K;
                done += K;
                if (red) {
                    rc = launch_reduce(h, pk + 3 * (size_t)h->R * (size_t)rec);
                    if (rc) return rc;
                    ++rec;
                }
            }
            // every chunk leaves the next step prepared in A
            h->prep_x = h->Ax;
            h->prep_u = h->Au;
            h->prep_id = h->Aid;
        }
        if (done < n_steps) {
            rc = run_steps(h, n_steps - done, reduce_every, pk, done, &rec);
            if (rc) return rc;
        }
        return DPD_OK;
    } catch (...) {
        return fail(h, DPD_EINVAL, "internal error");
    }
}

int dpd_forces(dpd_handle* h, float* F_out) {
    if (!h) return fail(nullptr, DPD_EINVAL, "handle is NULL");
    if (!h->have_state) return fail(h, DPD_ESTATE, "dpd_forces before dpd_set_state");
    if (!F_out) return fail(h, DPD_EINVAL, "F_out is NULL");
    try {
        int rc0 = unprepare(h);
        if (rc0) return rc0;
        for (const Rep& r : h->d.reps) {
            const size_t pb = (size_t)r.P.pbase;
            hipLaunchKernelGGL(k_key_rank, dim3(grid_for(r.P.N)), dim3(kBlock), 0, h->stream, r.P,
                               (const float2*)h->Sx + pb, h->key + pb, h->rank + pb, h->count);
        }
        LAUNCHCHK(h);
        int rc = bin_from_counts(h, h->count, true, nullptr, nullptr, nullptr, h->Sid, h->posid);
        if (rc) return rc;
        PairArgs a = {};
        a.cs = h->cs;
        a.src = h->src;
        a.xin = h->Sx;
        a.uin = h->Sv;
        a.idin = h->Sid;
        a.xout = h->Bx;
        a.uout = h->Bu;
        a.idout = h->Bid;
        a.Fout = h->Fs;
        a.status = h->status;
        a.step = (uint32_t)((uint64_t)h->step & 0xffffffffu);
        rc = launch_pair(h, MODE_FORCES, a, false);
        if (rc) return rc;
        for (const Rep& r : h->d.reps) {
            const size_t pb = (size_t)r.P.pbase;
            hipLaunchKernelGGL(k_unpermute, dim3(grid_for(r.P.N)), dim3(kBlock), 0, h->stream, r.P.N,
                               (const int*)h->Bid + pb, (const float2*)h->Fs + pb,
                               (float2*)F_out + pb);
        }
        LAUNCHCHK(h);
        return read_status(h);
    } catch (...) {
        return fail(h, DPD_EINVAL, "internal error");
    }
}

int dpd_get_state(dpd_handle* h, float* x, float* v, float* F, int64_t* step) {
    if (!h) return fail(nullptr, DPD_EINVAL, "handle is NULL");
    if (!h->have_state) return fail(h, DPD_ESTATE, "dpd_get_state before dpd_set_state");
    const float2* srcs[3] = {h->Sx, h->Sv, h->SF};
    float* dsts[3] = {x, v, F};
    for (int k = 0; k < 3; ++k) {
        if (!dsts[k]) continue;
        for (const Rep& r : h->d.reps) {
            const size_t pb = (size_t)r.P.pbase;
            hipLaunchKernelGGL(k_unpermute, dim3(grid_for(r.P.N)), dim3(kBlock), 0, h->stream, r.P.N,
                               (const int*)h->Sid + pb, srcs[k] + pb, (float2*)dsts[k] + pb);
        }
        LAUNCHCHK(h);
    }
    if (step) *step = h->step;
    return read_status(h);
}

int dpd_get_cells(dpd_handle* h, int32_t* cell_start_out, int32_t* ids_out) {
    if (!h) return fail(nullptr, DPD_EINVAL, "handle is NULL");
    if (!h->have_state) return fail(h, DPD_ESTATE, "dpd_get_cells before dpd_set_state");
    if (cell_start_out)
        HIPCHK(h, hipMemcpyAsync(cell_start_out, h->cs, ((size_t)h->d.cells + 1) * 4,
                                 hipMemcpyDeviceToDevice, h->stream));
    if (ids_out)
        HIPCHK(h, hipMemcpyAsync(ids_out, h->Sid, (size_t)h->d.N * 4, hipMemcpyDeviceToDevice,
                                 h->stream));
    return read_status(h);
}

// dpd_bin_velocity with window width eps[r] for replica r (host array).
int bin_velocity_impl(dpd_handle* h, int32_t M, const double* eps_rep, int32_t mode, float* u_out,
                      int32_t* n_out) {
    if (!h) return fail(nullptr, DPD_EINVAL, "handle is NULL");
    if (!h->have_state) return fail(h, DPD_ESTATE, "dpd_bin_velocity before dpd_set_state");
    if (M < 1 || M > h->d.bin_M_max) return fail(h, DPD_EINVAL, fmt("M = %d outside [1, %d]", M, h->d.bin_M_max));
    if (mode != 0 && mode != 1) return fail(h, DPD_EINVAL, "mode must be 0 or 1");
    if (!u_out || !n_out) return fail(h, DPD_EINVAL, "u_out and n_out must not be NULL");
    if (!eps_rep) return fail(h, DPD_EINVAL, "eps must not be NULL");
    for (int ri = 0; ri < h->R; ++ri)
        if (!std::isfinite(eps_rep[ri])) return fail(h, DPD_EINVAL, "eps must be finite");
    try {
        bool all_rows = true;
        for (int ri = 0; ri < h->R; ++ri) all_rows &= mode == 0 && eps_rep[ri] <= 0.0 && M <= 2048;
        if (!all_rows) {
            // id-order copies of x and v go to the scratch buffers (which may hold
            // the prepared next step)
            int rc0 = unprepare(h);
            if (rc0) return rc0;
        }
        const long long nbin = (long long)M * M;
        for (int ri = 0; ri < h->R; ++ri) {
            const Rep& rp = h->d.reps[ri];
            const DevParams& P = rp.P;
            const size_t pb = (size_t)P.pbase;
            const double eps = eps_rep[ri];
            const bool rows = mode == 0 && eps <= 0.0 && M <= 2048;
            float2* u = (float2*)u_out + (size_t)ri * nbin;
            int* n = (int*)n_out + (size_t)ri * nbin;
            // 64-bit fixed point: |v| <= 2^16 and <= 2^ceil(log2 n) contributors per bin
            const long long n_src = mode == 0 ? P.N : P.N / 2;
            int lg = 0;
            while ((1LL << lg) < n_src + 1) ++lg;
            const int S = std::min(32, 46 - lg);
            const double qscale = std::ldexp(1.0, S);
            if (rows) {
                // plain bins of particle velocities: one block per grid row, read
                // straight from the canonical state
                BinRowArgs r;
                r.Q = std::max(1, std::min(8, M / 32));
                r.x = h->Sx;
                r.v = h->Sv;
                r.cs = h->cs + P.cbase;
                r.u = u;
                r.n = n;
                r.status = h->status;
                r.M = M;
                r.nc = P.nc;
                r.L = rp.p.L;
                r.inv_dx = (double)M / rp.p.L;
                r.qscale = qscale;
                r.vmax = 65536.0;
                const size_t lds = (size_t)((M + r.Q - 1) / r.Q) * 24;
                hipLaunchKernelGGL(k_bin_rows, dim3(r.Q, M), dim3(kBinRowBlock), lds, h->stream, r);
                LAUNCHCHK(h);
                continue;
            }
            hipLaunchKernelGGL(k_unpermute, dim3(grid_for(P.N)), dim3(kBlock), 0, h->stream, P.N,
                               (const int*)h->Sid + pb, (const float2*)h->Sx + pb, h->Bx + pb);
            hipLaunchKernelGGL(k_unpermute, dim3(grid_for(P.N)), dim3(kBlock), 0, h->stream, P.N,
                               (const int*)h->Sid + pb, (const float2*)h->Sv + pb, h->Bu + pb);
            hipLaunchKernelGGL(k_fill_i32, dim3(grid_for(nbin * 6)), dim3(kBlock), 0, h->stream,
                               (int*)h->binacc, 0, nbin * 6);
            LAUNCHCHK(h);
            BinArgs b;
            b.x = h->Bx + pb;
            b.v = h->Bu + pb;
            b.acc = h->binacc;
            b.status = h->status;
            b.n_src = n_src;
            b.mode = mode;
            b.M = M;
            b.L = rp.p.L;
            b.inv_dx = (double)M / rp.p.L;
            b.dx = rp.p.L / (double)M;
            b.eps = eps;
            b.qscale = qscale;
            b.vmax = 65536.0;
            hipLaunchKernelGGL(k_bin_accum, dim3(grid_for(b.n_src)), dim3(kBlock), 0, h->stream, b);
            hipLaunchKernelGGL(k_bin_finalize, dim3(grid_for(nbin)), dim3(kBlock), 0, h->stream,
                               (int)nbin, (const long long*)h->binacc, b.qscale, u, n);
            LAUNCHCHK(h);
        }
        return DPD_OK;
    } catch (...) {
        return fail(h, DPD_EINVAL, "internal error");
    }
}

int dpd_bin_velocity(dpd_handle* h, int32_t M, double eps, int32_t mode, float* u_out,
                     int32_t* n_out) {
    if (!h) return fail(nullptr, DPD_EINVAL, "handle is NULL");
    try {
        std::vector<double> e(h->R, eps);
        return bin_velocity_impl(h, M, e.data(), mode, u_out, n_out);
    } catch (...) {
        return fail(h, DPD_EINVAL, "internal error");
    }
}

int dpd_bin_velocity_reps(dpd_handle* h, int32_t M, const double* eps, int32_t mode, float* u_out,
                          int32_t* n_out) {
    return bin_velocity_impl(h, M, eps, mode, u_out, n_out);
}

int dpd_agent_vcf(const float* x, const float* v, int64_t n_agents, double L, double dr,
                  int32_t n_bins, double* work, long long* sums, long long* counts, void* stream) {
    try {
        if (!x || !v || !work || !sums || !counts)
            return fail(nullptr, DPD_EINVAL, "x, v, work, sums and counts must not be NULL");
        if (n_agents < 1 || n_agents > (int64_t(1) << 29))
            return fail(nullptr, DPD_EINVAL, fmt("n_agents = %lld outside [1, 2^29]", (long long)n_agents));
        if (!(L > 0.0) || !std::isfinite(L) || !(dr > 0.0) || !std::isfinite(dr))
            return fail(nullptr, DPD_EINVAL, "L and dr must be positive and finite");
        if (n_bins < 1 || n_bins > kVcfMaxBins)
            return fail(nullptr, DPD_EINVAL, fmt("n_bins = %d outside [1, %d]", n_bins, kVcfMaxBins));
        hipStream_t s = (hipStream_t)stream;
        const int n = (int)n_agents;
        unsigned* status = reinterpret_cast<unsigned*>(work + 4 * (size_t)n);
        hipLaunchKernelGGL(k_fill_i32, dim3(grid_for(2LL * n_bins)), dim3(kBlock), 0, s, (int*)sums, 0,
                           2LL * n_bins);
        hipLaunchKernelGGL(k_fill_i32, dim3(grid_for(2LL * n_bins)), dim3(kBlock), 0, s, (int*)counts, 0,
                           2LL * n_bins);
        hipLaunchKernelGGL(k_fill_i32, dim3(1), dim3(kBlock), 0, s, (int*)status, 0, 2LL);
        hipLaunchKernelGGL(k_agent_com, dim3(grid_for(n)), dim3(kBlock), 0, s, n, L, (const float2*)x,
                           (const float2*)v, work);
        const int nt = (n + kVcfTile - 1) / kVcfTile;
        hipLaunchKernelGGL(k_vcf_pairs, dim3(nt, nt), dim3(kVcfTile), 0, s, n, L, dr, (int)n_bins,
                           (const double*)work, sums, counts, status);
        hipError_t err = hipGetLastError();
        if (err != hipSuccess) return fail(nullptr, DPD_EHIP, fmt("kernel launch: %s", hipGetErrorString(err)));
        unsigned st = 0;
        err = hipStreamSynchronize(s);
        if (err == hipSuccess) err = hipMemcpy(&st, status, sizeof st, hipMemcpyDeviceToHost);
        if (err != hipSuccess) return fail(nullptr, DPD_EHIP, fmt("hip: %s", hipGetErrorString(err)));
        if (st & kStatusRange)
            return fail(nullptr, DPD_ERANGE, "an agent velocity product |V_k . V_l| reached 4096");
        return DPD_OK;
    } catch (...) {
        return fail(nullptr, DPD_EINVAL, "internal error");
    }
}

int dpd_sync(dpd_handle* h) {
    if (!h) return fail(nullptr, DPD_EINVAL, "handle is NULL");
    return read_status(h);
}

int dpd_rng_words(const dpd_params* p, const int32_t* i, const int32_t* j, int64_t step,
                  int32_t n, uint32_t* words_out, float* alpha_out, void* stream) {
    DevParams P;
    std::string err;
    int rc = derive_one(p, P, &err);
    if (rc) return fail(nullptr, rc, err);
    if (n < 0 || !i || !j || !words_out) return fail(nullptr, DPD_EINVAL, "bad arguments");
    if (n == 0) return DPD_OK;
    hipStream_t s = (hipStream_t)stream;
    hipLaunchKernelGGL(k_rng_words, dim3(grid_for(n)), dim3(kBlock), 0, s, P, (const int*)i,
                       (const int*)j, (uint32_t)((uint64_t)step & 0xffffffffu), (int)n,
                       (uint4*)words_out, alpha_out);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return fail(nullptr, DPD_EHIP, fmt("kernel launch: %s", hipGetErrorString(e)));
    e = hipStreamSynchronize(s);
    if (e != hipSuccess) return fail(nullptr, DPD_EHIP, fmt("sync: %s", hipGetErrorString(e)));
    return DPD_OK;
}

int dpd_set_profiling(dpd_handle* h, int32_t on) {
    if (!h) return fail(nullptr, DPD_EINVAL, "handle is NULL");
    if (on && !h->profiling) {
        h->prof_ms = 0.0;
        h->prof_n = 0;
        h->ev_used = 0;
        h->prof_seq = 0;
    }
    h->profiling = on != 0;
    return DPD_OK;
}

int dpd_pair_kernel_time(dpd_handle* h, double* ms_total, int64_t* launches) {
    if (!h) return fail(nullptr, DPD_EINVAL, "handle is NULL");
    HIPCHK(h, hipStreamSynchronize(h->stream));
    for (size_t k = 0; k < h->ev_used; ++k) {
        float ms = 0.f;
        HIPCHK(h, hipEventElapsedTime(&ms, h->ev_start[k], h->ev_stop[k]));
        h->prof_ms += ms;
        h->prof_n += 1;
    }
    h->ev_used = 0;
    if (ms_total) *ms_total = h->prof_ms;
    if (launches) *launches = h->prof_n;
    return DPD_OK;
}

int dpd_cell_list_rebuilds(dpd_handle* h, int64_t* rebuilds) {
    if (!h) return fail(nullptr, DPD_EINVAL, "handle is NULL");
    if (!rebuilds) return fail(h, DPD_EINVAL, "rebuilds is NULL");
    int n = 0;
    HIPCHK(h, hipStreamSynchronize(h->stream));
    HIPCHK(h, hipMemcpy(&n, h->flags + 2, sizeof n, hipMemcpyDeviceToHost));
    *rebuilds = n;
    return DPD_OK;
}

int dpd_set_graph_chunk(dpd_handle* h, int32_t steps) {
    if (!h) return fail(nullptr, DPD_EINVAL, "handle is NULL");
    if (steps < 0 || (steps & 1) || steps > 4096)
        return fail(h, DPD_EINVAL, "graph chunk must be 0 or an even number of steps <= 4096");
    if (steps != h->graph_chunk) drop_graphs(h);
    h->graph_chunk = steps;
    return DPD_OK;
}

int dpd_set_schedule(dpd_handle* h, int32_t tile_x, int32_t tile_y, int32_t tile_order) {
    if (!h) return fail(nullptr, DPD_EINVAL, "handle is NULL");
    if (h->d.skin) return fail(h, DPD_EINVAL, "the schedule of a Verlet-skin handle is fixed");
    const bool dflt = tile_x == 0 && tile_y == 0;
    if (!dflt && (tile_x < 1 || tile_x > kTileMax || tile_y < 1 || tile_y > kTileMax))
        return fail(h, DPD_EINVAL, fmt("tile sides must be in [1, %d] (or both 0)", kTileMax));
    if (tile_order != 0 && tile_order != 1) return fail(h, DPD_EINVAL, "tile_order must be 0 or 1");
    try {
        return apply_schedule(h, Sched{tile_x, tile_y, 1.0, tile_order});
    } catch (...) {
        return fail(h, DPD_EINVAL, "internal error");
    }
}

int dpd_get_schedule(dpd_handle* h, int32_t* tile_x, int32_t* tile_y, int32_t* tile_order) {
    if (!h) return fail(nullptr, DPD_EINVAL, "handle is NULL");
    if (tile_x) *tile_x = P0(h).tile_x;
    if (tile_y) *tile_y = P0(h).tile_y;
    if (tile_order) *tile_order = h->tile_order;
    return DPD_OK;
}

int dpd_autotune(dpd_handle* h, int32_t trial_steps, int32_t* tile_x, int32_t* tile_y,
                 int32_t* tile_order, double* best_ms) {
    if (!h) return fail(nullptr, DPD_EINVAL, "handle is NULL");
    if (!h->have_state) return fail(h, DPD_ESTATE, "dpd_autotune before dpd_set_state");
    if (h->d.skin) return fail(h, DPD_EINVAL, "the schedule of a Verlet-skin handle is fixed");
    if (trial_steps < 1 || trial_steps > 100000) return fail(h, DPD_EINVAL, "trial_steps must be in [1, 100000]");
    try {
        const bool prof = h->profiling;
        h->profiling = false;
        const int64_t step0 = h->step;
        int rc = unprepare(h);
        if (!rc) rc = copy_state(h, true);
        hipEvent_t e0 = nullptr, e1 = nullptr;
        if (!rc && hipEventCreate(&e0) != hipSuccess) rc = fail(h, DPD_EHIP, "hipEventCreate failed");
        if (!rc && hipEventCreate(&e1) != hipSuccess) rc = fail(h, DPD_EHIP, "hipEventCreate failed");
        double best = 1e300;
        Derived best_d = h->d;
        int best_order = h->tile_order;
        // one trial: the state as saved, stepped under tiling nd; its time in
        // ms and, if asked, each replica's tiles that overflowed an LDS capacity
        // in the last step
        auto trial = [&](const Derived& nd, int order, float* ms, std::vector<int>* ovf_rep) -> int {
            drop_graphs(h);
            h->d = nd;
            h->tile_order = order;
            int r2 = upload_tables(h);
            if (!r2) r2 = copy_state(h, false);
            if (r2) return r2;
            h->step = step0;
            h->prepared = false;
            r2 = kick_drift(h);
            int64_t rec = 0;
            if (!r2) r2 = run_steps(h, 2, 0, nullptr, 0, &rec);  // untimed
            if (!r2 && hipEventRecord(e0, h->stream) != hipSuccess) r2 = fail(h, DPD_EHIP, "hipEventRecord failed");
            if (!r2) r2 = run_steps(h, trial_steps, 0, nullptr, 0, &rec);
            if (!r2 && hipEventRecord(e1, h->stream) != hipSuccess) r2 = fail(h, DPD_EHIP, "hipEventRecord failed");
            if (!r2 && hipEventSynchronize(e1) != hipSuccess) r2 = fail(h, DPD_EHIP, "hipEventSynchronize failed");
            if (!r2 && hipEventElapsedTime(ms, e0, e1) != hipSuccess) r2 = fail(h, DPD_EHIP, "hipEventElapsedTime failed");
            if (!r2 && ovf_rep) {
                // the last pair launch's list of overflowing tiles (cleared by
                // the next step's scan only)
                int n = 0;
                HIPCHK(h, hipMemcpy(&n, h->ovf, sizeof n, hipMemcpyDeviceToHost));
                n = std::max(0, std::min<int>(n, (int)nd.tiles));
                std::vector<int> list((size_t)n);
                if (n) HIPCHK(h, hipMemcpy(list.data(), h->ovf + 1, (size_t)n * 4, hipMemcpyDeviceToHost));
                ovf_rep->assign(nd.reps.size(), 0);
                for (int t : list)
                    for (size_t r = 0; r < nd.reps.size(); ++r) {
                        const long long t0 = nd.reps[r].P.tbase;
                        if (t >= t0 && t < t0 + (long long)nd.reps[r].P.ntx * nd.reps[r].P.nty) {
                            ++(*ovf_rep)[r];
                            break;
                        }
                    }
            }
            if (!r2) r2 = unprepare(h);
            return r2;
        };
        std::vector<std::vector<int>> seen;
        for (const Sched& c0 : kCandidates) {
            for (int order = 0; order < 2 && !rc; ++order) {
                Sched c = c0;
                c.order = order;
                // skip schedules that give tilings already timed, and those that
                // do not fit the per-tile arrays
                Derived nd = with_schedule(h->d, c);
                if (nd.tiles > h->d.tiles_alloc) continue;
                std::vector<int> sig{order};
                for (const Rep& r : nd.reps) sig.push_back(r.P.tile_x * 16 + r.P.tile_y);
                if (std::find(seen.begin(), seen.end(), sig) != seen.end()) continue;
                seen.push_back(sig);
                float ms = 0.f;
                rc = trial(nd, order, &ms, nullptr);
                if (!rc && ms < best) {
                    best = ms;
                    best_d = nd;
                    best_order = order;
                }
            }
            if (rc) break;
        }
        // A batch's replicas can differ in how their tiles fill (clusters form
        // in some and not in others): starting from the best schedule, every
        // replica with more than 2 % of its tiles overflowing in the last trial
        // step moves to the tiling with the next larger number of tiles among
        // the candidates and the finer ones, as long as the step gets faster
        // (at most eight rounds).  Every replica's tiling is then one of those
        // the per-tile arrays were sized for.
        if (!rc && h->R > 1) {
            const size_t R = best_d.reps.size();
            std::vector<std::vector<Sched>> ladder(R);
            std::vector<size_t> pos(R, 0);
            for (size_t r = 0; r < R; ++r) {
                std::vector<std::pair<long long, Sched>> opts;
                std::vector<Sched> all(std::begin(kCandidates), std::end(kCandidates));
                all.insert(all.end(), std::begin(kRefine), std::end(kRefine));
                for (const Sched& c0 : all) {
                    Rep rep = best_d.reps[r];
                    apply_tiling(rep, c0);
                    const long long nt = (long long)rep.P.ntx * rep.P.nty;
                    bool dup = false;
                    for (auto& o : opts) {
                        Rep q = best_d.reps[r];
                        apply_tiling(q, o.second);
                        dup |= q.P.tile_x == rep.P.tile_x && q.P.tile_y == rep.P.tile_y;
                    }
                    if (!dup) opts.push_back({nt, c0});
                }
                std::stable_sort(opts.begin(), opts.end(),
                                 [](const auto& x, const auto& y) { return x.first < y.first; });
                for (auto& o : opts) ladder[r].push_back(o.second);
                for (size_t k = 0; k < ladder[r].size(); ++k) {
                    Rep q = best_d.reps[r];
                    apply_tiling(q, ladder[r][k]);
                    if (q.P.tile_x == best_d.reps[r].P.tile_x && q.P.tile_y == best_d.reps[r].P.tile_y) pos[r] = k;
                }
            }
            float ms = 0.f;
            std::vector<int> ovf;
            rc = trial(best_d, best_order, &ms, &ovf);
            for (int round = 0; round < 8 && !rc; ++round) {
                Derived nd = best_d;
                bool changed = false;
                for (size_t r = 0; r < R; ++r) {
                    const long long nt = (long long)best_d.reps[r].P.ntx * best_d.reps[r].P.nty;
                    if ((long long)ovf[r] * 50 > nt && pos[r] + 1 < ladder[r].size()) {
                        apply_tiling(nd.reps[r], ladder[r][pos[r] + 1]);
                        changed = true;
                    }
                }
                if (!changed) break;
                assign_offsets(&nd);
                if (nd.tiles > h->d.tiles_alloc) break;
                std::vector<int> ovf2;
                rc = trial(nd, best_order, &ms, &ovf2);
                if (rc || !(ms < best)) break;
                best = ms;
                for (size_t r = 0; r < R; ++r)
                    if (nd.reps[r].P.tile_x != best_d.reps[r].P.tile_x ||
                        nd.reps[r].P.tile_y != best_d.reps[r].P.tile_y)
                        ++pos[r];
                best_d = nd;
                ovf = ovf2;
            }
        }
        if (e0) (void)hipEventDestroy(e0);
        if (e1) (void)hipEventDestroy(e1);
        h->profiling = prof;
        if (rc) return rc;
        // the chosen schedule, and the state as it was
        drop_graphs(h);
        h->d = best_d;
        h->tile_order = best_order;
        rc = upload_tables(h);
        if (!rc) rc = copy_state(h, false);
        if (!rc) rc = rebin_stored(h);
        if (rc) return rc;
        h->step = step0;
        h->prepared = false;
        if (tile_x) *tile_x = P0(h).tile_x;
        if (tile_y) *tile_y = P0(h).tile_y;
        if (tile_order) *tile_order = best_order;
        if (best_ms) *best_ms = best / trial_steps;
        return read_status(h);
    } catch (...) {
        return fail(h, DPD_EINVAL, "internal error");
    }
}

int dpd_copy_kernel(const void* src, void* dst, size_t bytes, void* stream) {
    if (!src || !dst || (bytes & 15)) return fail(nullptr, DPD_EINVAL, "bad copy arguments");
    const long long n = (long long)(bytes / 16);
    if (n == 0) return DPD_OK;
    int G = grid_for(n);
    if (G > 256 * 64) G = 256 * 64;
    hipLaunchKernelGGL(k_copy16, dim3(G), dim3(kBlock), 0, (hipStream_t)stream, (const uint4*)src,
                       (uint4*)dst, n);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return fail(nullptr, DPD_EHIP, fmt("kernel launch: %s", hipGetErrorString(e)));
    return DPD_OK;
}

int dpd_forces_noalloc(const dpd_params* p, const float* x, const float* v, int64_t step,
                       float* F_out, void* stream) {
    try {
        if (!p) return fail(nullptr, DPD_EINVAL, "params is NULL");
        if (!x || !v || !F_out) return fail(nullptr, DPD_EINVAL, "x, v and F_out must not be NULL");
        // forces do not depend on the skin (bitwise) and bin nothing: the
        // smallest layout for these parameters
        dpd_params q = *p;
        q.skin = 0.0f;
        q.bin_M_max = 1;
        Derived d;
        std::string err;
        int rc = derive(&q, 1, &d, &err);
        if (rc) return fail(nullptr, rc, err);
        if (d.lay.total > kNoAllocScratchBytes)
            return fail(nullptr, DPD_EWORKSPACE,
                        fmt("%lld particles need %zu bytes of scratch; the static scratch of "
                            "dpd_forces_noalloc holds %zu (about %lld particles at this density)",
                            (long long)d.N, d.lay.total, kNoAllocScratchBytes,
                            (long long)((double)kNoAllocScratchBytes * (double)d.N / (double)d.lay.total)));
        void* ws = nullptr;
        rc = noalloc_scratch(&ws);
        if (rc) return rc;
        dpd_handle* h = nullptr;
        rc = dpd_create(&q, ws, kNoAllocScratchBytes, stream, &h);
        if (rc) return rc;
        rc = dpd_set_state(h, x, v, step, nullptr);
        if (!rc) rc = dpd_get_state(h, nullptr, nullptr, F_out, nullptr);
        if (rc) g_last_error = h->err;
        dpd_destroy(h);
        return rc;
    } catch (...) {
        return fail(nullptr, DPD_EINVAL, "internal error");
    }
}

}  // extern "C"
