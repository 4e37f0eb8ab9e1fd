// engine.hip -- host side of the DPD engine: parameter checks, workspace
// layout, launch sequences and the C ABI declared in include/dpd.h.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <algorithm>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "../../include/dpd.h"
#include "kernels.h"

using namespace dpd;

namespace {

thread_local std::string g_last_error = "no error";

struct Layout {
    size_t off_Sx, off_Sv, off_SF, off_Sid;
    size_t off_Ax, off_Au, off_Aid, off_Bx, off_Bu, off_Bid;
    size_t off_key, off_rank, off_src, off_count, off_cs;
    size_t off_scan_part, off_red, off_Fs, off_binacc, off_status, off_ovf;
    size_t off_count2, off_xref, off_rec, off_flags;  // Verlet skin
    size_t total;
};

struct Derived {
    DevParams P;
    int n_tiles;
    int n_scan_blocks;  // chunks of the cell-count scan
    int bin_M_max;
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

// Validate parameters and derive the launch constants and workspace layout.
int derive(const dpd_params* p, Derived* d, std::string* err) {
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
    const double width = p->r_c + (double)p->skin;  // smallest cell width
    const double ncd = std::floor(p->L / width);
    if (!(ncd >= 3.0)) { *err = "L must be at least 3 (r_c + skin) (n_c >= 3)"; return DPD_EINVAL; }
    if (ncd > 46340.0) { *err = "too many cells (n_c^2 must fit in int32)"; return DPD_EINVAL; }
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

    DevParams& P = d->P;
    P.N = (int)(2 * p->n_agents);
    P.nc = (int)ncd;
    P.n_cells = P.nc * P.nc;
    // tile + halo must not wrap onto itself: tile side <= n_c - 2.  With a skin
    // the cells are wider; the default tile keeps about 56 particles.
    int tx = kTileX, ty = kTileY;
    if (p->skin > 0.0f) {
        const double cell_n = (2.0 * (double)p->n_agents) / ((double)ncd * ncd);  // particles per cell
        const double sc = std::sqrt(std::max(cell_n, 1e-9));
        tx = std::max(1, std::min(kTileMax, (int)std::lround(kTileX / sc)));
        ty = std::max(1, std::min(kTileMax, (int)std::lround(kTileY / sc)));
    }
    P.tile_x = std::min(p->tile ? p->tile : tx, P.nc - 2);
    P.tile_y = std::min(p->tile ? p->tile : ty, P.nc - 2);
    P.ntx = (P.nc + P.tile_x - 1) / P.tile_x;
    P.nty = (P.nc + P.tile_y - 1) / P.tile_y;
    {
        const int w_full = P.tile_x + 2, w_last = (P.nc - (P.ntx - 1) * P.tile_x) + 2;
        P.wmul_full = (65536 + w_full - 1) / w_full;
        P.wmul_last = (65536 + w_last - 1) / w_last;
        // (tile + 1/2) / ntx lies at least 1/(2 ntx) >= 2^-17 from an integer, far
        // beyond the 2^-21 error of the product for tile < 2^31
        P.inv_ntx = 1.0 / (double)P.ntx;
    }
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

    d->n_tiles = P.ntx * P.nty;
    d->n_scan_blocks = (P.n_cells + kScanTile - 1) / kScanTile;
    d->bin_M_max = p->bin_M_max ? p->bin_M_max : 256;

    const size_t N = (size_t)P.N;
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
    L.off_count = take((size_t)P.n_cells * 4);
    L.off_cs = take(((size_t)P.n_cells + 1) * 4);
    L.off_red = take(((size_t)d->n_tiles + kRedParts) * 3 * 8);  // per tile, then per part
    L.off_Fs = take(N * 8);
    L.off_binacc = take((size_t)d->bin_M_max * d->bin_M_max * 3 * 8);
    L.off_status = take(16);
    L.off_ovf = take(((size_t)d->n_tiles + 1) * 4);
    L.off_scan_part = take((size_t)d->n_scan_blocks * 4);
    L.off_flags = take(64);  // two displacement flags (by step parity)
    if (P.skin_on) {
        L.off_count2 = take((size_t)P.n_cells * 4);
        L.off_xref = take(N * 8);
        L.off_rec = take((size_t)d->n_tiles * kRecStride);
    } else {
        L.off_count2 = L.off_xref = L.off_rec = 0;
    }
    L.total = o;
    return DPD_OK;
}

inline int grid_for(long long n, int block = kBlock) { return (int)((n + block - 1) / block); }

}  // namespace

struct dpd_handle {
    dpd_params p;
    Derived d;
    hipStream_t stream;
    char* ws;
    float2 *Sx, *Sv, *SF, *Ax, *Au, *Bx, *Bu, *Fs;
    int *Sid, *Aid, *Bid, *key, *rank, *src, *count, *cs;
    unsigned* status;
    int* ovf;  // [0]: count of tiles left to the overflow kernel, then their indices
    int* scan_part;
    // Verlet skin: second counter array, rebuild positions, tile records, flags
    int* count2;
    float2* xref;
    unsigned char* rec;
    int* flags;
    double* red;
    long long* binacc;
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

// cell_start from count (count cleared) and the slot -> input map.  Within a
// cell the slots are in arrival order; the pair kernel places each cell's
// members by id itself.  With id_of_input != NULL every cell is also ordered by
// id here (only for the state loaded with a given force, which no pair kernel
// passes through before it is stored).
int bin_from_counts(dpd_handle* h, int* count, const int* rebuild, int* moved_clear,
                    const int* id_of_input) {
    const DevParams& P = h->d.P;
    const int G = h->d.n_scan_blocks;
    hipLaunchKernelGGL(k_scan_reduce, dim3(G), dim3(kBlock), 0, h->stream, (const int*)count,
                       P.n_cells, h->scan_part, rebuild, moved_clear, h->flags + 2);
    hipLaunchKernelGGL(k_scan_final, dim3(G), dim3(kBlock), 0, h->stream, count, P.n_cells,
                       (const int*)h->scan_part, h->cs, h->ovf, rebuild);
    hipLaunchKernelGGL(k_scatter, dim3(std::min(grid_for(P.N), 4096)), dim3(kBlock), 0, h->stream,
                       P.N, (const int*)h->key, (const int*)h->rank, (const int*)h->cs, h->src,
                       rebuild);
    if (id_of_input)
        hipLaunchKernelGGL(k_cell_sort, dim3(grid_for(P.n_cells)), dim3(kBlock), 0, h->stream,
                           P.n_cells, (const int*)h->cs, h->src, id_of_input);
    LAUNCHCHK(h);
    return DPD_OK;
}

// Per-cell counter array of step s (with a Verlet skin the two arrays alternate
// by step parity: step s fills the one for the keys of x_{s+1} while the other,
// consumed by the binning of step s, is cleared tile by tile).
int* counter_of(dpd_handle* h, int64_t s) {
    return (h->count2 && (s & 1)) ? h->count2 : h->count;
}

int launch_pair(dpd_handle* h, int mode, const PairArgs& a, bool reduce) {
    const DevParams& P = h->d.P;
    const int G = h->d.n_tiles;
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
    // the Verlet-skin variant of the kernel only where a skin is set (a force
    // evaluation alone keeps no record)
    const bool skin = P.skin_on && mode != MODE_FORCES;
    if (mode == MODE_STEP && skin)
        hipLaunchKernelGGL((k_pair<MODE_STEP, true>), dim3(G), dim3(kWave), 0, h->stream, P, b, (int)reduce);
    else if (mode == MODE_STEP)
        hipLaunchKernelGGL((k_pair<MODE_STEP, false>), dim3(G), dim3(kWave), 0, h->stream, P, b, (int)reduce);
    else if (mode == MODE_FINAL && skin)
        hipLaunchKernelGGL((k_pair<MODE_FINAL, true>), dim3(G), dim3(kWave), 0, h->stream, P, b, (int)reduce);
    else if (mode == MODE_FINAL)
        hipLaunchKernelGGL((k_pair<MODE_FINAL, false>), dim3(G), dim3(kWave), 0, h->stream, P, b, (int)reduce);
    else
        hipLaunchKernelGGL((k_pair<MODE_FORCES, false>), dim3(G), dim3(kWave), 0, h->stream, P, b, 0);
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
    // tiles over an LDS capacity (dense clusters), if any
    const int Go = std::min(G, 64);
    if (mode == MODE_STEP)
        hipLaunchKernelGGL(k_pair_overflow<MODE_STEP>, dim3(Go), dim3(kWave), 0, h->stream, P, b, (int)reduce);
    else if (mode == MODE_FINAL)
        hipLaunchKernelGGL(k_pair_overflow<MODE_FINAL>, dim3(Go), dim3(kWave), 0, h->stream, P, b, (int)reduce);
    else
        hipLaunchKernelGGL(k_pair_overflow<MODE_FORCES>, dim3(Go), dim3(kWave), 0, h->stream, P, b, 0);
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
    return DPD_OK;
}

// Drop the prepared next step (its cell counts are cleared so that the next
// binning starts from zero).
int unprepare(dpd_handle* h) {
    if (!h->prepared) return DPD_OK;
    hipLaunchKernelGGL(k_fill_i32, dim3(grid_for(h->d.P.n_cells)), dim3(kBlock), 0, h->stream,
                       h->count, 0, (long long)h->d.P.n_cells);
    if (h->count2)
        hipLaunchKernelGGL(k_fill_i32, dim3(grid_for(h->d.P.n_cells)), dim3(kBlock), 0, h->stream,
                           h->count2, 0, (long long)h->d.P.n_cells);
    LAUNCHCHK(h);
    h->prepared = false;
    return DPD_OK;
}

}  // namespace

extern "C" {

int dpd_workspace_bytes(const dpd_params* p, size_t* bytes) {
    try {
        Derived d;
        std::string err;
        int rc = derive(p, &d, &err);
        if (rc) return fail(nullptr, rc, err);
        if (!bytes) return fail(nullptr, DPD_EINVAL, "bytes is NULL");
        *bytes = d.lay.total;
        return DPD_OK;
    } catch (...) {
        return fail(nullptr, DPD_EINVAL, "internal error");
    }
}

int64_t dpd_cells_per_side(const dpd_params* p) {
    Derived d;
    std::string err;
    int rc = derive(p, &d, &err);
    if (rc) return fail(nullptr, rc, err);
    return d.P.nc;
}

int dpd_create(const dpd_params* p, void* workspace, size_t bytes, void* stream,
               dpd_handle** out) {
    try {
        if (!out) return fail(nullptr, DPD_EINVAL, "out is NULL");
        *out = nullptr;
        Derived d;
        std::string err;
        int rc = derive(p, &d, &err);
        if (rc) return fail(nullptr, rc, err);
        if (!workspace || ((uintptr_t)workspace & 255u))
            return fail(nullptr, DPD_EWORKSPACE, "workspace is NULL or not 256-byte aligned");
        if (bytes < d.lay.total)
            return fail(nullptr, DPD_EWORKSPACE,
                        fmt("workspace has %zu bytes, needs %zu", bytes, d.lay.total));
        dpd_handle* h = new (std::nothrow) dpd_handle();
        if (!h) return fail(nullptr, DPD_EINVAL, "out of host memory");
        h->p = *p;
        h->d = d;
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
        h->scan_part = (int*)(w + L.off_scan_part);
        h->flags = (int*)(w + L.off_flags);
        h->count2 = d.P.skin_on ? (int*)(w + L.off_count2) : nullptr;
        h->xref = d.P.skin_on ? (float2*)(w + L.off_xref) : nullptr;
        h->rec = d.P.skin_on ? (unsigned char*)(w + L.off_rec) : nullptr;
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
        // clear the counters the kernels rely on
        hipLaunchKernelGGL(k_fill_i32, dim3(grid_for(d.P.n_cells)), dim3(kBlock), 0, h->stream,
                           h->count, 0, (long long)d.P.n_cells);
        hipLaunchKernelGGL(k_fill_i32, dim3(1), dim3(kBlock), 0, h->stream, (int*)h->status, 0, 4LL);
        hipLaunchKernelGGL(k_fill_i32, dim3(1), dim3(kBlock), 0, h->stream, h->ovf, 0, 1LL);
        hipLaunchKernelGGL(k_fill_i32, dim3(1), dim3(kBlock), 0, h->stream, h->flags, 0, 16LL);
        if (d.P.skin_on) {
            hipLaunchKernelGGL(k_fill_i32, dim3(grid_for(d.P.n_cells)), dim3(kBlock), 0, h->stream,
                               h->count2, 0, (long long)d.P.n_cells);
            // no tile record is valid before the first rebuild
            const long long words = (long long)d.n_tiles * (long long)(kRecStride / 4);
            hipLaunchKernelGGL(k_fill_i32, dim3(grid_for(words)), dim3(kBlock), 0, h->stream,
                               (int*)h->rec, 0, words);
        }
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) {
            std::string m = fmt("kernel launch: %s", hipGetErrorString(e));
            delete h;
            return fail(nullptr, DPD_EHIP, m);
        }
        *out = h;
        return DPD_OK;
    } catch (...) {
        return fail(nullptr, DPD_EINVAL, "internal error");
    }
}

void dpd_destroy(dpd_handle* h) {
    if (!h) return;
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
        const DevParams& P = h->d.P;
        int rc0 = unprepare(h);
        if (rc0) return rc0;
        hipLaunchKernelGGL(k_load_input, dim3(grid_for(P.N)), dim3(kBlock), 0, h->stream, P,
                           (const float2*)x, (const float2*)v, h->Ax, h->Au, h->Aid, h->key,
                           h->rank, h->count, h->status);
        LAUNCHCHK(h);
        int rc = bin_from_counts(h, h->count, nullptr, nullptr, F ? h->Aid : nullptr);
        if (rc) return rc;
        if (F) {
            hipLaunchKernelGGL(k_gather_state, dim3(grid_for(P.N)), dim3(kBlock), 0, h->stream, P.N,
                               (const int*)h->src, (const float2*)h->Ax, (const float2*)h->Au,
                               (const int*)h->Aid, (const float2*)F, h->Sx, h->Sv, h->Sid, h->SF,
                               h->status);
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
        const DevParams& P = h->d.P;
        const bool want_pk = reduce_every > 0 && pk_out != nullptr;
        float2 *inx, *inu, *outx, *outu;
        int *inid, *outid;
        if (h->prepared) {
            // the previous call already made this step's half kick, drift and keys
            inx = h->prep_x;
            inu = h->prep_u;
            inid = h->prep_id;
        } else {
            // first half kick + drift from the stored state; with a skin the first
            // step rebuilds
            hipLaunchKernelGGL(k_kick_drift, dim3(grid_for(P.N)), dim3(kBlock), 0, h->stream, P,
                               (const float2*)h->Sx, (const float2*)h->Sv, (const float2*)h->SF,
                               (const int*)h->Sid, h->Ax, h->Au, h->Aid, h->key, h->rank,
                               counter_of(h, h->step), h->status);
            if (P.skin_on)
                hipLaunchKernelGGL(k_fill_i32, dim3(1), dim3(kBlock), 0, h->stream,
                                   h->flags + (h->step & 1), 1, 1LL);
            LAUNCHCHK(h);
            inx = h->Ax;
            inu = h->Au;
            inid = h->Aid;
        }
        h->prepared = false;
        const bool in_a = (inx == h->Ax);
        outx = in_a ? h->Bx : h->Ax;
        outu = in_a ? h->Bu : h->Au;
        outid = in_a ? h->Bid : h->Aid;
        int rec = 0;
        for (int k = 1; k <= n_steps; ++k) {
            // forces of step s = step + k: the binning consumes the keys of x_s
            // (counters of step s - 1) if this step rebuilds
            const int64_t s = h->step + k;
            int* consumed = counter_of(h, s - 1);
            const int* rebuild = P.skin_on ? h->flags + ((s - 1) & 1) : nullptr;
            int* moved = P.skin_on ? h->flags + (s & 1) : nullptr;
            int rc = bin_from_counts(h, consumed, rebuild, moved, nullptr);
            if (rc) return rc;
            const bool last = (k == n_steps);
            const bool red = want_pk && (k % reduce_every == 0);
            PairArgs a = {};
            a.cs = h->cs;
            a.src = h->src;
            a.xin = inx;
            a.uin = inu;
            a.idin = inid;
            a.status = h->status;
            a.red = h->red;
            a.step = (uint32_t)((uint64_t)(h->step + k) & 0xffffffffu);
            a.keyout = h->key;
            a.rankout = h->rank;
            a.count = counter_of(h, s);
            if (P.skin_on) {
                a.rebuild = rebuild;
                a.rec = h->rec;
                a.xref = h->xref;
                a.moved = moved;
                a.count_clear = consumed;
            }
            if (last) {
                a.xout = h->Sx;
                a.uout = h->Sv;
                a.idout = h->Sid;
                a.Fout = h->SF;
                a.pxout = outx;
                a.puout = outu;
                a.pidout = outid;
                rc = launch_pair(h, MODE_FINAL, a, red);
            } else {
                a.xout = outx;
                a.uout = outu;
                a.idout = outid;
                rc = launch_pair(h, MODE_STEP, a, red);
            }
            if (rc) return rc;
            if (red) {
                const int parts = std::min(kRedParts, h->d.n_tiles);
                double* part = h->red + 3 * (size_t)h->d.n_tiles;
                hipLaunchKernelGGL(k_reduce_part, dim3(parts), dim3(kBlock), 0, h->stream,
                                   (const double*)h->red, h->d.n_tiles, part);
                hipLaunchKernelGGL(k_reduce_final, dim3(1), dim3(kBlock), 0, h->stream,
                                   (const double*)part, parts, h->p.mass, pk_out + 3 * rec);
                LAUNCHCHK(h);
                ++rec;
            }
            std::swap(inx, outx);
            std::swap(inu, outu);
            std::swap(inid, outid);
        }
        // the last launch left the next step's start in what is now `in`
        h->prepared = true;
        h->prep_x = inx;
        h->prep_u = inu;
        h->prep_id = inid;
        h->step += n_steps;
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
        const DevParams& P = h->d.P;
        int rc0 = unprepare(h);
        if (rc0) return rc0;
        hipLaunchKernelGGL(k_key_rank, dim3(grid_for(P.N)), dim3(kBlock), 0, h->stream, P,
                           (const float2*)h->Sx, h->key, h->rank, h->count);
        LAUNCHCHK(h);
        int rc = bin_from_counts(h, h->count, nullptr, nullptr, nullptr);
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
        hipLaunchKernelGGL(k_unpermute, dim3(grid_for(P.N)), dim3(kBlock), 0, h->stream, P.N,
                           (const int*)h->Bid, (const float2*)h->Fs, (float2*)F_out);
        LAUNCHCHK(h);
        return read_status(h);
    } catch (...) {
        return fail(h, DPD_EINVAL, "internal error");
    }
}

int dpd_get_state(dpd_handle* h, float* x, float* v, float* F, int64_t* step) {
    if (!h) return fail(nullptr, DPD_EINVAL, "handle is NULL");
    if (!h->have_state) return fail(h, DPD_ESTATE, "dpd_get_state before dpd_set_state");
    const DevParams& P = h->d.P;
    const float2* srcs[3] = {h->Sx, h->Sv, h->SF};
    float* dsts[3] = {x, v, F};
    for (int k = 0; k < 3; ++k) {
        if (!dsts[k]) continue;
        hipLaunchKernelGGL(k_unpermute, dim3(grid_for(P.N)), dim3(kBlock), 0, h->stream, P.N,
                           (const int*)h->Sid, srcs[k], (float2*)dsts[k]);
        LAUNCHCHK(h);
    }
    if (step) *step = h->step;
    return read_status(h);
}

int dpd_get_cells(dpd_handle* h, int32_t* cell_start_out, int32_t* ids_out) {
    if (!h) return fail(nullptr, DPD_EINVAL, "handle is NULL");
    if (!h->have_state) return fail(h, DPD_ESTATE, "dpd_get_cells before dpd_set_state");
    const DevParams& P = h->d.P;
    if (cell_start_out)
        HIPCHK(h, hipMemcpyAsync(cell_start_out, h->cs, ((size_t)P.n_cells + 1) * 4,
                                 hipMemcpyDeviceToDevice, h->stream));
    if (ids_out)
        HIPCHK(h, hipMemcpyAsync(ids_out, h->Sid, (size_t)P.N * 4, hipMemcpyDeviceToDevice,
                                 h->stream));
    return read_status(h);
}

int dpd_bin_velocity(dpd_handle* h, int32_t M, double eps, int32_t mode, float* u_out,
                     int32_t* n_out) {
    if (!h) return fail(nullptr, DPD_EINVAL, "handle is NULL");
    if (!h->have_state) return fail(h, DPD_ESTATE, "dpd_bin_velocity before dpd_set_state");
    if (M < 1 || M > h->d.bin_M_max) return fail(h, DPD_EINVAL, fmt("M = %d outside [1, %d]", M, h->d.bin_M_max));
    if (mode != 0 && mode != 1) return fail(h, DPD_EINVAL, "mode must be 0 or 1");
    if (!u_out || !n_out) return fail(h, DPD_EINVAL, "u_out and n_out must not be NULL");
    if (!std::isfinite(eps)) return fail(h, DPD_EINVAL, "eps must be finite");
    try {
        const DevParams& P = h->d.P;
        // 64-bit fixed point: |v| <= 2^16 and <= 2^ceil(log2 n) contributors per bin
        const long long n_src = mode == 0 ? P.N : P.N / 2;
        int lg = 0;
        while ((1LL << lg) < n_src + 1) ++lg;
        const int S = std::min(32, 46 - lg);
        const double qscale = std::ldexp(1.0, S);
        if (mode == 0 && eps <= 0.0 && M <= 2048) {
            // plain bins of particle velocities: one block per grid row, read
            // straight from the canonical state
            BinRowArgs r;
            r.Q = std::max(1, std::min(8, M / 32));
            r.x = h->Sx;
            r.v = h->Sv;
            r.cs = h->cs;
            r.u = (float2*)u_out;
            r.n = (int*)n_out;
            r.status = h->status;
            r.M = M;
            r.nc = P.nc;
            r.L = h->p.L;
            r.inv_dx = (double)M / h->p.L;
            r.qscale = qscale;
            r.vmax = 65536.0;
            const size_t lds = (size_t)((M + r.Q - 1) / r.Q) * 24;
            hipLaunchKernelGGL(k_bin_rows, dim3(r.Q, M), dim3(kBinRowBlock), lds, h->stream, r);
            LAUNCHCHK(h);
            return DPD_OK;
        }
        // id-order copies of x and v into the scratch buffers (which may hold the
        // prepared next step)
        int rc0 = unprepare(h);
        if (rc0) return rc0;
        hipLaunchKernelGGL(k_unpermute, dim3(grid_for(P.N)), dim3(kBlock), 0, h->stream, P.N,
                           (const int*)h->Sid, (const float2*)h->Sx, h->Bx);
        hipLaunchKernelGGL(k_unpermute, dim3(grid_for(P.N)), dim3(kBlock), 0, h->stream, P.N,
                           (const int*)h->Sid, (const float2*)h->Sv, h->Bu);
        const long long nbin = (long long)M * M;
        hipLaunchKernelGGL(k_fill_i32, dim3(grid_for(nbin * 6)), dim3(kBlock), 0, h->stream,
                           (int*)h->binacc, 0, nbin * 6);
        LAUNCHCHK(h);
        BinArgs b;
        b.x = h->Bx;
        b.v = h->Bu;
        b.acc = h->binacc;
        b.status = h->status;
        b.n_src = mode == 0 ? P.N : P.N / 2;
        b.mode = mode;
        b.M = M;
        b.L = h->p.L;
        b.inv_dx = (double)M / h->p.L;
        b.dx = h->p.L / (double)M;
        b.eps = eps;
        b.qscale = qscale;
        b.vmax = 65536.0;
        hipLaunchKernelGGL(k_bin_accum, dim3(grid_for(b.n_src)), dim3(kBlock), 0, h->stream, b);
        hipLaunchKernelGGL(k_bin_finalize, dim3(grid_for(nbin)), dim3(kBlock), 0, h->stream,
                           (int)nbin, (const long long*)h->binacc, b.qscale, (float2*)u_out,
                           (int*)n_out);
        LAUNCHCHK(h);
        return DPD_OK;
    } catch (...) {
        return fail(h, DPD_EINVAL, "internal error");
    }
}

int dpd_sync(dpd_handle* h) {
    if (!h) return fail(nullptr, DPD_EINVAL, "handle is NULL");
    return read_status(h);
}

int dpd_rng_words(const dpd_params* p, const int32_t* i, const int32_t* j, int64_t step,
                  int32_t n, uint32_t* words_out, float* alpha_out, void* stream) {
    Derived d;
    std::string err;
    int rc = derive(p, &d, &err);
    if (rc) return fail(nullptr, rc, err);
    if (n < 0 || !i || !j || !words_out) return fail(nullptr, DPD_EINVAL, "bad arguments");
    if (n == 0) return DPD_OK;
    hipStream_t s = (hipStream_t)stream;
    hipLaunchKernelGGL(k_rng_words, dim3(grid_for(n)), dim3(kBlock), 0, s, d.P, (const int*)i,
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

}  // extern "C"
