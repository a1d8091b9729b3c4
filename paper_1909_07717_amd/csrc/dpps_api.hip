// dpps_api.hip -- host runtime and C ABI of libdpps (see include/dpps.h).
//
// The runtime validates requests, lays out outputs, builds the tile list
// (bookkeeping only: which window and which first point each tile covers),
// stages inputs through pinned memory, and launches the kernels of
// dpps_kernels.hip.  Every step of the search itself runs on the GPU.
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdarg.h>
#include <stdint.h>
#include <stdio.h>
#include <string.h>

#include <new>
#include <string>
#include <vector>

#include "runtime.h"

using namespace dpps;

namespace dpps {

thread_local std::string g_last_error;

int fail(int code, const char *fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_last_error = buf;
    return code;
}

bool finite_pos(float x) { return isfinite(x) && x > 0.0f; }

int lattice_dim(float len, float h, int32_t *n)
{
    double q = (double)len / (double)h;
    double r = nearbyint(q);
    if (!(fabs(q - r) <= 1e-3) || r < 1.0 || r > 1e6) return -1;
    *n = (int32_t)r + 1;
    return 0;
}

int check_params(const dpps_params *p)
{
    if (!p) return fail(DPPS_E_INVALID, "params is NULL");
    const float pos[] = {p->field_len, p->field_wid, p->goal_width, p->robot_radius, p->vmax,
                         p->amax, p->slide_decel, p->roll_decel, p->gravity, p->dist_norm,
                         p->goal_eps};
    for (float x : pos)
        if (!finite_pos(x)) return fail(DPPS_E_INVALID, "a positive parameter is not positive/finite");
    const float fin[] = {p->goal_x, p->margin_s, p->margin_cap_s, p->w_angle, p->w_dist,
                         p->w_margin};
    for (float x : fin)
        if (!isfinite(x)) return fail(DPPS_E_INVALID, "a parameter is not finite");
    if (!(p->slide_ratio > 0.0f && p->slide_ratio < 1.0f))
        return fail(DPPS_E_INVALID, "slide_ratio must be in (0, 1)");
    if (!(p->roll_decel < p->slide_decel))
        return fail(DPPS_E_INVALID, "roll_decel must be below slide_decel");
    if (!(p->chip_angle > 0.0f && p->chip_angle < 1.5707f))
        return fail(DPPS_E_INVALID, "chip_angle must be in (0, pi/2)");
    if (p->n_samples != 64 && p->n_samples != 128 && p->n_samples != 192 && p->n_samples != 256)
        return fail(DPPS_E_INVALID, "n_samples must be 64, 128, 192 or 256 (got %d)", p->n_samples);
    if (p->out_flags & ~DPPS_OUT_REDUCED) return fail(DPPS_E_INVALID, "unknown out_flags bits");
    if (p->reserved != 0) return fail(DPPS_E_INVALID, "reserved must be 0");
    if (p->margin_cap_s < 0.0f) return fail(DPPS_E_INVALID, "margin_cap_s < 0");
    return DPPS_OK;
}

DevParams derive(const dpps_params *p)
{
    DevParams P;
    memset(&P, 0, sizeof P);
    double A = p->amax, V = p->vmax, as = p->slide_decel, ar = p->roll_decel;
    double rho = p->slide_ratio, th = p->chip_angle, g = p->gravity;
    P.field_len = p->field_len;
    P.field_wid = p->field_wid;
    P.goal_x = p->goal_x;
    P.half_goal_w = 0.5f * p->goal_width;
    P.goal_eps = p->goal_eps;
    P.R = p->robot_radius;
    P.RA = (float)(p->robot_radius * A);
    P.V = p->vmax;
    P.A = p->amax;
    P.invV = (float)(1.0 / V);
    P.Vh = (float)(V / sqrt(2.0));
    P.V2 = (float)(V * V);
    P.inv2V = (float)(0.5 / V);
    P.halfV = (float)(0.5 * V);
    P.invA2 = (float)(2.0 / A);
    P.a_s = p->slide_decel;
    P.a_r = p->roll_decel;
    P.ratio = p->slide_ratio;
    P.cos_th = (float)cos(th);
    double lam2 = cos(th), lam3 = 2.0 * sin(th) / g, lam1 = lam2 * lam3;
    P.lam1_inv = (float)(1.0 / lam1);
    // flat: slide time k1 v0, slide distance k2 v0^2, roll time k3 v0, roll distance k4 v0^2
    double k1 = (1.0 - rho) / as, k2 = (1.0 - rho * rho) / (2.0 * as);
    double k3 = rho / ar, k4 = rho * rho / (2.0 * ar);
    double cD = k2 + k4, cTs = k1 + k3;
    P.f_icD = (float)(1.0 / cD);
    P.f_icA = (float)(cTs * cTs / cD);
    P.f_icB = (float)(1.0 / (1.0 / k1 - 0.5 * as));
    double fal = k2 - rho * k1 - 0.5 * ar * k1 * k1, fbe = rho + ar * k1;
    P.f_alpha = (float)fal;
    P.f_hbeta = (float)(0.5 * fbe);
    P.f_hbeta2 = (float)(0.25 * fbe * fbe);
    P.f_hfast = (float)(0.5 * as);
    P.f_pfast = 1.0f;
    // chip: flight time lam3 v0, carry lam1 v0^2, then roll from lam2 v0
    double ccD = lam1 + lam2 * lam2 / (2.0 * ar), ccTs = lam3 + lam2 / ar;
    P.c_icD = (float)(1.0 / ccD);
    P.c_icA = (float)(ccTs * ccTs / ccD);
    P.c_icB = (float)(lam3 / lam2);
    double cal = -0.5 * ar * lam3 * lam3, cbe = lam2 + ar * lam3;
    P.c_alpha = (float)cal;
    P.c_hbeta = (float)(0.5 * cbe);
    P.c_hbeta2 = (float)(0.25 * cbe * cbe);
    P.c_hfast = 0.0f;
    P.c_pfast = (float)lam2;
    P.half_ar = (float)(0.5 * ar);
    P.margin_cap = p->margin_cap_s;
    P.w_ang_pi = (float)(p->w_angle / M_PI);
    P.w_dist = p->w_dist;
    P.inv_dist_norm = (float)(1.0 / p->dist_norm);
    P.w_margin = p->w_margin;
    P.K = p->n_samples;
    P.out_flags = (int32_t)p->out_flags;
    P.bp.a_s = p->slide_decel;
    P.bp.a_r = p->roll_decel;
    P.bp.ratio = p->slide_ratio;
    P.bp.cos_th = cos((double)p->chip_angle);
    P.bp.sin_th = sin((double)p->chip_angle);
    P.bp.g = p->gravity;
    P.margin_d = p->margin_s;
    P.invK_d = 1.0 / (double)p->n_samples;
    return P;
}

int build_tables(const dpps_params *p, int32_t n_frames, const dpps_frame *frames,
                 const dpps_robot *robots, const dpps_window *windows,
                 const dpps_variant *variants, int tile_points, HostTables &T)
{
    if (n_frames < 0) return fail(DPPS_E_INVALID, "n_frames < 0");
    if (n_frames > 0 && (!frames || !robots || !windows || !variants))
        return fail(DPPS_E_INVALID, "NULL input array");
    // cleared, not reallocated: repeated calls reuse the vectors' storage
    T.frames.clear();
    T.robots.clear();
    T.variants.clear();
    T.wins.clear();
    T.tiles.clear();
    T.points = 0;
    T.frames.reserve(n_frames);
    const bool reduced = (p->out_flags & DPPS_OUT_REDUCED) != 0;
    for (int32_t f = 0; f < n_frames; ++f) {
        const dpps_frame &F = frames[f];
        if (F.n_team < 1 || F.n_team > DPPS_MAX_SIDE || F.n_opp < 0 || F.n_opp > DPPS_MAX_SIDE)
            return fail(DPPS_E_INVALID, "frame %d: n_team %d / n_opp %d out of range", f, F.n_team,
                        F.n_opp);
        if (F.passer < 0 || F.passer >= F.n_team)
            return fail(DPPS_E_INVALID, "frame %d: passer %d out of range", f, F.passer);
        if (F.robot_off < 0 || F.window_off < 0 || F.variant_off < 0 || F.n_windows < 0)
            return fail(DPPS_E_INVALID, "frame %d: negative offset", f);
        if (F.n_variants < 1) return fail(DPPS_E_INVALID, "frame %d: no variants", f);
        if (F.n_variants > DPPS_MAX_VARIANTS)
            return fail(DPPS_E_UNSUPPORTED, "frame %d: %d variants (max %d)", f, F.n_variants,
                        DPPS_MAX_VARIANTS);
        if (reduced && F.n_variants > 255)
            return fail(DPPS_E_UNSUPPORTED, "frame %d: too many variants for REDUCED", f);
        if (!isfinite(F.ball_x) || !isfinite(F.ball_y))
            return fail(DPPS_E_INVALID, "frame %d: ball not finite", f);
        if (F.out_off < 0) return fail(DPPS_E_INVALID, "frame %d: out_off < 0", f);
        FrameDev D;
        memset(&D, 0, sizeof D);
        D.n_team = F.n_team;
        D.n_opp = F.n_opp;
        D.passer = F.passer;
        D.robot_off = (int32_t)T.robots.size();
        D.n_windows = F.n_windows;
        D.win_off = (int32_t)T.wins.size();
        D.n_variants = F.n_variants;
        D.variant_off = (int32_t)T.variants.size();
        D.ball_x = F.ball_x;
        D.ball_y = F.ball_y;
        for (int r = 0; r < F.n_team + F.n_opp; ++r) {
            const dpps_robot &R = robots[F.robot_off + r];
            if (!isfinite(R.x) || !isfinite(R.y) || !isfinite(R.vx) || !isfinite(R.vy))
                return fail(DPPS_E_INVALID, "frame %d robot %d: not finite", f, r);
            T.robots.push_back(R);
        }
        for (int v = 0; v < F.n_variants; ++v) {
            const dpps_variant &Vv = variants[F.variant_off + v];
            if (Vv.type != DPPS_FLAT && Vv.type != DPPS_CHIP)
                return fail(DPPS_E_INVALID, "frame %d variant %d: bad type %d", f, v, Vv.type);
            if (!finite_pos(Vv.v0) || Vv.v0 > 100.0f)
                return fail(DPPS_E_INVALID, "frame %d variant %d: v0 must be in (0, 100]", f, v);
            T.variants.push_back(Vv);
        }
        int64_t elem = 0;
        const int32_t tile_begin = (int32_t)T.tiles.size();
        for (int w = 0; w < F.n_windows; ++w) {
            const dpps_window &Wn = windows[F.window_off + w];
            int32_t Nx, Ny;
            if (!finite_pos(Wn.h) || lattice_dim(p->field_len, Wn.h, &Nx) ||
                lattice_dim(p->field_wid, Wn.h, &Ny))
                return fail(DPPS_E_INVALID, "frame %d window %d: spacing %g does not divide the field",
                            f, w, (double)Wn.h);
            if (Wn.nx < 0 || Wn.ny < 0 || Wn.i0 < 0 || Wn.j0 < 0 || Wn.i0 + Wn.nx > Nx ||
                Wn.j0 + Wn.ny > Ny)
                return fail(DPPS_E_INVALID, "frame %d window %d: outside the %dx%d lattice", f, w,
                            Nx, Ny);
            WinDev W;
            memset(&W, 0, sizeof W);
            W.h = Wn.h;
            W.i0 = Wn.i0;
            W.j0 = Wn.j0;
            W.nx = Wn.nx;
            W.ny = Wn.ny;
            W.halfNx = 0.5f * (float)(Nx - 1);
            W.halfNy = 0.5f * (float)(Ny - 1);
            W.frame = f;
            W.npts = Wn.nx * Wn.ny;
            W.elem_base = (int32_t)elem;
            W.out_base = F.out_off + elem;
            elem += (int64_t)W.npts * (reduced ? 1 : F.n_variants);
            if (elem >= 0x7FFFFFFF)
                return fail(DPPS_E_UNSUPPORTED, "frame %d: more than 2^31 output elements", f);
            int32_t widx = (int32_t)T.wins.size();
            if (tile_points > 0)
                for (int32_t p0 = 0; p0 < W.npts; p0 += tile_points) T.tiles.push_back({widx, p0});
            T.points += W.npts;
            T.wins.push_back(W);
        }
        D.tile_begin = tile_begin;
        D.tile_count = (int32_t)T.tiles.size() - tile_begin;
        T.frames.push_back(D);
    }
    // full (non-reduced) keys index elements as window base + v * npts + p
    if (reduced) {
        // in REDUCED mode the key still encodes the variant: rebase per frame
        for (auto &F : T.frames) {
            int64_t e = 0;
            for (int w = 0; w < F.n_windows; ++w) {
                WinDev &W = T.wins[F.win_off + w];
                W.elem_base = (int32_t)e;
                e += (int64_t)W.npts * F.n_variants;
            }
        }
    }
    return DPPS_OK;
}

}  // namespace dpps

// ----------------------------------------------------------------------------
// contexts and batches
// ----------------------------------------------------------------------------

size_t align_up(size_t x, size_t a) { return (x + a - 1) / a * a; }

int arena_reserve(dpps_ctx *c, DeviceArena &A, size_t bytes)
{
    if (bytes <= A.cap) return DPPS_OK;
    size_t want = align_up(bytes + bytes / 4, 1 << 16);
    if (c->p.hbm_budget_bytes && c->budget_used - A.cap + want > c->p.hbm_budget_bytes) {
        want = bytes;
        if (c->budget_used - A.cap + want > c->p.hbm_budget_bytes)
            return fail(DPPS_E_BUDGET, "request needs %zu device bytes; budget %llu (in use %llu)",
                        bytes, (unsigned long long)c->p.hbm_budget_bytes,
                        (unsigned long long)c->budget_used);
    }
    if (A.ptr) {
        HIP_OK(hipStreamSynchronize(c->stream));
        HIP_OK(hipFree(A.ptr));
        c->budget_used -= A.cap;
        A.ptr = nullptr;
        A.cap = 0;
    }
    if (hipMalloc(&A.ptr, want) != hipSuccess) {
        (void)hipGetLastError();
        A.ptr = nullptr;
        return fail(DPPS_E_NOMEM, "hipMalloc(%zu) failed", want);
    }
    A.cap = want;
    c->budget_used += want;
    return DPPS_OK;
}

void graph_drop(dpps_batch *b)
{
    if (b->exec) (void)hipGraphExecDestroy(b->exec);
    if (b->graph) (void)hipGraphDestroy(b->graph);
    b->exec = nullptr;
    b->graph = nullptr;
}

void ring_free(dpps_ctx *c)
{
    for (hipEvent_t e : c->ring0) (void)hipEventDestroy(e);
    for (hipEvent_t e : c->ring1) (void)hipEventDestroy(e);
    c->ring0.clear();
    c->ring1.clear();
    c->ring_used = 0;
}

Layout table_layout(const HostTables &T)
{
    Layout L;
    size_t o = 0;
    L.off_frames = o; o = align_up(o + T.frames.size() * sizeof(FrameDev), 256);
    L.off_robots = o; o = align_up(o + T.robots.size() * sizeof(dpps_robot), 256);
    L.off_variants = o; o = align_up(o + T.variants.size() * sizeof(dpps_variant), 256);
    L.off_wins = o; o = align_up(o + T.wins.size() * sizeof(WinDev), 256);
    L.off_tiles = o; o = align_up(o + T.tiles.size() * sizeof(TileDev), 256);
    L.total = o < 256 ? 256 : o;
    return L;
}

void pack_tables(const HostTables &T, const Layout &L, char *dst)
{
    if (!T.frames.empty()) memcpy(dst + L.off_frames, T.frames.data(), T.frames.size() * sizeof(FrameDev));
    if (!T.robots.empty()) memcpy(dst + L.off_robots, T.robots.data(), T.robots.size() * sizeof(dpps_robot));
    if (!T.variants.empty())
        memcpy(dst + L.off_variants, T.variants.data(), T.variants.size() * sizeof(dpps_variant));
    if (!T.wins.empty()) memcpy(dst + L.off_wins, T.wins.data(), T.wins.size() * sizeof(WinDev));
    if (!T.tiles.empty()) memcpy(dst + L.off_tiles, T.tiles.data(), T.tiles.size() * sizeof(TileDev));
}

int batch_reserve(dpps_ctx *c, dpps_batch *b, const Layout &L)
{
    int rc = arena_reserve(c, b->arena, L.total);
    if (rc) return rc;
    char *base = (char *)b->arena.ptr;
    b->d_frames = (FrameDev *)(base + L.off_frames);
    b->d_robots = (dpps_robot *)(base + L.off_robots);
    b->d_variants = (dpps_variant *)(base + L.off_variants);
    b->d_wins = (WinDev *)(base + L.off_wins);
    b->d_tiles = (TileDev *)(base + L.off_tiles);
    size_t n = (size_t)(b->n_frames > 0 ? b->n_frames : 1);
    size_t nt = b->T.tiles.size() > 0 ? b->T.tiles.size() : 1;
    size_t aux = 256 + align_up(nt * sizeof(TileRec), 256) + n * sizeof(dpps_best);
    void *old = b->aux.ptr;
    rc = arena_reserve(c, b->aux, aux);
    if (rc) return rc;
    char *ab = (char *)b->aux.ptr;
    b->d_counter = (uint32_t *)ab;
    b->d_tile_rec = (TileRec *)(ab + 256);
    b->d_best = (dpps_best *)(ab + 256 + align_up(nt * sizeof(TileRec), 256));
    // a fresh allocation starts with the work counter at zero; afterwards the
    // finalize kernel rearms it at the end of every launch
    if (b->aux.ptr != old) HIP_OK(hipMemset(b->aux.ptr, 0, 256));
    return DPPS_OK;
}

// Regenerate the tile list for b->tile_points (frames and windows unchanged).
void retile(HostTables &T, int tile_points)
{
    T.tiles.clear();
    for (FrameDev &F : T.frames) {
        F.tile_begin = (int32_t)T.tiles.size();
        for (int w = 0; w < F.n_windows; ++w) {
            const int32_t widx = F.win_off + w;
            for (int32_t p0 = 0; p0 < T.wins[widx].npts; p0 += tile_points)
                T.tiles.push_back({widx, p0});
        }
        F.tile_count = (int32_t)T.tiles.size() - F.tile_begin;
    }
}

// Synchronous upload of a batch's tables (after creation or a new tile size).
int batch_upload(dpps_ctx *c, dpps_batch *b)
{
    graph_drop(b);
    retile(b->T, b->tile_points);
    Layout L = table_layout(b->T);
    int rc = batch_reserve(c, b, L);
    if (rc) return rc;
    std::vector<char> host(L.total);
    pack_tables(b->T, L, host.data());
    HIP_OK(hipStreamSynchronize(c->stream));
    HIP_OK(hipMemcpy(b->arena.ptr, host.data(), L.total, hipMemcpyHostToDevice));
    return DPPS_OK;
}

int run_batch(dpps_ctx *c, dpps_batch *b, const dpps_outputs *out, hipStream_t st,
                     bool timed, const dpps_power_params *power, float *v0_out)
{
    if (!out) return fail(DPPS_E_INVALID, "outputs is NULL");
    if (b->tile_points != c->tile_points)
        return fail(DPPS_E_INVALID, "batch built for tile_points %d, context now uses %d",
                    b->tile_points, c->tile_points);
    LaunchArgs a;
    memset(&a, 0, sizeof a);
    a.P = c->P;
    a.frames = b->d_frames;
    a.robots = b->d_robots;
    a.variants = b->d_variants;
    a.wins = b->d_wins;
    a.tiles = b->d_tiles;
    a.n_tiles = (int32_t)b->T.tiles.size();
    a.n_frames = b->n_frames;
    a.tile_points = c->tile_points;
    // the search kernel cuts a tile into chunks of 4 points
    if (a.tile_points < 4 || a.tile_points % 4)
        return fail(DPPS_E_INVALID, "tile_points %d is not a multiple of 4", a.tile_points);
    a.persistent = c->persistent;
    a.counter = b->d_counter;
    a.tile_rec = b->d_tile_rec;
    a.mask = out->mask;
    a.score = out->score;
    bool reduced = (c->p.out_flags & DPPS_OUT_REDUCED) != 0;
    a.t_team = reduced ? nullptr : out->t_team;
    a.t_opp = reduced ? nullptr : out->t_opp;
    a.best = out->best ? out->best : b->d_best;
    if (power) {
        a.power = 1;
        a.p_buffer = power->buffer_s;
        a.p_vmin = power->v_min;
        a.p_vmax = power->v_max;
        a.v0_out = v0_out;
    }
    int per_cu = c->wg_per_cu > 0 ? c->wg_per_cu
                                  : search_occupancy(c->p.n_samples, c->waves, c->tile_points);
    int64_t cap = (int64_t)c->n_cu * per_cu;
    int grid = (int)(a.n_tiles < cap ? a.n_tiles : cap);
    if (!c->persistent) grid = a.n_tiles;
    // one frame on a persistent grid: one best record per workgroup
    if (c->persistent && b->n_frames == 1) a.wg_records = grid;
    void *e0 = timed ? (void *)c->ev0 : nullptr, *e1 = timed ? (void *)c->ev1 : nullptr;
    if (timed && c->ring_used < (int)c->ring0.size()) {
        e0 = (void *)c->ring0[c->ring_used];
        e1 = (void *)c->ring1[c->ring_used];
        ++c->ring_used;
    }
    int rc = launch_search(a, c->waves, grid, (void *)st, e0, e1);
    c->timed = timed && e1 == (void *)c->ev1;
    if (rc) {
        hipError_t e = hipGetLastError();
        return fail(DPPS_E_DEVICE, "kernel launch failed: %s", hipGetErrorString(e));
    }
    return DPPS_OK;
}

extern "C" {

const char *dpps_strerror(int code)
{
    switch (code) {
    case DPPS_OK: return "ok";
    case DPPS_E_INVALID: return "invalid argument";
    case DPPS_E_NOMEM: return "out of memory";
    case DPPS_E_DEVICE: return "HIP device error";
    case DPPS_E_BUDGET: return "device memory budget exceeded";
    case DPPS_E_UNSUPPORTED: return "unsupported request";
    default: return "unknown error";
    }
}

const char *dpps_last_error(void) { return g_last_error.c_str(); }

int dpps_version(void) { return 1; }

int dpps_create(dpps_ctx **out, const dpps_params *p, int device, void *hip_stream)
{
    if (!out) return fail(DPPS_E_INVALID, "out is NULL");
    *out = nullptr;
    int rc = check_params(p);
    if (rc) return rc;
    int ndev = 0;
    HIP_OK(hipGetDeviceCount(&ndev));
    if (device < 0 || device >= ndev) return fail(DPPS_E_INVALID, "device %d of %d", device, ndev);
    dpps_ctx *c = new (std::nothrow) dpps_ctx();
    if (!c) return fail(DPPS_E_NOMEM, "context allocation failed");
    c->p = *p;
    c->P = derive(p);
    c->device = device;
    c->scratch.ctx = c;
    c->fallback.ctx = c;
    c->rays.ctx = c;
    c->shots.ctx = c;
    c->runs.ctx = c;
    if (hipSetDevice(device) != hipSuccess) {
        delete c;
        return fail(DPPS_E_DEVICE, "hipSetDevice(%d) failed", device);
    }
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, device) == hipSuccess && prop.multiProcessorCount > 0)
        c->n_cu = prop.multiProcessorCount;
    if (hip_stream) {
        c->stream = (hipStream_t)hip_stream;
    } else {
        // a blocking stream: ordered with the legacy default stream, so callers
        // that pass no stream see results in default-stream order
        if (hipStreamCreate(&c->stream) != hipSuccess) {
            delete c;
            return fail(DPPS_E_DEVICE, "hipStreamCreate failed");
        }
        c->own_stream = true;
    }
    if (hipEventCreateWithFlags(&c->staged, hipEventDisableTiming) != hipSuccess ||
        hipEventCreateWithFlags(&c->landed, hipEventDisableTiming) != hipSuccess ||
        hipEventCreate(&c->ev0) != hipSuccess || hipEventCreate(&c->ev1) != hipSuccess) {
        dpps_destroy(c);
        return fail(DPPS_E_DEVICE, "hipEventCreate failed");
    }
    rc = noalloc_setup(c);
    if (rc) {
        const std::string msg = dpps_last_error();
        dpps_destroy(c);
        return fail(rc, "%s", msg.c_str());
    }
    *out = c;
    return DPPS_OK;
}

static void batch_free_device(dpps_batch *b)
{
    graph_drop(b);
    if (b->arena.ptr) (void)hipFree(b->arena.ptr);
    if (b->aux.ptr) (void)hipFree(b->aux.ptr);
    if (b->ctx) b->ctx->budget_used -= b->arena.cap + b->aux.cap;
    b->arena = DeviceArena();
    b->aux = DeviceArena();
}

void dpps_destroy(dpps_ctx *c)
{
    if (!c) return;
    if (c->stream) (void)hipStreamSynchronize(c->stream);
    ring_free(c);
    batch_free_device(&c->scratch);
    batch_free_device(&c->fallback);
    batch_free_device(&c->rays);
    batch_free_device(&c->shots);
    batch_free_device(&c->runs);
    if (c->ray_aux.ptr) (void)hipFree(c->ray_aux.ptr);
    if (c->ray_dirs.ptr) (void)hipFree(c->ray_dirs.ptr);
    noalloc_release(c);
    if (c->pinned) (void)hipHostFree(c->pinned);
    if (c->pinned_best) (void)hipHostFree(c->pinned_best);
    if (c->staged) (void)hipEventDestroy(c->staged);
    if (c->landed) (void)hipEventDestroy(c->landed);
    if (c->ev0) (void)hipEventDestroy(c->ev0);
    if (c->ev1) (void)hipEventDestroy(c->ev1);
    if (c->own_stream && c->stream) (void)hipStreamDestroy(c->stream);
    delete c;
}

int dpps_layout(const dpps_params *p, int32_t n_frames, dpps_frame *frames,
                const dpps_window *windows, int64_t *total)
{
    int rc = check_params(p);
    if (rc) return rc;
    if (!total || n_frames < 0 || (n_frames > 0 && (!frames || !windows)))
        return fail(DPPS_E_INVALID, "bad layout arguments");
    bool reduced = (p->out_flags & DPPS_OUT_REDUCED) != 0;
    int64_t off = 0;
    for (int32_t f = 0; f < n_frames; ++f) {
        frames[f].out_off = off;
        if (frames[f].n_windows < 0 || frames[f].window_off < 0)
            return fail(DPPS_E_INVALID, "frame %d: bad window slice", f);
        for (int w = 0; w < frames[f].n_windows; ++w) {
            const dpps_window &W = windows[frames[f].window_off + w];
            if (W.nx < 0 || W.ny < 0) return fail(DPPS_E_INVALID, "frame %d: negative window", f);
            off += (int64_t)W.nx * W.ny * (reduced ? 1 : frames[f].n_variants);
        }
    }
    *total = off;
    return DPPS_OK;
}

int dpps_request_bytes(const dpps_params *p, int32_t n_frames, const dpps_frame *frames,
                       const dpps_window *windows, int32_t tile_points, uint64_t *bytes)
{
    int rc = check_params(p);
    if (rc) return rc;
    if (!bytes || n_frames < 0 || (n_frames > 0 && (!frames || !windows)))
        return fail(DPPS_E_INVALID, "bad request-size arguments");
    if (tile_points == 0) tile_points = 8;
    if (tile_points < 1) return fail(DPPS_E_INVALID, "tile_points %d", tile_points);
    int64_t nr = 0, nv = 0, nw = 0, nt = 0;
    for (int32_t f = 0; f < n_frames; ++f) {
        const dpps_frame &F = frames[f];
        if (F.n_team < 0 || F.n_opp < 0 || F.n_variants < 0 || F.n_windows < 0 || F.window_off < 0)
            return fail(DPPS_E_INVALID, "frame %d: negative count or offset", f);
        nr += F.n_team + F.n_opp;
        nv += F.n_variants;
        nw += F.n_windows;
        for (int w = 0; w < F.n_windows; ++w) {
            const dpps_window &W = windows[F.window_off + w];
            if (W.nx < 0 || W.ny < 0) return fail(DPPS_E_INVALID, "frame %d: negative window", f);
            nt += ((int64_t)W.nx * W.ny + tile_points - 1) / tile_points;
        }
    }
    // the table arena (table_layout) and the record arena (batch_reserve)
    size_t t = 0;
    t = align_up(t + (size_t)n_frames * sizeof(FrameDev), 256);
    t = align_up(t + (size_t)nr * sizeof(dpps_robot), 256);
    t = align_up(t + (size_t)nv * sizeof(dpps_variant), 256);
    t = align_up(t + (size_t)nw * sizeof(WinDev), 256);
    t = align_up(t + (size_t)nt * sizeof(TileDev), 256);
    if (t < 256) t = 256;
    const size_t aux = 256 + align_up((size_t)(nt > 0 ? nt : 1) * sizeof(TileRec), 256) +
                       (size_t)(n_frames > 0 ? n_frames : 1) * sizeof(dpps_best);
    *bytes = (uint64_t)(t + aux);
    return DPPS_OK;
}

uint64_t dpps_device_bytes(const dpps_ctx *c) { return c ? c->budget_used : 0; }

int dpps_set_launch(dpps_ctx *c, int32_t tile_points, int32_t waves_per_wg, int32_t wg_per_cu)
{
    if (!c) return fail(DPPS_E_INVALID, "ctx is NULL");
    if (tile_points) {
        if (tile_points < 8 || tile_points > 64 || tile_points % 8)
            return fail(DPPS_E_INVALID, "tile_points must be a multiple of 8 in [8, 64]");
        c->tile_points = tile_points;
    }
    if (waves_per_wg) {
        if (waves_per_wg != 1 && waves_per_wg != 2 && waves_per_wg != 4 && waves_per_wg != 8)
            return fail(DPPS_E_INVALID, "waves_per_wg must be 1, 2, 4 or 8");
        c->waves = waves_per_wg;
    }
    if (wg_per_cu) {
        if (wg_per_cu == -1) {
            c->persistent = 0;
        } else if (wg_per_cu == -2) {
            c->persistent = 1;
            c->wg_per_cu = 0;
        } else {
            if (wg_per_cu < 1 || wg_per_cu > 32)
                return fail(DPPS_E_INVALID, "wg_per_cu must be -2, -1 or in [1, 32]");
            c->persistent = 1;
            c->wg_per_cu = wg_per_cu;
        }
    }
    return DPPS_OK;
}

int dpps_get_launch(const dpps_ctx *c, int32_t *tile_points, int32_t *waves_per_wg,
                    int32_t *wg_per_cu)
{
    if (!c) return fail(DPPS_E_INVALID, "ctx is NULL");
    if (tile_points) *tile_points = c->tile_points;
    if (waves_per_wg) *waves_per_wg = c->waves;
    if (wg_per_cu)
        *wg_per_cu = !c->persistent ? -1
                     : c->wg_per_cu > 0 ? c->wg_per_cu
                                        : search_occupancy(c->p.n_samples, c->waves, c->tile_points);
    return DPPS_OK;
}

}  // extern "C"

// Validate host frames and copy their tables into a batch the context owns
// (c->scratch or c->fallback), through the pinned staging buffer and an
// asynchronous copy on st; device memory grows only when a request is larger
// than any before.
int stage_batch(dpps_ctx *c, dpps_batch *b, int32_t n_frames, const dpps_frame *frames,
                const dpps_robot *robots, const dpps_window *windows,
                const dpps_variant *variants, hipStream_t st)
{
    int rc = build_tables(&c->p, n_frames, frames, robots, windows, variants, c->tile_points, b->T);
    if (rc) return rc;
    b->n_frames = n_frames;
    b->tile_points = c->tile_points;
    return stage_tables(c, b, st);
}

int read_best(dpps_ctx *c, dpps_best *h, const dpps_best *d, int n, hipStream_t st)
{
    if (n <= 0) return DPPS_OK;
    if (n > c->pinned_best_cap) {
        // the previous read has completed (every read waits for its copy)
        if (c->pinned_best) HIP_OK(hipHostFree(c->pinned_best));
        c->pinned_best = nullptr;
        c->pinned_best_cap = 0;
        const int64_t want = n < 64 ? 64 : n;
        if (hipHostMalloc((void **)&c->pinned_best, (size_t)want * sizeof(dpps_best),
                          hipHostMallocDefault) != hipSuccess)
            return fail(DPPS_E_NOMEM, "hipHostMalloc of %lld best records failed", (long long)want);
        c->pinned_best_cap = want;
    }
    HIP_OK(hipMemcpyAsync(c->pinned_best, d, (size_t)n * sizeof(dpps_best), hipMemcpyDeviceToHost,
                          st));
    HIP_OK(hipEventRecord(c->landed, st));
    const hipError_t e = hipEventSynchronize(c->landed);
    if (e != hipSuccess) return fail(DPPS_E_DEVICE, "waiting for the best records: %s", hipGetErrorString(e));
    memcpy(h, c->pinned_best, (size_t)n * sizeof(dpps_best));
    return DPPS_OK;
}

// Copy the host tables already in b->T to the batch's device memory through
// the pinned staging buffer (asynchronous on st).
int stage_tables(dpps_ctx *c, dpps_batch *b, hipStream_t st)
{
    int rc;
    graph_drop(b);
    Layout L = table_layout(b->T);
    // the previous call's copy must have left the pinned buffer
    HIP_OK(hipEventSynchronize(c->staged));
    if (L.total > c->pinned_cap) {
        if (c->pinned) HIP_OK(hipHostFree(c->pinned));
        c->pinned = nullptr;
        size_t want = align_up(L.total + L.total / 4, 1 << 16);
        if (hipHostMalloc(&c->pinned, want, hipHostMallocDefault) != hipSuccess) {
            c->pinned_cap = 0;
            return fail(DPPS_E_NOMEM, "hipHostMalloc(%zu) failed", want);
        }
        c->pinned_cap = want;
    }
    rc = batch_reserve(c, b, L);
    if (rc) return rc;
    pack_tables(b->T, L, (char *)c->pinned);
    HIP_OK(hipMemcpyAsync(b->arena.ptr, c->pinned, L.total, hipMemcpyHostToDevice, st));
    HIP_OK(hipEventRecord(c->staged, st));
    return DPPS_OK;
}

extern "C" {

int dpps_search_batch(dpps_ctx *c, int32_t n_frames, const dpps_frame *frames,
                      const dpps_robot *robots, const dpps_window *windows,
                      const dpps_variant *variants, const dpps_outputs *out, void *hip_stream)
{
    if (!c) return fail(DPPS_E_INVALID, "ctx is NULL");
    if (!out) return fail(DPPS_E_INVALID, "outputs is NULL");
    HIP_OK(hipSetDevice(c->device));
    hipStream_t st = hip_stream ? (hipStream_t)hip_stream : c->stream;
    int rc = stage_batch(c, &c->scratch, n_frames, frames, robots, windows, variants, st);
    if (rc) return rc;
    return run_batch(c, &c->scratch, out, st, true);
}

int dpps_search_power(dpps_ctx *c, int32_t n_frames, const dpps_frame *frames,
                      const dpps_robot *robots, const dpps_window *windows,
                      const dpps_power_params *pp, const dpps_outputs *out, float *d_v0,
                      void *hip_stream)
{
    if (!c || !pp || !out) return fail(DPPS_E_INVALID, "NULL argument");
    if (!(pp->buffer_s >= 0.0f) || !isfinite(pp->buffer_s) || !(pp->v_min > 0.0f) ||
        !(pp->v_max >= pp->v_min) || !isfinite(pp->v_max) || pp->v_max > 100.0f ||
        pp->reserved != 0)
        return fail(DPPS_E_INVALID, "power: buffer >= 0, 0 < v_min <= v_max <= 100, reserved 0");
    if (c->p.out_flags & DPPS_OUT_REDUCED)
        return fail(DPPS_E_UNSUPPORTED, "the power search has one variant per point: no REDUCED");
    if (n_frames < 0) return fail(DPPS_E_INVALID, "n_frames < 0");
    HIP_OK(hipSetDevice(c->device));
    hipStream_t st = hip_stream ? (hipStream_t)hip_stream : c->stream;
    if (n_frames == 0) return DPPS_OK;
    if (!frames) return fail(DPPS_E_INVALID, "NULL input array");
    // one flat variant per frame (its speed is computed per point)
    std::vector<dpps_frame> fr(frames, frames + n_frames);
    std::vector<dpps_variant> one(1, dpps_variant{DPPS_FLAT, pp->v_min});
    for (dpps_frame &F : fr) {
        F.n_variants = 1;
        F.variant_off = 0;
    }
    int rc = stage_batch(c, &c->scratch, n_frames, fr.data(), robots, windows, one.data(), st);
    if (rc) return rc;
    return run_batch(c, &c->scratch, out, st, true, pp, d_v0);
}

int dpps_ray_search(dpps_ctx *c, int32_t n_frames, const dpps_frame *frames,
                    const dpps_robot *robots, const dpps_variant *variants,
                    const dpps_ray_params *rp, const dpps_ray_outputs *out, void *hip_stream)
{
    if (!c || !rp || !out || !out->best) return fail(DPPS_E_INVALID, "NULL argument");
    if (rp->n_dirs < 1 || rp->n_dirs > 4096) return fail(DPPS_E_INVALID, "n_dirs must be in [1, 4096]");
    if (!(rp->w_time >= 0.0f) || !isfinite(rp->w_time) || !(rp->w_refract >= 0.0f) ||
        !isfinite(rp->w_refract) || rp->reserved != 0)
        return fail(DPPS_E_INVALID, "ray weights must be finite and >= 0, reserved 0");
    if (n_frames < 0) return fail(DPPS_E_INVALID, "n_frames < 0");
    HIP_OK(hipSetDevice(c->device));
    hipStream_t st = hip_stream ? (hipStream_t)hip_stream : c->stream;
    if (n_frames == 0) return DPPS_OK;
    if (!frames) return fail(DPPS_E_INVALID, "NULL input array");
    // validate as for dpps_search_batch, the windows aside
    std::vector<dpps_frame> fr(frames, frames + n_frames);
    for (dpps_frame &F : fr) {
        F.n_windows = 0;
        F.window_off = 0;
        F.out_off = 0;
    }
    const dpps_window no_window = {0.0f, 0, 0, 0, 0};
    dpps_batch *b = &c->rays;
    int rc = build_tables(&c->p, n_frames, fr.data(), robots, &no_window, variants, c->tile_points,
                          b->T);
    if (rc) return rc;
    // tiles of directions of one frame; outputs frame by frame.  A tile
    // holds one direction per wave and up to ray_tile_dirs when there are
    // enough directions to give every resident workgroup four such tiles (a
    // single frame runs one direction per wave, for latency)
    const int rw = c->ray_waves > 0 ? c->ray_waves : c->waves;
    const int64_t ray_cap = (int64_t)c->n_cu * ray_occupancy(c->p.n_samples, rw);
    const int64_t per_wg = (int64_t)n_frames * rp->n_dirs / (4 * ray_cap);
    int td = (int)(per_wg < c->ray_tile_dirs ? per_wg : c->ray_tile_dirs) / rw * rw;
    if (td < rw) td = rw;
    b->T.tiles.clear();
    int64_t base = 0;
    for (int32_t f = 0; f < n_frames; ++f) {
        FrameDev &F = b->T.frames[f];
        F.tile_begin = (int32_t)b->T.tiles.size();
        for (int d0 = 0; d0 < rp->n_dirs; d0 += td) b->T.tiles.push_back({f, d0});
        F.tile_count = (int32_t)b->T.tiles.size() - F.tile_begin;
        F.ray_base = base;
        base += (int64_t)rp->n_dirs * F.n_variants;
    }
    b->n_frames = n_frames;
    b->tile_points = c->tile_points;
    rc = stage_tables(c, b, st);
    if (rc) return rc;
    const size_t nt = b->T.tiles.size();
    void *old = c->ray_aux.ptr;
    rc = arena_reserve(c, c->ray_aux, 256 + nt * sizeof(RayRec));
    if (rc) return rc;
    // a fresh allocation starts with the work counter at zero; afterwards the
    // finalize kernel rearms it at the end of every launch
    if (c->ray_aux.ptr != old) HIP_OK(hipMemset(c->ray_aux.ptr, 0, 256));
    // the direction table, recomputed when the direction count changes (and
    // waited for, so that calls on other streams read it complete)
    if (c->ray_dirs_n != rp->n_dirs) {
        rc = arena_reserve(c, c->ray_dirs, 4096 * sizeof(double2));
        if (rc) return rc;
        if (launch_ray_dirs((double2 *)c->ray_dirs.ptr, rp->n_dirs, (void *)st))
            return fail(DPPS_E_DEVICE, "direction table launch failed");
        HIP_OK(hipStreamSynchronize(st));
        c->ray_dirs_n = rp->n_dirs;
    }
    RayArgs a;
    memset(&a, 0, sizeof a);
    a.P = c->P;
    a.frames = b->d_frames;
    a.robots = b->d_robots;
    a.variants = b->d_variants;
    a.tiles = b->d_tiles;
    a.dirs = (const double2 *)c->ray_dirs.ptr;
    a.n_tiles = (int32_t)nt;
    a.n_frames = n_frames;
    a.tile_dirs = td;
    a.n_dirs = rp->n_dirs;
    a.w_time = rp->w_time;
    a.w_refract = rp->w_refract;
    a.counter = (uint32_t *)c->ray_aux.ptr;
    a.tile_rec = (RayRec *)((char *)c->ray_aux.ptr + 256);
    a.mask = out->mask;
    a.score = out->score;
    a.t_team = out->t_team;
    a.t_opp = out->t_opp;
    a.s_recv = out->s_recv;
    a.best = out->best;
    const int grid = (int)((int64_t)nt < ray_cap ? (int64_t)nt : ray_cap);
    // with a timing ring open (dpps_timing_begin), the ray kernel is timed
    void *e0 = nullptr, *e1 = nullptr;
    if (c->ring_used < (int)c->ring0.size()) {
        e0 = (void *)c->ring0[c->ring_used];
        e1 = (void *)c->ring1[c->ring_used];
        ++c->ring_used;
    }
    if (launch_ray(a, rw, grid, (void *)st, e0, e1))
        return fail(DPPS_E_DEVICE, "ray launch failed");
    return DPPS_OK;
}

int dpps_shot_decision(dpps_ctx *c, int32_t n_frames, const dpps_frame *frames,
                       const dpps_robot *robots, const dpps_window *windows,
                       const dpps_shot_params *sp, dpps_shot *d_ball, dpps_shot *d_map,
                       void *hip_stream)
{
    if (!c || !sp || !d_ball) return fail(DPPS_E_INVALID, "NULL argument");
    if (!(sp->v_shot > 0.0f) || !(sp->v_shot <= 100.0f) || !(sp->min_angle >= 0.0f) ||
        !isfinite(sp->min_angle) || !(sp->margin_s >= 0.0f) || !isfinite(sp->margin_s) ||
        sp->reserved != 0)
        return fail(DPPS_E_INVALID,
                    "shot: 0 < v_shot <= 100, finite min_angle >= 0 and margin_s >= 0, reserved 0");
    if (n_frames < 0) return fail(DPPS_E_INVALID, "n_frames < 0");
    HIP_OK(hipSetDevice(c->device));
    hipStream_t st = hip_stream ? (hipStream_t)hip_stream : c->stream;
    if (n_frames == 0) return DPPS_OK;
    if (!frames) return fail(DPPS_E_INVALID, "NULL input array");
    // one (unused) flat variant per frame; without a map the windows are skipped
    std::vector<dpps_frame> fr(frames, frames + n_frames);
    const dpps_variant one = {DPPS_FLAT, sp->v_shot};
    for (dpps_frame &F : fr) {
        F.n_variants = 1;
        F.variant_off = 0;
        if (!d_map) {
            F.n_windows = 0;
            F.window_off = 0;
        }
    }
    const dpps_window no_window = {0.0f, 0, 0, 0, 0};
    dpps_batch *b = &c->shots;
    int rc = build_tables(&c->p, n_frames, fr.data(), robots, d_map ? windows : &no_window, &one,
                          c->shot_tile, b->T);
    if (rc) return rc;
    b->n_frames = n_frames;
    b->tile_points = c->shot_tile;
    rc = stage_tables(c, b, st);
    if (rc) return rc;
    ShotArgs a;
    memset(&a, 0, sizeof a);
    a.P = c->P;
    a.frames = b->d_frames;
    a.robots = b->d_robots;
    a.variants = b->d_variants;
    a.wins = b->d_wins;
    a.tiles = b->d_tiles;
    a.n_tiles = (int32_t)b->T.tiles.size();
    a.n_frames = n_frames;
    a.tile_points = c->shot_tile;
    a.v_shot = sp->v_shot;
    a.min_angle = sp->min_angle;
    a.margin = sp->margin_s;
    a.ball = d_ball;
    a.map = d_map;
    if (launch_shot(a, c->shot_waves, (void *)st)) return fail(DPPS_E_DEVICE, "shot launch failed");
    return DPPS_OK;
}

int dpps_running_points(dpps_ctx *c, int32_t n_frames, const dpps_frame *frames,
                        const dpps_robot *robots, const dpps_window *zones,
                        const dpps_run_params *rp, float *d_score, dpps_run_best *d_best,
                        void *hip_stream)
{
    if (!c || !rp || !d_best) return fail(DPPS_E_INVALID, "NULL argument");
    const float w[5] = {rp->w_goal, rp->w_ball, rp->w_angle, rp->w_guard, rp->w_defense};
    for (float x : w)
        if (!isfinite(x)) return fail(DPPS_E_INVALID, "running points: weights must be finite");
    if (!finite_pos(rp->ball_norm) || !finite_pos(rp->guard_norm) || !finite_pos(rp->mark_radius) ||
        !finite_pos(rp->ang_fall) || !(rp->ang_lo >= 0.0f) || !(rp->ang_hi >= rp->ang_lo) ||
        !isfinite(rp->ang_hi) || !(rp->def_depth >= 0.0f) || !(rp->def_depth <= c->p.field_len) ||
        !(rp->def_width >= 0.0f) || !(rp->def_width <= c->p.field_wid) || rp->reserved != 0)
        return fail(DPPS_E_INVALID, "running points: norms and ang_fall > 0, 0 <= ang_lo <= ang_hi, "
                                    "defense area within the field, reserved 0");
    if (n_frames < 0) return fail(DPPS_E_INVALID, "n_frames < 0");
    HIP_OK(hipSetDevice(c->device));
    hipStream_t st = hip_stream ? (hipStream_t)hip_stream : c->stream;
    if (n_frames == 0) return DPPS_OK;
    if (!frames) return fail(DPPS_E_INVALID, "NULL input array");
    // one (unused) variant per frame; the zones are the frames' windows
    std::vector<dpps_frame> fr(frames, frames + n_frames);
    const dpps_variant one = {DPPS_FLAT, 1.0f};
    for (dpps_frame &F : fr) {
        F.n_variants = 1;
        F.variant_off = 0;
    }
    dpps_batch *b = &c->runs;
    int rc = build_tables(&c->p, n_frames, fr.data(), robots, zones, &one, 256, b->T);
    if (rc) return rc;
    b->n_frames = n_frames;
    b->tile_points = 256;
    rc = stage_tables(c, b, st);
    if (rc) return rc;
    RunArgs a;
    memset(&a, 0, sizeof a);
    a.P = c->P;
    a.R = *rp;
    a.frames = b->d_frames;
    a.robots = b->d_robots;
    a.variants = b->d_variants;
    a.wins = b->d_wins;
    a.n_wins = (int32_t)b->T.wins.size();
    a.score = d_score;
    a.best = d_best;
    if (launch_run(a, (void *)st)) return fail(DPPS_E_DEVICE, "running-point launch failed");
    return DPPS_OK;
}

int dpps_search(dpps_ctx *c, const dpps_frame *frame, const dpps_robot *robots,
                const dpps_window *windows, const dpps_variant *variants,
                const dpps_outputs *out, dpps_best *h_best)
{
    if (!c || !frame || !out || !h_best) return fail(DPPS_E_INVALID, "NULL argument");
    dpps_outputs o = *out;
    o.best = nullptr;
    HIP_OK(hipSetDevice(c->device));
    int rc = stage_batch(c, &c->scratch, 1, frame, robots, windows, variants, c->stream);
    if (rc) return rc;
    // no timing events around the kernel of a single synchronous search
    rc = run_batch(c, &c->scratch, &o, c->stream, false);
    if (rc) return rc;
    // a direct copy and a stream synchronisation: over 2 x 3000 frames this
    // gave a shorter tail (p99 0.245 vs 0.305 ms for the full frame) than the
    // pinned read-back that the surrogate path uses (which there gives the
    // lower median)
    HIP_OK(hipMemcpyAsync(h_best, c->scratch.d_best, sizeof(dpps_best), hipMemcpyDeviceToHost,
                          c->stream));
    HIP_OK(hipStreamSynchronize(c->stream));
    return DPPS_OK;
}

int dpps_batch_create(dpps_ctx *c, int32_t n_frames, const dpps_frame *frames,
                      const dpps_robot *robots, const dpps_window *windows,
                      const dpps_variant *variants, dpps_batch **outb)
{
    if (!c || !outb) return fail(DPPS_E_INVALID, "NULL argument");
    *outb = nullptr;
    HIP_OK(hipSetDevice(c->device));
    dpps_batch *b = new (std::nothrow) dpps_batch();
    if (!b) return fail(DPPS_E_NOMEM, "batch allocation failed");
    b->ctx = c;
    int rc = build_tables(&c->p, n_frames, frames, robots, windows, variants, c->tile_points, b->T);
    if (rc) {
        delete b;
        return rc;
    }
    b->n_frames = n_frames;
    b->tile_points = c->tile_points;
    rc = batch_upload(c, b);
    if (rc) {
        dpps_batch_destroy(b);
        return rc;
    }
    *outb = b;
    return DPPS_OK;
}

// ----------------------------------------------------------------------------
// autotuner: launch shapes timed on the caller's batch, cached per class
// ----------------------------------------------------------------------------

#ifndef DPPS_KERNEL_REV
#define DPPS_KERNEL_REV "unknown"
#endif

// Cache key of a launch shape: architecture, kernel sources, K, largest
// variant and interceptor counts, log2 points per frame and frames, output
// mode.
static std::string tune_key(const dpps_ctx *c, const dpps_batch *b)
{
    hipDeviceProp_t prop;
    std::string arch = "unknown";
    if (hipGetDeviceProperties(&prop, c->device) == hipSuccess) arch = prop.gcnArchName;
    size_t sp = arch.find(':');
    if (sp != std::string::npos) arch = arch.substr(0, sp);
    int vmax = 0, rmax = 0;
    for (const FrameDev &F : b->T.frames) {
        if (F.n_variants > vmax) vmax = F.n_variants;
        if (F.n_team - 1 + F.n_opp > rmax) rmax = F.n_team - 1 + F.n_opp;
    }
    int64_t pts = b->T.points;
    int nf = b->n_frames > 0 ? b->n_frames : 1;
    int lp = 0, lf = 0;
    for (int64_t x = pts / nf; x > 1; x >>= 1) ++lp;
    for (int x = nf; x > 1; x >>= 1) ++lf;
    char buf[160];
    // t2: the candidate set with explicit persistent grids
    snprintf(buf, sizeof buf, "%s|rev%s|t2|K%d|V%d|R%d|P2^%d|F2^%d|%s", arch.c_str(), DPPS_KERNEL_REV,
             c->p.n_samples, vmax, rmax, lp, lf,
             (c->p.out_flags & DPPS_OUT_REDUCED) ? "reduced" : "full");
    return buf;
}

static bool tune_lookup(const char *path, const std::string &key, int *tp, int *wv, int *pc)
{
    FILE *fp = path ? fopen(path, "r") : nullptr;
    if (!fp) return false;
    char line[512];
    bool found = false;
    std::string want = "{\"key\": \"" + key + "\",";
    while (fgets(line, sizeof line, fp)) {
        if (strncmp(line, want.c_str(), want.size()) != 0) continue;
        int a, w, p;
        const char *q = strstr(line, "\"tile_points\":");
        if (q && sscanf(q, "\"tile_points\": %d, \"waves\": %d, \"wg_per_cu\": %d", &a, &w, &p) == 3) {
            *tp = a;
            *wv = w;
            *pc = p;
            found = true;  // the last entry for a key wins
        }
    }
    fclose(fp);
    return found;
}

int dpps_autotune(dpps_ctx *c, dpps_batch *b, const dpps_outputs *out, void *hip_stream,
                  const char *cache_path, int32_t reps, float *best_ms)
{
    if (!c || !b || !out) return fail(DPPS_E_INVALID, "NULL argument");
    if (reps < 1 || reps > 100) return fail(DPPS_E_INVALID, "reps must be in [1, 100]");
    HIP_OK(hipSetDevice(c->device));
    hipStream_t st = hip_stream ? (hipStream_t)hip_stream : c->stream;
    const std::string key = tune_key(c, b);
    int tp = 0, wv = 0, pc = 0;
    if (tune_lookup(cache_path, key, &tp, &wv, &pc)) {
        int rc = dpps_set_launch(c, tp, wv, pc);
        if (rc) return rc;
        if (b->tile_points != c->tile_points) {
            b->tile_points = c->tile_points;
            rc = batch_upload(c, b);
            if (rc) return rc;
        }
        if (best_ms) *best_ms = -1.0f;
        return DPPS_OK;
    }
    const int tps[] = {8, 16, 32, 64};
    const int wvs[] = {1, 2, 4, 8};
    // persistent with the occupancy grid, one workgroup per tile, and
    // persistent grids of 2 and 4 workgroups per CU (a grid larger than what
    // fits waits for free slots, which can balance better)
    const int pcs[] = {-2, -1, 2, 4};
    float best = 1e30f;
    int btp = c->tile_points, bwv = c->waves, bpc = c->persistent ? (c->wg_per_cu ? c->wg_per_cu : -2) : -1;
    for (int t : tps) {
        c->tile_points = t;
        b->tile_points = t;
        int rc = batch_upload(c, b);
        if (rc) return rc;
        for (int w : wvs) {
            for (int pch : pcs) {
                rc = dpps_set_launch(c, t, w, pch);
                if (rc) return rc;
                rc = run_batch(c, b, out, st, true);  // warm-up
                if (rc) return rc;
                float tot = 0.0f;
                for (int r = 0; r < reps; ++r) {
                    rc = run_batch(c, b, out, st, true);
                    if (rc) return rc;
                    float ms = dpps_last_kernel_ms(c);
                    if (ms < 0.0f) return fail(DPPS_E_DEVICE, "kernel timing failed");
                    tot += ms;
                }
                float avg = tot / (float)reps;
                if (avg < best) {
                    best = avg;
                    btp = t;
                    bwv = w;
                    bpc = pch;
                }
            }
        }
    }
    int rc = dpps_set_launch(c, btp, bwv, bpc);
    if (rc) return rc;
    b->tile_points = btp;
    rc = batch_upload(c, b);
    if (rc) return rc;
    if (best_ms) *best_ms = best;
    if (cache_path) {
        FILE *fp = fopen(cache_path, "a");
        if (!fp) return fail(DPPS_E_INVALID, "cannot write %s", cache_path);
        fprintf(fp, "{\"key\": \"%s\", \"tile_points\": %d, \"waves\": %d, \"wg_per_cu\": %d, "
                    "\"kernel_ms\": %.5f}\n", key.c_str(), btp, bwv, bpc, (double)best);
        fclose(fp);
    }
    return DPPS_OK;
}

int dpps_batch_set_robots(dpps_ctx *c, dpps_batch *b, const dpps_robot *robots, void *hip_stream)
{
    if (!c || !b || !robots) return fail(DPPS_E_INVALID, "NULL argument");
    // robots are given in the batch's own packed order (frame by frame)
    size_t n = b->T.robots.size();
    for (size_t i = 0; i < n; ++i)
        if (!isfinite(robots[i].x) || !isfinite(robots[i].y) || !isfinite(robots[i].vx) ||
            !isfinite(robots[i].vy))
            return fail(DPPS_E_INVALID, "robot %zu not finite", i);
    memcpy(b->T.robots.data(), robots, n * sizeof(dpps_robot));
    hipStream_t st = hip_stream ? (hipStream_t)hip_stream : c->stream;
    HIP_OK(hipMemcpyAsync(b->d_robots, b->T.robots.data(), n * sizeof(dpps_robot),
                          hipMemcpyHostToDevice, st));
    HIP_OK(hipStreamSynchronize(st));
    return DPPS_OK;
}

int dpps_batch_run(dpps_ctx *c, dpps_batch *b, const dpps_outputs *out, void *hip_stream,
                   int use_graph)
{
    if (!c || !b || !out) return fail(DPPS_E_INVALID, "NULL argument");
    HIP_OK(hipSetDevice(c->device));
    hipStream_t st = hip_stream ? (hipStream_t)hip_stream : c->stream;
    if (b->tile_points != c->tile_points) {
        // the context's tile size changed since the batch was built
        HIP_OK(hipStreamSynchronize(st));
        b->tile_points = c->tile_points;
        int rc = batch_upload(c, b);
        if (rc) return rc;
    }
    if (!use_graph) return run_batch(c, b, out, st, true);
    int cfg[3] = {c->tile_points, c->waves, c->persistent ? c->wg_per_cu : -1};
    bool same = b->exec && memcmp(&b->graph_out, out, sizeof *out) == 0 &&
                b->graph_stream == (void *)st && memcmp(cfg, b->graph_cfg, sizeof cfg) == 0;
    if (!same) {
        graph_drop(b);
        HIP_OK(hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal));
        int rc = run_batch(c, b, out, st, false);
        hipGraph_t g = nullptr;
        hipError_t e = hipStreamEndCapture(st, &g);
        if (rc) {
            if (g) (void)hipGraphDestroy(g);
            return rc;
        }
        if (e != hipSuccess) return fail(DPPS_E_DEVICE, "graph capture failed: %s", hipGetErrorString(e));
        b->graph = g;
        HIP_OK(hipGraphInstantiate(&b->exec, g, nullptr, nullptr, 0));
        b->graph_out = *out;
        b->graph_stream = (void *)st;
        memcpy(b->graph_cfg, cfg, sizeof cfg);
    }
    HIP_OK(hipGraphLaunch(b->exec, st));
    c->timed = false;
    return DPPS_OK;
}

void dpps_batch_destroy(dpps_batch *b)
{
    if (!b) return;
    if (b->ctx && b->ctx->stream) (void)hipStreamSynchronize(b->ctx->stream);
    batch_free_device(b);
    delete b;
}

int64_t dpps_batch_tiles(const dpps_batch *b) { return b ? (int64_t)b->T.tiles.size() : -1; }
int64_t dpps_batch_points(const dpps_batch *b) { return b ? b->T.points : -1; }

int dpps_timing_begin(dpps_ctx *c, int32_t max_runs)
{
    if (!c || max_runs < 1 || max_runs > 1 << 20) return fail(DPPS_E_INVALID, "bad timing request");
    HIP_OK(hipSetDevice(c->device));
    ring_free(c);
    c->ring0.resize(max_runs, nullptr);
    c->ring1.resize(max_runs, nullptr);
    for (int i = 0; i < max_runs; ++i) {
        if (hipEventCreate(&c->ring0[i]) != hipSuccess || hipEventCreate(&c->ring1[i]) != hipSuccess) {
            ring_free(c);
            return fail(DPPS_E_DEVICE, "hipEventCreate failed");
        }
    }
    return DPPS_OK;
}

int dpps_timing_end(dpps_ctx *c, float *total_ms, int32_t *n_runs)
{
    if (!c || !total_ms || !n_runs) return fail(DPPS_E_INVALID, "NULL argument");
    double tot = 0.0;
    int n = c->ring_used;
    for (int i = 0; i < n; ++i) {
        float ms = 0.0f;
        HIP_OK(hipEventSynchronize(c->ring1[i]));
        HIP_OK(hipEventElapsedTime(&ms, c->ring0[i], c->ring1[i]));
        tot += ms;
    }
    *total_ms = (float)tot;
    *n_runs = n;
    ring_free(c);
    return DPPS_OK;
}

float dpps_last_kernel_ms(dpps_ctx *c)
{
    if (!c || !c->timed) return -1.0f;
    if (hipEventSynchronize(c->ev1) != hipSuccess) return -1.0f;
    float ms = -1.0f;
    if (hipEventElapsedTime(&ms, c->ev0, c->ev1) != hipSuccess) return -1.0f;
    return ms;
}

}  // extern "C"
