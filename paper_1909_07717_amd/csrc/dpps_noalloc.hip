// dpps_noalloc.hip -- dpps_search_batch for callers that cannot allocate.
//
// The batched search keeps its per-request device state (the frames' tables,
// the tile list, one best record per tile and the persistent work counter)
// in memory the context grows on demand.  This entry point puts that state
// in one fixed device array per GPU instead, and stages the tables through
// host storage reserved when the context is created, so that a call makes
// no device, pinned or host allocation.  The kernels are the batched
// search's own: they receive the array's device address exactly as they
// receive the context's buffers.
#include <hip/hip_runtime.h>
#include <string.h>

#include <mutex>

#include "runtime.h"

using namespace dpps;

namespace {

constexpr size_t SCRATCH_BYTES = (size_t)DPPS_NOALLOC_SCRATCH_BYTES;
constexpr size_t COUNTER_BYTES = 256;
constexpr int MAX_DEVICES = 64;

// The fixed array: every GPU that loads the library holds its own copy
// until the process ends.  Host code must never pass this name to a kernel
// or a copy (on the host it is only a stand-in); it uses the device address
// that hipGetSymbolAddress returns for the current device.
static __device__ __align__(256) unsigned char scratch[SCRATCH_BYTES];

std::mutex g_mu;
unsigned char *g_addr[MAX_DEVICES] = {};

// Device address of `scratch` on `device` (which must be current), looked up
// once per device.
int scratch_address(int device, unsigned char **out)
{
    if (device < 0 || device >= MAX_DEVICES)
        return fail(DPPS_E_UNSUPPORTED, "device %d: the fixed search array supports devices 0-%d",
                    device, MAX_DEVICES - 1);
    std::lock_guard<std::mutex> lk(g_mu);
    if (!g_addr[device]) {
        void *p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p)
            return fail(DPPS_E_DEVICE, "hipGetSymbolAddress of the fixed search array: %s",
                        hipGetErrorString(e));
        g_addr[device] = (unsigned char *)p;
    }
    *out = g_addr[device];
    return DPPS_OK;
}

size_t tables_bytes(int64_t nf, int64_t nr, int64_t nv, int64_t nw, int64_t nt)
{
    size_t o = 0;
    o = align_up(o + (size_t)nf * sizeof(FrameDev), 256);
    o = align_up(o + (size_t)nr * sizeof(dpps_robot), 256);
    o = align_up(o + (size_t)nv * sizeof(dpps_variant), 256);
    o = align_up(o + (size_t)nw * sizeof(WinDev), 256);
    o = align_up(o + (size_t)nt * sizeof(TileDev), 256);
    return o < 256 ? 256 : o;
}

size_t records_bytes(int64_t nt) { return align_up((size_t)(nt > 0 ? nt : 1) * sizeof(TileRec), 256); }

}  // namespace

int noalloc_setup(dpps_ctx *c)
{
    int rc = scratch_address(c->device, &c->na_scratch);
    if (rc) return rc;
    c->na.ctx = c;
    // host tables that no request fitting the array can outgrow: each table
    // alone is at most the array's size
    HostTables &T = c->na.T;
    T.frames.reserve(SCRATCH_BYTES / sizeof(FrameDev));
    T.robots.reserve(SCRATCH_BYTES / sizeof(dpps_robot));
    T.variants.reserve(SCRATCH_BYTES / sizeof(dpps_variant));
    T.wins.reserve(SCRATCH_BYTES / sizeof(WinDev));
    T.tiles.reserve(SCRATCH_BYTES / sizeof(TileDev));
    if (hipHostMalloc(&c->na_pinned, SCRATCH_BYTES, hipHostMallocDefault) != hipSuccess) {
        c->na_pinned = nullptr;
        return fail(DPPS_E_NOMEM, "hipHostMalloc(%zu) for the fixed search array's staging",
                    SCRATCH_BYTES);
    }
    HIP_OK(hipEventCreateWithFlags(&c->na_staged, hipEventDisableTiming));
    return DPPS_OK;
}

void noalloc_release(dpps_ctx *c)
{
    if (c->na_pinned) (void)hipHostFree(c->na_pinned);
    if (c->na_staged) (void)hipEventDestroy(c->na_staged);
    c->na_pinned = nullptr;
    c->na_staged = nullptr;
}

extern "C" {

int dpps_search_batch_noalloc(dpps_ctx *c, int32_t n_frames, const dpps_frame *frames,
                              const dpps_robot *robots, const dpps_window *windows,
                              const dpps_variant *variants, const dpps_outputs *out,
                              void *hip_stream)
{
    if (!c) return fail(DPPS_E_INVALID, "ctx is NULL");
    if (!out || !out->best) return fail(DPPS_E_INVALID, "outputs or outputs->best is NULL");
    if (!c->na_scratch || !c->na_pinned || !c->na_staged)
        return fail(DPPS_E_DEVICE, "the fixed search array was not set up");
    if (n_frames < 0) return fail(DPPS_E_INVALID, "n_frames < 0");
    if (n_frames > 0 && (!frames || !robots || !windows || !variants))
        return fail(DPPS_E_INVALID, "NULL input array");
    // sizes first, from the counts alone, so that the tables are built only
    // for a request that fits (they then never outgrow their reserved storage)
    const int tp = c->tile_points;
    int64_t nr = 0, nv = 0, nw = 0, nt = 0;
    for (int32_t f = 0; f < n_frames; ++f) {
        const dpps_frame &F = frames[f];
        if (F.n_team < 1 || F.n_team > DPPS_MAX_SIDE || F.n_opp < 0 || F.n_opp > DPPS_MAX_SIDE ||
            F.n_variants < 1 || F.n_variants > DPPS_MAX_VARIANTS || F.n_windows < 0 ||
            F.robot_off < 0 || F.window_off < 0 || F.variant_off < 0)
            return fail(DPPS_E_INVALID, "frame %d: counts or offsets out of range", f);
        nr += F.n_team + F.n_opp;
        nv += F.n_variants;
        nw += F.n_windows;
        for (int w = 0; w < F.n_windows; ++w) {
            const dpps_window &Wn = windows[F.window_off + w];
            if (Wn.nx < 0 || Wn.ny < 0)
                return fail(DPPS_E_INVALID, "frame %d window %d: negative size", f, w);
            nt += ((int64_t)Wn.nx * Wn.ny + tp - 1) / tp;
            if (nt > (int64_t)(SCRATCH_BYTES / sizeof(TileRec)))
                return fail(DPPS_E_BUDGET, "request needs more than the fixed %zu-byte search "
                            "array (frame %d: over %lld tiles)", SCRATCH_BYTES, f, (long long)nt);
        }
        const size_t need = COUNTER_BYTES + tables_bytes(f + 1, nr, nv, nw, nt) + records_bytes(nt);
        if (need > SCRATCH_BYTES)
            return fail(DPPS_E_BUDGET, "request needs more than the fixed %zu-byte search array "
                        "(%d frames, %lld tiles so far)", SCRATCH_BYTES, f + 1, (long long)nt);
    }
    HIP_OK(hipSetDevice(c->device));
    hipStream_t st = hip_stream ? (hipStream_t)hip_stream : c->stream;
    dpps_batch *b = &c->na;
    // the previous call's copy must have left the staging buffer before the
    // tables (which it was packed from) are rebuilt
    HIP_OK(hipEventSynchronize(c->na_staged));
    int rc = build_tables(&c->p, n_frames, frames, robots, windows, variants, tp, b->T);
    if (rc) return rc;
    const Layout L = table_layout(b->T);
    const size_t off_rec = COUNTER_BYTES + L.total;
    if (off_rec + records_bytes((int64_t)b->T.tiles.size()) > SCRATCH_BYTES)
        return fail(DPPS_E_BUDGET, "request exceeds the fixed %zu-byte search array", SCRATCH_BYTES);
    b->n_frames = n_frames;
    b->tile_points = tp;
    unsigned char *base = c->na_scratch + COUNTER_BYTES;
    b->d_frames = (FrameDev *)(base + L.off_frames);
    b->d_robots = (dpps_robot *)(base + L.off_robots);
    b->d_variants = (dpps_variant *)(base + L.off_variants);
    b->d_wins = (WinDev *)(base + L.off_wins);
    b->d_tiles = (TileDev *)(base + L.off_tiles);
    b->d_counter = (uint32_t *)c->na_scratch;
    b->d_tile_rec = (TileRec *)(c->na_scratch + off_rec);
    b->d_best = nullptr;
    pack_tables(b->T, L, (char *)c->na_pinned);
    HIP_OK(hipMemcpyAsync(base, c->na_pinned, L.total, hipMemcpyHostToDevice, st));
    HIP_OK(hipEventRecord(c->na_staged, st));
    // the array keeps the last call's contents: the 8 work counters start at 0
    if (launch_zero_words(b->d_counter, 8, (void *)st))
        return fail(DPPS_E_DEVICE, "clearing the work counter failed: %s",
                    hipGetErrorString(hipGetLastError()));
    return run_batch(c, b, out, st, false);
}

}  // extern "C"
