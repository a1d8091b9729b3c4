// runtime.h -- host-side internals of libdpps shared by its C ABI sources.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <string>
#include <vector>

#include "dpps_internal.h"

namespace dpps {

// Record a message for dpps_last_error() and return code.
int fail(int code, const char *fmt, ...) __attribute__((format(printf, 2, 3)));
int check_params(const dpps_params *p);
DevParams derive(const dpps_params *p);
int lattice_dim(float len, float h, int32_t *n);

// Host-side description of a batch: the device tables before upload.
struct HostTables {
    std::vector<FrameDev> frames;
    std::vector<dpps_robot> robots;
    std::vector<dpps_variant> variants;
    std::vector<WinDev> wins;
    std::vector<TileDev> tiles;
    int64_t points = 0;
};

// Validate host frames and build their device tables; tile_points 0 builds
// no tiles (windows validated only).
int build_tables(const dpps_params *p, int32_t n_frames, const dpps_frame *frames,
                 const dpps_robot *robots, const dpps_window *windows,
                 const dpps_variant *variants, int tile_points, HostTables &T);

}  // namespace dpps

#define HIP_OK(expr)                                                                          \
    do {                                                                                      \
        hipError_t e_ = (expr);                                                               \
        if (e_ != hipSuccess)                                                                 \
            return fail(DPPS_E_DEVICE, "%s failed: %s", #expr, hipGetErrorString(e_));        \
    } while (0)

using dpps::fail;

struct DeviceArena {
    void *ptr = nullptr;
    size_t cap = 0;
};

struct dpps_batch {
    dpps_ctx *ctx = nullptr;
    dpps::HostTables T;
    int32_t n_frames = 0;
    int tile_points = 0;
    DeviceArena arena;       // frames, robots, variants, wins, tiles
    dpps::FrameDev *d_frames = nullptr;
    dpps_robot *d_robots = nullptr;
    dpps_variant *d_variants = nullptr;
    dpps::WinDev *d_wins = nullptr;
    dpps::TileDev *d_tiles = nullptr;
    DeviceArena aux;         // work counter, tile records, best
    uint32_t *d_counter = nullptr;
    dpps::TileRec *d_tile_rec = nullptr;
    dpps_best *d_best = nullptr;
    // graph cache
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    dpps_outputs graph_out;
    void *graph_stream = nullptr;
    int graph_cfg[3] = {0, 0, 0};
};

struct dpps_ctx {
    dpps_params p;
    dpps::DevParams P;
    int device = 0;
    hipStream_t stream = nullptr;
    bool own_stream = false;
    int n_cu = 256;
    int tile_points = 8;
    int waves = 4;
    int wg_per_cu = 0;       // 0: as many as fit (occupancy of the search kernel)
    int persistent = 1;
    dpps_batch scratch;      // used by dpps_search / dpps_search_batch / host-frame surrogate
    dpps_batch fallback;     // exact searches of surrogate frames without a feasible proposal
    dpps_batch rays;         // tables of dpps_ray_search
    DeviceArena ray_aux;     // its work counter and per-tile records
    DeviceArena ray_dirs;    // unit vectors of the kick directions (4096 at most)
    int ray_dirs_n = 0;      // the direction count they were computed for
    int ray_tile_dirs = 32;  // directions per tile of dpps_ray_search
    int ray_waves = 4;       // waves per workgroup of dpps_ray_search (4: 0.260 ms per
                             // 512-frame call, 8: 0.272 ms)
    dpps_batch shots;        // tables of dpps_shot_decision
    int shot_tile = 16;      // window points per workgroup of the shot map
    int shot_waves = 4;      // waves per workgroup of the shot map
    dpps_batch runs;         // tables of dpps_running_points
    void *pinned = nullptr;
    size_t pinned_cap = 0;
    hipEvent_t staged = nullptr;   // pinned staging consumed
    dpps_best *pinned_best = nullptr;  // pinned landing buffer of best records read back
    int64_t pinned_best_cap = 0;
    hipEvent_t landed = nullptr;   // best records in pinned_best
    hipEvent_t ev0 = nullptr, ev1 = nullptr;
    bool timed = false;
    uint64_t budget_used = 0;
    // optional ring of event pairs bracketing the search kernel of each run
    std::vector<hipEvent_t> ring0, ring1;
    int ring_used = 0;
    // dpps_search_batch_noalloc: the device's fixed array (its address on
    // this context's device), host tables reserved for its largest request,
    // and a pinned staging buffer of its size, all set up by dpps_create
    unsigned char *na_scratch = nullptr;
    dpps_batch na;
    void *na_pinned = nullptr;
    hipEvent_t na_staged = nullptr;  // na_pinned consumed by the last copy
};

// Sizes of the table section of the arena.
struct Layout {
    size_t off_frames, off_robots, off_variants, off_wins, off_tiles, total;
};

size_t align_up(size_t x, size_t a);
int arena_reserve(dpps_ctx *c, DeviceArena &A, size_t bytes);
void graph_drop(dpps_batch *b);
Layout table_layout(const dpps::HostTables &T);
void pack_tables(const dpps::HostTables &T, const Layout &L, char *dst);
int batch_reserve(dpps_ctx *c, dpps_batch *b, const Layout &L);
int batch_upload(dpps_ctx *c, dpps_batch *b);
int run_batch(dpps_ctx *c, dpps_batch *b, const dpps_outputs *out, hipStream_t st, bool timed,
              const dpps_power_params *power = nullptr, float *v0_out = nullptr);
int stage_batch(dpps_ctx *c, dpps_batch *b, int32_t n_frames, const dpps_frame *frames,
                const dpps_robot *robots, const dpps_window *windows,
                const dpps_variant *variants, hipStream_t st);
int stage_tables(dpps_ctx *c, dpps_batch *b, hipStream_t st);
// Set up the fixed-array search on the context's (current) device.
int noalloc_setup(dpps_ctx *c);
void noalloc_release(dpps_ctx *c);
// Copy n best records from device memory to h (host) after the work queued
// on st, through the context's pinned buffer (no staging of pageable memory),
// waiting on an event recorded after the copy.
int read_best(dpps_ctx *c, dpps_best *h, const dpps_best *d, int n, hipStream_t st);
