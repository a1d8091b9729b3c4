// dpps_internal.h -- structures shared by the host runtime and the HIP kernels
// of libdpps (not part of the public ABI).
#pragma once

#include <stdint.h>

#include "../../include/dpps.h"

namespace dpps {

// Constants derived once per context from dpps_params: reciprocals, the
// robot model in time units scaled by the acceleration limit, and the
// coefficients that invert the ball model for the critical kick speed.
// The ball model's parameters in float64 (the per-variant ball constants
// are derived from them): decelerations while sliding and rolling, the speed
// ratio at the end of sliding, the chip angle's cosine and sine, gravity.
struct BallParams64 {
    double a_s, a_r, ratio, cos_th, sin_th, g;
};

struct DevParams {
    // geometry
    float field_len, field_wid;
    float goal_x, half_goal_w, goal_eps;
    float R, RA;       // robot radius, and scaled by amax
    float V, A, invV;
    float Vh;          // vmax / sqrt(2): speed limit in the kernel's velocity units
    float V2, inv2V, halfV;  // vmax^2, 1 / (2 vmax), vmax / 2
    float invA2;       // 2 / amax: robot stage units (A T / 2) to seconds
    // ball model
    float a_s, a_r, ratio, cos_th, lam1_inv;  // lam1 = sin(2 th) / g  (carry = lam1 v0^2)
    // flat inversion: stopped / rolling / sliding regimes (icD = 1 / cD,
    // icA = 1 / cA, icB = 1 / cB; alpha, hbeta = beta / 2, hbeta2 = hbeta^2:
    // the slow root's terms with numerator and denominator halved)
    float f_icD, f_icA, f_icB, f_alpha, f_hbeta, f_hbeta2, f_hfast, f_pfast;
    // chip inversion: stopped / rolling / in-flight regimes (same layout)
    float c_icD, c_icA, c_icB, c_alpha, c_hbeta, c_hbeta2, c_hfast, c_pfast;
    float half_ar;
    // scoring
    float margin_cap, w_ang_pi, w_dist, inv_dist_norm, w_margin;
    int32_t K;
    int32_t out_flags;
    // float64 copies used by the per-variant finish
    BallParams64 bp;
    double margin_d;
    double invK_d;
};

// One (frame, window) pair of a batch.
struct WinDev {
    float h;
    int32_t i0, j0, nx, ny;
    float halfNx, halfNy;   // (Nx - 1) / 2, (Ny - 1) / 2 of the full lattice
    int32_t frame;
    int32_t npts;           // nx * ny
    int32_t elem_base;      // frame-relative index of this window's first element
    int64_t out_base;       // absolute output element of this window's first (reduced) element
};

// A tile of the passing-point search: p0 / tile_points = k, and the tile
// holds chunks k, k + T, k + 2T, ... of 4 consecutive points (up to
// tile_points points) of a window cut into T tiles.  A tile of the shot map: points p0 .. p0 + tile_points -
// 1; of the direction sweep: directions p0 .. p0 + tile_dirs - 1.
struct TileDev {
    int32_t win;
    int32_t p0;
};

// Best pass found by one tile: packed key (score bits << 32 | ~element), and
// the interception times of that pass.
struct TileRec {
    unsigned long long key;
    float t_team, t_opp;
    float v0, pad;          // kick speed of that pass (the per-point power search)
};

// Device-side copy of a frame (the public struct plus derived indices).
struct FrameDev {
    int32_t n_team, n_opp, passer, robot_off;
    int32_t n_windows, win_off, n_variants, variant_off;
    float ball_x, ball_y;
    int32_t tile_begin, tile_count;
    int64_t ray_base;       // direction x variant search: first output element
};

// Fallback tables built on the device: frames whose best pass is not
// feasible, or scores below `below`, get one window over the whole lattice
// (nx x ny points at spacing h) in frames / wins; map[slot] is the frame,
// *count the number of such frames.
struct FallbackArgs {
    const FrameDev *src;
    const dpps_best *best;
    int32_t n;
    float below;
    int32_t nx, ny;
    float h;
    int32_t tiles_per_frame;
    FrameDev *frames;
    WinDev *wins;
    int32_t *map;
    int32_t *count;
};

struct LaunchArgs {
    DevParams P;
    const FrameDev *frames;
    const dpps_robot *robots;
    const dpps_variant *variants;
    const WinDev *wins;
    const TileDev *tiles;
    int32_t n_tiles;
    int32_t n_frames;
    int32_t tile_points;
    int32_t persistent;
    uint32_t *counter;      // 8 persistent work counters (one per class of workgroup
                            // index mod 8); the finalize kernel resets them
    TileRec *tile_rec;      // one per tile
    // per-point passing power (Eq. 1-2) instead of the frames' variants
    int32_t power;
    float p_buffer, p_vmin, p_vmax;
    float *v0_out;          // power per point (may be NULL)
    uint8_t *mask;
    float *score;
    float *t_team;
    float *t_opp;
    dpps_best *best;
    // Tables built on the device (the exact fallback of the surrogate search):
    // with tiles_per_frame > 0 the tiles are implicit (tile t is tile
    // t % tiles_per_frame of window t / tiles_per_frame),
    // and with n_frames_dev the number of frames is read on the device
    // (n_frames and n_tiles are then upper bounds); with best_map, frame f's
    // best record goes to best[best_map[f]].
    int32_t tiles_per_frame;
    const int32_t *n_frames_dev;
    const int32_t *best_map;
    // > 0 (one frame, persistent grid of wg_records workgroups): each
    // workgroup keeps its best over all its tiles and writes that one record
    // to tile_rec[blockIdx.x]; the finalize kernel reduces those records
    int32_t wg_records;
    // with fb_on, the finalize kernel also appends each frame whose best pass
    // needs the exact fallback to the fallback tables (slot by atomic count;
    // fb.count must be 0 before the launch; fb.src is not used: the frame's
    // own entry of `frames` is copied)
    int32_t fb_on;
    FallbackArgs fb;
};

// Best pass of one tile of the direction x variant search.
struct RayRec {
    unsigned long long key;  // ordered score bits << 32 | ~(d * n_variants + v)
    float t_team, t_opp, s_recv, open_angle, refract, pad;
};

struct RayArgs {
    DevParams P;
    const FrameDev *frames;
    const dpps_robot *robots;
    const dpps_variant *variants;
    const TileDev *tiles;   // win = frame, p0 = first direction of the tile
    const double2 *dirs;    // (cos, sin) of each kick direction (launch_ray_dirs)
    int32_t n_tiles;
    int32_t n_frames;
    int32_t tile_dirs;
    int32_t n_dirs;
    float w_time, w_refract;
    uint32_t *counter;      // persistent work counter; the finalize kernel resets it
    RayRec *tile_rec;
    uint8_t *mask;
    float *score;
    float *t_team;
    float *t_opp;
    float *s_recv;
    dpps_ray_best *best;
};

// Shooting decision (from each frame's ball, and from window points).
struct ShotArgs {
    DevParams P;
    const FrameDev *frames;
    const dpps_robot *robots;
    const dpps_variant *variants;
    const WinDev *wins;
    const TileDev *tiles;
    int32_t n_tiles;
    int32_t n_frames;
    int32_t tile_points;
    float v_shot, min_angle, margin;
    dpps_shot *ball;        // one record per frame
    dpps_shot *map;         // one record per window point (may be NULL)
};

// Running points: one workgroup per zone (window).
struct RunArgs {
    DevParams P;
    dpps_run_params R;
    const FrameDev *frames;
    const dpps_robot *robots;
    const dpps_variant *variants;
    const WinDev *wins;
    int32_t n_wins;
    float *score;           // per point (may be NULL)
    dpps_run_best *best;    // per zone
};

// host-side launchers (dpps_kernels.hip)
// ev_start / ev_stop (hipEvent_t or NULL) bracket the search kernel only.
int launch_search(const LaunchArgs &a, int waves_per_wg, int grid, void *stream, void *ev_start,
                  void *ev_stop);
// Zero n 32-bit words of device memory on `stream` (a kernel, no memset).
int launch_zero_words(uint32_t *p, int n, void *stream);
// Resident workgroups per CU of the search kernel for this K and block size.
int search_occupancy(int K, int waves_per_wg, int tile_points);
// Direction x variant search (ray kernel then its finalize) on `stream`;
// ev_start / ev_stop (hipEvent_t or NULL) bracket the ray kernel only.
// (cos, sin) of theta_d = 2 pi d / n for d < n into dirs (n <= 4096).
int launch_ray_dirs(double2 *dirs, int n, void *stream);
int launch_ray(const RayArgs &a, int waves_per_wg, int grid, void *stream, void *ev_start,
               void *ev_stop);
int ray_occupancy(int K, int waves_per_wg);
// Shooting decisions: the ball kernel, then (with a.map) the window kernel.
int launch_shot(const ShotArgs &a, int waves_per_wg, void *stream);
int launch_run(const RunArgs &a, void *stream);

}  // namespace dpps
