// dpps_kernels.hip -- HIP kernels (gfx950) of the SBIP-DPPS passing-point search.
//
// Work decomposition
//   One workgroup per tile of candidate points (persistent workgroups pull
//   tiles from an atomic counter, or one workgroup per tile).  A wave
//   evaluates one candidate point at a time with its 64 lanes spread over the
//   K path samples (K/64 per lane):
//
//   1. robot stage   for every interceptor and every sample, the robot's
//                    arrival time (straight line, bounded acceleration and
//                    speed, at rest on the sample); the minimum over teammates
//                    and over opponents is kept per sample.  Sample positions
//                    depend on the point only, so this stage is shared by all
//                    pass variants (Sec. 4.2 traverses speeds for fixed paths).
//   2. critical speed per sample, the kick speed at which the ball reaches the
//                    sample exactly when the first teammate (opponent) does;
//                    a slower kick is intercepted there, a faster one is not
//                    (the ball model of Sec. 4.1 is monotone in the kick speed).
//   3. first crossing per variant (SBIP, Sec. 4.2): the lowest sample whose
//                    critical speed is at least v0; the running maximum of the
//                    critical speeds over the samples is non-decreasing, so
//                    every variant lane finds its crossing by binary search in
//                    the wave's LDS row of running maxima.
//   4. finish        lanes become variants: ball time at the crossing sample
//                    (float64), margin, feasibility and the Eq. (3) score
//                    (Sec. 4.3); results are staged in LDS and written as whole
//                    rows per tile.  Each tile records its best pass; a small
//                    finalize kernel reduces the records of each frame.
//
// The open goal angle (Sec. 4.3/4.4) is computed with lanes = opponents.
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

#include "dpps_internal.h"

namespace dpps {

#define MAX_ROB (2 * DPPS_MAX_SIDE)
#define MAX_VAR DPPS_MAX_VARIANTS
#define MAX_TILE 64
#define MAX_WAVES 8
#define MAX_K 256
#define PM_ROWS 4  // running-maximum rows per wave: flat team / opp, chip team / opp

// Dynamic LDS of the search and ray kernels: PM_ROWS rows of K floats per wave.
static size_t pm_bytes(int K, int waves) { return (size_t)waves * PM_ROWS * K * sizeof(float); }

struct VarConst {
    double va1, a1, va2, a2, soff2, toff2, split, D, sf_reach;
};

struct StageLDS {
    float4 rob[MAX_ROB];      // (x, y, vx, vy): team interceptors, then opponents
    float v0[MAX_VAR];
    int32_t type[MAX_VAR];
    int32_t vidx[MAX_VAR];    // the caller's index of each staged variant
    VarConst vc[MAX_VAR];
    int32_t n_tm, n_op, n_var, has_flat, has_chip, frame;
    int32_t vel_ok;           // every robot's speed is at most vmax
    float bx, by;
    BallParams64 bp;          // persistent kernels: written once at the start
};

// A wave's path-frame block: MAX_ROB entries, then MAX_ROB bound keys.
#define PR_ENTRIES (MAX_ROB + MAX_ROB / 4)

// Dynamic LDS of the search kernel, sized by the launch: each wave's
// running-maximum rows and its two path-frame blocks, then the tile's staged
// score and mask maps (MAX_VAR rows of tile_points).
static size_t search_lds_bytes(int K, int waves, int tile_points)
{
    const size_t maps = (size_t)MAX_VAR * tile_points * (sizeof(float) + 1);
    return pm_bytes(K, waves) + (size_t)waves * 2 * PR_ENTRIES * sizeof(float4) +
           ((maps + 15) & ~(size_t)15);
}
__device__ __forceinline__ uint32_t *bound_keys(float4 *pr) { return (uint32_t *)(pr + MAX_ROB); }
__device__ __forceinline__ const uint32_t *bound_keys(const float4 *pr)
{
    return (const uint32_t *)(pr + MAX_ROB);
}

struct OutLDS {
    TileRec wbest[MAX_WAVES];
    TileRec wgbest;           // the workgroup's best over its tiles (one-frame launches)
};

__device__ __forceinline__ float rsq(float x) { return __builtin_amdgcn_rsqf(x); }
__device__ __forceinline__ float hsqrt(float x) { return __builtin_amdgcn_sqrtf(x); }
__device__ __forceinline__ float hrcp(float x) { return __builtin_amdgcn_rcpf(x); }
__device__ __forceinline__ float med3(float x, float lo, float hi)
{
    return __builtin_amdgcn_fmed3f(x, lo, hi);
}
__device__ __forceinline__ int lane_id() { return __lane_id(); }
__device__ __forceinline__ int uni(int x) { return __builtin_amdgcn_readfirstlane(x); }
__device__ __forceinline__ float unif(float x)
{
    return __int_as_float(__builtin_amdgcn_readfirstlane(__float_as_int(x)));
}
__device__ __forceinline__ float readlane_f(float x, int l)
{
    return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(x), l));
}
__device__ __forceinline__ int readlane_i(int x, int l) { return __builtin_amdgcn_readlane(x, l); }

// Ball constants of one variant (float64): phase split, speeds and
// decelerations, offsets, stopping distance D and the minimum reachable
// distance (the carry of a chip).
__device__ VarConst var_const(const BallParams64 &B, int type, float v0f)
{
    VarConst c;
    double v0 = (double)v0f;
    if (type == DPPS_CHIP) {
        double vh = v0 * B.cos_th, vz = v0 * B.sin_th;
        double tf = 2.0 * vz / B.g;
        double sf = vh * tf;
        c.va1 = vh; c.a1 = B.a_r;             // unused: split < 0
        c.va2 = vh; c.a2 = B.a_r; c.soff2 = sf; c.toff2 = tf;
        c.split = -1.0;
        c.D = sf + vh * vh / (2.0 * B.a_r);
        c.sf_reach = sf;
    } else {
        double v1 = B.ratio * v0;
        double t1 = (v0 - v1) / B.a_s;
        double d1 = (v0 * v0 - v1 * v1) / (2.0 * B.a_s);
        c.va1 = v0; c.a1 = B.a_s;
        c.va2 = v1; c.a2 = B.a_r; c.soff2 = d1; c.toff2 = t1;
        c.split = d1;
        c.D = d1 + v1 * v1 / (2.0 * B.a_r);
        c.sf_reach = 0.0;
    }
    return c;
}

// Stage the frame into LDS: interceptors (passer dropped), scaled by amax so
// that the robot model runs in units where the acceleration limit is 1; the
// per-variant ball constants in float64 (from B: persistent kernels pass
// their LDS copy, so that the float64 parameters do not hold scalar
// registers across the whole tile loop).  Called by all threads of a block.
__device__ void stage_frame(const DevParams &P, const BallParams64 &B, const FrameDev *frames,
                            const dpps_robot *robots, const dpps_variant *variants, int f,
                            StageLDS &S)
{
    const FrameDev F = frames[f];
    int tid = threadIdx.x;
    int nrob = F.n_team + F.n_opp;
    if (tid < nrob) {
        dpps_robot r = robots[F.robot_off + tid];
        int slot;
        if (tid < F.n_team) {
            slot = tid < F.passer ? tid : tid - 1;
        } else {
            slot = F.n_team - 1 + (tid - F.n_team);
        }
        if (tid != F.passer || tid >= F.n_team) S.rob[slot] = make_float4(r.x, r.y, r.vx, r.vy);
    }
    if (tid < F.n_variants) {
        // staged in order of kick type, then speed (stable): within a type
        // the first crossing never moves earlier as the speed grows
        const dpps_variant v = variants[F.variant_off + tid];
        int rank = 0;
        for (int j = 0; j < F.n_variants; ++j) {
            const dpps_variant u = variants[F.variant_off + j];
            rank += u.type < v.type ||
                    (u.type == v.type && (u.v0 < v.v0 || (u.v0 == v.v0 && j < tid)));
        }
        S.v0[rank] = v.v0;
        S.type[rank] = v.type;
        S.vidx[rank] = tid;
        S.vc[rank] = var_const(B, v.type, v.v0);
    }
    if (tid == 0) {
        S.n_tm = F.n_team - 1;
        S.n_op = F.n_opp;
        S.n_var = F.n_variants;
        int hf = 0, hc = 0;
        for (int v = 0; v < F.n_variants; ++v) {
            int t = variants[F.variant_off + v].type;
            hf |= t == DPPS_FLAT;
            hc |= t == DPPS_CHIP;
        }
        S.has_flat = hf;
        S.has_chip = hc;
        int ok = 1;
        for (int r = 0; r < nrob; ++r) {
            const dpps_robot R = robots[F.robot_off + r];
            ok &= fmaf(R.vx, R.vx, R.vy * R.vy) <= P.V * P.V;
        }
        S.vel_ok = ok;
        S.frame = f;
        S.bx = F.ball_x;
        S.by = F.ball_y;
    }
}

// Inclusive prefix maximum over the 64 lanes of a wave (lane l gets the
// maximum of lanes 0..l): four DPP row shifts give it within each row of 16
// lanes (lanes without a source see the identity), then two DPP row
// broadcasts carry lane 15 into row 1 and row 3, and lane 31 into rows 2
// and 3.  The maxima of critical speeds and arrival times are taken on the
// bit patterns: those are non-negative floats or +inf, which order as their
// bits read as signed integers, and an integer max needs no NaN quieting, so
// each DPP lane shift fuses into its max (identity INT_MIN, the bits of
// -0.0).
template <int CTRL, int ROW_MASK>
__device__ __forceinline__ int dpp_imax(int v)
{
    const int u = __builtin_amdgcn_update_dpp(INT_MIN, v, CTRL, ROW_MASK, 0xf, false);
    return max(v, u);
}

__device__ __forceinline__ int wave_prefix_imax(int v)
{
    v = dpp_imax<0x111, 0xf>(v);  // row_shr:1
    v = dpp_imax<0x112, 0xf>(v);  // row_shr:2
    v = dpp_imax<0x114, 0xf>(v);  // row_shr:4
    v = dpp_imax<0x118, 0xf>(v);  // row_shr:8
    v = dpp_imax<0x142, 0xa>(v);  // row_bcast:15 into rows 1 and 3
    return dpp_imax<0x143, 0xc>(v);  // row_bcast:31 into rows 2 and 3
}

// Lane l gets lane l - 1's value, lane 0 gets INT_MIN (DPP wave_shr:1).
__device__ __forceinline__ int wave_shift_up_i(int v)
{
    return __builtin_amdgcn_update_dpp(INT_MIN, v, 0x138, 0xf, 0xf, false);
}

// Order this wave's accesses to its own LDS row.
__device__ __forceinline__ void wave_lds_sync()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Arrival time of one robot at one sample.  Lengths are scaled by amax (a
// distance d becomes A d) and speeds by 1/sqrt(2); with that scaling the
// time-optimal straight-line motion that ends at rest takes
//   A T = R(D') + sigma sqrt(2) u',
//   R(D) = 2 sqrt(D) if D <= V^2, else D / V + V (cruising at vmax = V),
// where u' is the (scaled) speed toward the point, s = u'^2 the scaled
// stopping distance, delta the scaled distance still to cover, and either
// (overshoot: the robot cannot stop before the point, or is already there at
// rest) D' = s - delta, sigma = +1, or D' = s + delta, sigma = -1 (moving
// toward) / +1 (moving away).  The function returns A T / 2.
//
// The sample and the robot are given in the path frame of the candidate
// point: the sample lies at distance fq * LA along the path from the ball;
// r = (t, q^2, w.e, q w.n) holds the robot's own coordinate along the path
// (t) and across it (q), and its scaled velocity w projected on the path
// direction e and on the normal n.  The offset from the robot to the sample
// is then h e + q n with h = fq LA - t, its length sqrt(h^2 + q^2), and the
// speed toward the sample (h w.e + q w.n) / length.  With CLAMP that speed is
// limited to vmax; without it the caller knows that no robot is faster.
template <bool CLAMP>
__device__ __forceinline__ float robot_time_h(float4 r, float fq, float LA, const DevParams &P)
{
    const float h = fmaf(fq, LA, -r.x);
    const float r2 = fmaf(h, h, r.y);
    const float inv = rsq(r2);
    const float del = fmaxf(fmaf(r2, inv, -P.RA), 0.0f);
    float u = fmaf(h, r.z, r.w) * inv;
    if (CLAMP) u = med3(u, -P.Vh, P.Vh);
    const float ss = u * fabsf(u);  // its magnitude is u^2 (the add's abs modifier)
    const bool over = ss >= del;
    const float Dp = fabsf(ss) + (over ? -del : del);
    const float sg = over ? u : -u;
    const float rh = Dp > P.V2 ? fmaf(Dp, P.inv2V, P.halfV) : hsqrt(Dp);
    return fmaf(sg, 0.70710678118654752f, rh);
}

// Earliest arrival (A T / 2) of robots [j0, j0 + n) of the point's path
// frame `pr` at each of the lane's samples.
template <int KPL, bool CLAMP>
__device__ __forceinline__ void robot_stage(const float4 *pr, const DevParams &P, int j0, int n,
                                            const float (&fs)[KPL], float LA, float (&T)[KPL])
{
    // robots in pairs: two independent chains, joined by a three-way minimum
    int j = j0;
    for (; j + 1 < j0 + n; j += 2) {
        const float4 ra = pr[j], rb = pr[j + 1];
#pragma unroll
        for (int q = 0; q < KPL; ++q)
            T[q] = fminf(T[q], fminf(robot_time_h<CLAMP>(ra, fs[q], LA, P),
                                     robot_time_h<CLAMP>(rb, fs[q], LA, P)));
    }
    if (j < j0 + n) {
        const float4 r = pr[j];
#pragma unroll
        for (int q = 0; q < KPL; ++q) T[q] = fminf(T[q], robot_time_h<CLAMP>(r, fs[q], LA, P));
    }
}

// Robots [j0, j0 + n) of a side, sorted by ascending lower bound on their
// arrival times: after the first two, the side's latest arrival over all the
// wave's samples so far is taken, and the robots whose bound is not below it
// (a suffix of the sorted order) are left out: they cannot lower any
// sample's minimum, so the minima are those of all the side's robots.
// Arrival times are non-negative or +inf, bounds non-negative: both compare
// as their bits.
// The robots of the side among [j0, j0 + n) whose bound is below the
// latest of the arrival minima T over the wave's samples (a prefix of the
// sorted order; at least `done`).
template <int KPL>
__device__ __forceinline__ int robots_needed(const float4 *pr, int n, int done,
                                             uint32_t side_bit, const float (&T)[KPL])
{
    int m = __float_as_int(T[0]);
#pragma unroll
    for (int q = 1; q < KPL; ++q) m = max(m, __float_as_int(T[q]));
    m = __builtin_amdgcn_readlane(wave_prefix_imax(m), 63);
    const int l = lane_id();
    const uint32_t k = l < MAX_ROB ? bound_keys(pr)[l] : 0xFFFFFFFFu;
    const bool below = k != 0xFFFFFFFFu && (k & 0x80000000u) == side_bit &&
                       (int)(k & 0x7FFFFFFFu & ~(uint32_t)(MAX_ROB - 1)) < m;
    return min(max((int)__builtin_popcountll(__ballot(below)), done), n);
}

// Robots [j0, j0 + n) of a side, sorted by ascending lower bound on their
// arrival times: after the first two, and again after the next two, the
// side's latest arrival over all the wave's samples so far is taken, and the
// robots whose bound is not below it (a suffix of the sorted order) are left
// out: they cannot lower any sample's minimum, so the minima are those of
// all the side's robots.  Arrival times are non-negative or +inf, bounds
// non-negative: both compare as their bits.
template <int KPL, bool CLAMP>
__device__ __forceinline__ void robot_stage_bounded(const float4 *pr, const DevParams &P, int j0,
                                                    int n, uint32_t side_bit,
                                                    const float (&fs)[KPL], float LA,
                                                    float (&T)[KPL])
{
    // one copy of the pair body (the kernel's code stays small enough for
    // the instruction cache): the tests run after the pairs at 0 and 2
    int need = n;
    int j = 0;
    for (; j + 1 < need; j += 2) {
        const float4 ra = pr[j0 + j], rb = pr[j0 + j + 1];
#pragma unroll
        for (int q = 0; q < KPL; ++q)
            T[q] = fminf(T[q], fminf(robot_time_h<CLAMP>(ra, fs[q], LA, P),
                                     robot_time_h<CLAMP>(rb, fs[q], LA, P)));
        if (j < 4 && need > j + 2) need = robots_needed<KPL>(pr, need, j + 2, side_bit, T);
    }
    if (j < need) {
        const float4 r = pr[j0 + j];
#pragma unroll
        for (int q = 0; q < KPL; ++q) T[q] = fminf(T[q], robot_time_h<CLAMP>(r, fs[q], LA, P));
    }
}

// Path frame of a ball path along the unit direction e = (ux, uy) for the
// staged robots (lanes = robots), in float64 and then rounded once: for robot
// j with offset a = ball - x_j and normal n = (-e_y, e_x): t = -a.e and
// q = a.n (scaled by amax), w = velocity / sqrt(2), and pr[j] =
// (t, q^2, w.e, q w.n).  The lane frames robot l (lanes with l >= n_rob
// idle); every lane of the wave takes part (the row syncs are wave-wide).
template <bool SORT>
__device__ __forceinline__ void path_frame_dir(const StageLDS &S, const DevParams &P, float4 *pr,
                                               int n_rob, int n_tm, double LA, double ux,
                                               double uy, double bx, double by, int l)
{
    float4 fr = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
    uint32_t key = 0xFFFFFFFFu;
    if (l < n_rob) {
        const float4 r = S.rob[l];
        const double A = (double)P.A;
        const double ax = bx - (double)r.x, ay = by - (double)r.y;
        const double t = -(ax * ux + ay * uy) * A;
        const double q = (ay * ux - ax * uy) * A;
        const double we = ((double)r.z * ux + (double)r.w * uy) * 0.70710678118654752;
        const double wn = ((double)r.w * ux - (double)r.z * uy) * 0.70710678118654752;
        fr = make_float4((float)t, (float)(q * q + 1e-30), (float)we, (float)(q * wn));
        if (SORT) {
            // A lower bound on the robot's arrival time (robot stage units)
            // at every sample of the segment [0, LA] along e.  With delta =
            // max(dist - RA, 0) for its distance to the segment, and u' the
            // speed toward a sample (clamped to +-vmax/sqrt 2 as the stage
            // clamps it), the time -u'/sqrt 2 + R(u'^2 + delta) falls as u'
            // grows up to sqrt(delta) and grows with delta, so with U the
            // largest u' toward any sample: U < sqrt(delta) bounds it by
            // -U/sqrt 2 + R(U^2 + delta); otherwise, whatever the velocity,
            // by sqrt(delta / 2) for delta <= vmax^2 / 2 and else
            // delta / (2 vmax) + vmax / 4.  U: the scaled velocity w' = (w.e,
            // w.n) against the directions (h, q) to the samples, h in [-t,
            // LA - t]: |w'| when w' lies among them, else the larger end.
            // Less 2^-12 for the rounding of both computations, then
            // truncated to make room for the lane in the low bits.
            const double tc = t < 0.0 ? -t : (t > LA ? t - LA : 0.0);
            const float dseg = hsqrt((float)(q * q + tc * tc));
            const float del = fmaxf(dseg - P.RA, 0.0f);
            const float qf = (float)q, h0 = (float)(-t), h1 = (float)(LA - t);
            const float wef = (float)we, wnf = (float)wn;
            const float sq = qf < 0.0f ? -1.0f : 1.0f;
            const bool among = (h1 * wnf - qf * wef) * sq >= 0.0f &&
                               (wef * qf - wnf * h0) * sq >= 0.0f;
            const float u0 = fmaf(h0, wef, qf * wnf) * rsq(fmaxf(fmaf(h0, h0, qf * qf), 1e-30f));
            const float u1 = fmaf(h1, wef, qf * wnf) * rsq(fmaxf(fmaf(h1, h1, qf * qf), 1e-30f));
            const float U = med3(among ? hsqrt(fmaf(wef, wef, wnf * wnf)) : fmaxf(u0, u1),
                                 -P.Vh, P.Vh);
            float lb;
            if (U * fabsf(U) < del) {
                const float D = fmaf(U, U, del);
                lb = fmaf(-0.70710678118654752f, U,
                          D > P.V2 ? fmaf(D, P.inv2V, P.halfV) : hsqrt(D));
            } else {
                lb = del <= 0.5f * P.V2 ? hsqrt(0.5f * del) : fmaf(del, P.inv2V, 0.5f * P.halfV);
            }
            key = (__float_as_uint(lb * (1.0f - 1.0f / 4096.0f)) & ~(uint32_t)(MAX_ROB - 1)) |
                  (uint32_t)l | (l >= n_tm ? 0x80000000u : 0u);
        }
    }
    if (SORT) {
        // Rank by key: each side's robots by ascending bound (the side bit
        // puts the team's first), written to the rows in that order.  The
        // keys stay in the row's key block, by robot, for the bound test.
        uint32_t *const pk = bound_keys(pr);
        if (l < MAX_ROB) pk[l] = key;
        wave_lds_sync();
        int rank = 0;
        for (int j = 0; j < n_rob; j += 4) {
            const uint4 k4 = *(const uint4 *)(pk + j);
            rank += (k4.x < key) + (k4.y < key) + (k4.z < key) + (k4.w < key);
        }
        if (l < n_rob) pr[rank] = fr;
    } else if (l < n_rob) {
        pr[l] = fr;
    }
    // the row is written and read by this wave only
    wave_lds_sync();
}

// The same for the path from the ball to candidate point c: e = (c - ball) /
// |c - ball| (a point on the ball gets e = (1, 0); it is never reachable).
// 1 / |c - ball| is the hardware estimate refined by one Newton step
// (relative error far below the float32 rounding that follows).  Returns
// |c - ball| A.
__device__ __forceinline__ float path_frame(const StageLDS &S, const DevParams &P, float4 *pr,
                                            int n_rob, int n_tm, double cx64, double cy64,
                                            double bx, double by, int l)
{
    const double ex = cx64 - bx, ey = cy64 - by;
    const double L2 = ex * ex + ey * ey;
    double iL = __builtin_amdgcn_rsq(L2);
    iL = iL * (1.5 - 0.5 * L2 * iL * iL);
    const bool pos = L2 > 0.0;
    const double L = pos ? L2 * iL : 0.0;
    const double ux = pos ? ex * iL : 1.0, uy = pos ? ey * iL : 0.0;
    path_frame_dir<true>(S, P, pr, n_rob, n_tm, L * (double)P.A, ux, uy, bx, by, l);
    return (float)(L * (double)P.A);
}

// First crossings by running maxima.  The first crossing of a variant on
// one side is the lowest sample k whose critical speed vc_k is at least the
// kick speed v0 (K: none).  The running maximum of vc over the samples is
// non-decreasing, so that crossing is the number of samples whose running
// maximum is still below v0.  The wave writes each side's running maxima to a
// row of its LDS block (samples are lane-major: lane l holds k = l KPL + q),
// then every variant lane counts by binary search in its kick type's two rows,
// the team's and the opponents' searches interleaved.  The decisions are the
// comparisons v0 <= vc_k of a scan over k.
template <int KPL>
__device__ __forceinline__ void store_running_max(const float (&vc)[KPL], float *row)
{
    const int l = lane_id();
    int run[KPL];
    run[0] = __float_as_int(vc[0]);
#pragma unroll
    for (int q = 1; q < KPL; ++q) run[q] = max(run[q - 1], __float_as_int(vc[q]));
    const int excl = wave_shift_up_i(wave_prefix_imax(run[KPL - 1]));
#pragma unroll
    for (int q = 0; q < KPL; ++q) row[l * KPL + q] = __int_as_float(max(excl, run[q]));
}

template <int KPL>
__device__ __forceinline__ void count_below(const float *rt, const float *ro, float v0, int &kt,
                                            int &ko)
{
    // a search over 2^n >= K entries, those past K read as the last one (the
    // rows are non-decreasing, so the count only exceeds K when every entry
    // is below v0, and is then clamped); no branches, both sides interleaved.
    // The search moves row pointers (the step's offset goes into the LDS
    // read's immediate); when K is a power of two no read can pass the end.
    constexpr int K = KPL * 64;
    constexpr int S0 = KPL >= 3 ? 128 : (KPL == 2 ? 64 : 32);  // half of 2^n
    constexpr bool POW2 = (K & (K - 1)) == 0;
    const float *pt = rt, *po = ro;
    const float *const et = rt + (K - 1), *const eo = ro + (K - 1);
#pragma unroll
    for (int st = S0; st > 0; st >>= 1) {
        const float mt = POW2 ? pt[st - 1] : *min(pt + (st - 1), et);
        const float mo = POW2 ? po[st - 1] : *min(po + (st - 1), eo);
        pt += mt < v0 ? st : 0;
        po += mo < v0 ? st : 0;
    }
    const float mt = POW2 ? *pt : *min(pt, et);
    const float mo = POW2 ? *po : *min(po, eo);
    const int lt = (int)(pt - rt) + (mt < v0 ? 1 : 0);
    const int lo = (int)(po - ro) + (mo < v0 ? 1 : 0);
    kt = POW2 ? lt : min(lt, K);
    ko = POW2 ? lo : min(lo, K);
}

// Kick speed at which the ball covers distance s in exactly time T (the
// ball's distance at a fixed time grows with the kick speed).  Regimes at
// time T: stopped (s <= cA T^2), decelerating at the slower rate
// (quadratic in v0), or still in the fast phase (s >= cB T^2: sliding for a
// flat kick, in the air for a chip).  Stopped, the ball has covered its
// whole range cD v0^2, so v0 = sqrt(s / cD), which depends on the sample
// only.  In the fast phase a flat kick slides, v0 = (s + hfast T^2) / T, and
// a chip flies, v0 = s / (pfast T).  The slow root 2Q / (beta T +
// sqrt(4 alpha Q + beta^2 T^2)) is taken with numerator and denominator
// halved (Q / (hbeta T + sqrt(alpha Q + hbeta^2 T^2)), hbeta = beta / 2:
// power-of-two scalings, so the same value).  The terms that depend on the
// sample only, s / cA, s / cB and the stopped root, come precomputed, so
// that both sides share them.  T must be finite (a side with no robot has
// no crossing; the caller skips it).  Every regime's terms are formed first
// and then picked by plain selects (the fast and slow roots share one
// division), so that the lanes of a wave (samples in different regimes) do
// not split into branches.
template <bool CHIP>
__device__ __forceinline__ float vcrit(float T, float s, float s_icA, float s_icB, float v_stop,
                                       float alpha, float hbeta, float hbeta2, float hfast,
                                       float pfast, float half_ar)
{
    const float T2 = T * T;
    const float Q = fmaf(half_ar, T2, s);
    const bool stop = s_icA <= T2;
    const bool fast = s_icB >= T2;
    const float m_slow = fmaxf(fmaf(alpha, Q, hbeta2 * T2), 0.0f);
    const float d_slow = fmaf(hbeta, T, hsqrt(m_slow));
    const float N = fast ? (CHIP ? s : fmaf(hfast, T2, s)) : Q;
    const float D = fast ? (CHIP ? pfast * T : T) : d_slow;
    return stop ? v_stop : N * hrcp(D);
}

// The side-independent terms of the inversion at the lane's samples for one
// kick type.
template <int KPL, bool CHIP>
struct SampleTerms {
    float icA[KPL], icB[KPL], vst[KPL];
    __device__ __forceinline__ SampleTerms(const DevParams &P, const float (&sk)[KPL])
    {
#pragma unroll
        for (int q = 0; q < KPL; ++q) {
            icA[q] = sk[q] * (CHIP ? P.c_icA : P.f_icA);
            icB[q] = sk[q] * (CHIP ? P.c_icB : P.f_icB);
            vst[q] = hsqrt(sk[q] * (CHIP ? P.c_icD : P.f_icD));
        }
    }
};

// Critical speeds of one side at the lane's samples for one kick type (0 for
// every sample when the side has no robot).
template <int KPL, bool CHIP>
__device__ __forceinline__ void side_vcrit(const DevParams &P, int n_side, const float (&T)[KPL],
                                           const float (&sk)[KPL],
                                           const SampleTerms<KPL, CHIP> &st,
                                           const float (&vair)[KPL], float (&v)[KPL])
{
    if (n_side == 0) {
#pragma unroll
        for (int q = 0; q < KPL; ++q) v[q] = 0.0f;
        return;
    }
#pragma unroll
    for (int q = 0; q < KPL; ++q) {
        if (CHIP)
            v[q] = fminf(vair[q], vcrit<true>(T[q], sk[q], st.icA[q], st.icB[q], st.vst[q],
                                              P.c_alpha, P.c_hbeta, P.c_hbeta2, P.c_hfast,
                                              P.c_pfast, P.half_ar));
        else
            v[q] = vcrit<false>(T[q], sk[q], st.icA[q], st.icB[q], st.vst[q], P.f_alpha,
                                P.f_hbeta, P.f_hbeta2, P.f_hfast, P.f_pfast, P.half_ar);
    }
}

// Square root of a non-negative float64 from the hardware reciprocal square
// root estimate with two Newton steps (0 for 0): within a few units in the
// last place, in about half the instructions of the correctly rounded sqrt.
__device__ __forceinline__ double sqrt64(double q)
{
    double y = __builtin_amdgcn_rsq(q);
    y = y * fma(-0.5 * q, y * y, 1.5);
    y = y * fma(-0.5 * q, y * y, 1.5);
    return q > 0.0 ? q * y : 0.0;
}

// Ball time (float64) to distance s for staged variant c.
__device__ __forceinline__ double ball_time64(const VarConst &c, double s)
{
    bool ph1 = s <= c.split;
    double va = ph1 ? c.va1 : c.va2;
    double ac = ph1 ? c.a1 : c.a2;
    double so = ph1 ? 0.0 : c.soff2;
    double to = ph1 ? 0.0 : c.toff2;
    double x = s - so;
    double q = fmax(va * va - 2.0 * ac * x, 0.0);
    // sqrt(q) and the division from the hardware estimates with two Newton
    // steps each (relative error far below the float32 results need)
    double y = __builtin_amdgcn_rsq(q);
    y = y * fma(-0.5 * q, y * y, 1.5);
    y = y * fma(-0.5 * q, y * y, 1.5);
    const double den = va + (q > 0.0 ? q * y : 0.0);
    double r = __builtin_amdgcn_rcp(den);
    r = r * fma(-den, r, 2.0);
    r = r * fma(-den, r, 2.0);
    return fma(2.0 * x, r, to);
}

// Order-preserving map of a float's bits to an unsigned key (negative scores
// order below positive ones); a finite score never maps to 0, which marks
// "no feasible pass" in the argmax keys.
__device__ __forceinline__ uint32_t ordered_bits(float x)
{
    const uint32_t u = __float_as_uint(x);
    return u ^ ((u & 0x80000000u) ? 0xFFFFFFFFu : 0x80000000u);
}

__device__ __forceinline__ float unordered_bits(uint32_t k)
{
    return __uint_as_float(k ^ ((k & 0x80000000u) ? 0x80000000u : 0xFFFFFFFFu));
}

template <int CTRL, int ROW_MASK>
__device__ __forceinline__ unsigned long long dpp_max_u64(unsigned long long x)
{
    const int lo = __builtin_amdgcn_update_dpp(0, (int)(uint32_t)x, CTRL, ROW_MASK, 0xf, false);
    const int hi = __builtin_amdgcn_update_dpp(0, (int)(uint32_t)(x >> 32), CTRL, ROW_MASK, 0xf,
                                               false);
    const unsigned long long y = ((unsigned long long)(uint32_t)hi << 32) | (uint32_t)lo;
    return y > x ? y : x;
}

// Largest 64-bit key over the wave, on every lane: the DPP scan steps of
// wave_prefix_max (lanes without a source see 0), then lane 63's total.
__device__ __forceinline__ unsigned long long wave_max_u64(unsigned long long x)
{
    x = dpp_max_u64<0x111, 0xf>(x);
    x = dpp_max_u64<0x112, 0xf>(x);
    x = dpp_max_u64<0x114, 0xf>(x);
    x = dpp_max_u64<0x118, 0xf>(x);
    x = dpp_max_u64<0x142, 0xa>(x);
    x = dpp_max_u64<0x143, 0xc>(x);
    const uint32_t lo = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)x, 63);
    const uint32_t hi = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)(x >> 32), 63);
    return ((unsigned long long)hi << 32) | lo;
}

// Open goal angle at c = (cx, cy) against the staged opponents; lanes are
// opponents.  Returns the same value on every lane.
__device__ float open_angle(const StageLDS &S, const DevParams &P, float cx, float cy, int n_op,
                            int n_tm)
{
    int l = lane_id();
    float dxg = fmaxf(P.goal_x - cx, P.goal_eps);
    // lanes < n_op: direction to the opponent; lanes 62/63: to the goal posts
    float4 o = S.rob[n_tm + (l < n_op ? l : 0)];
    float ox = o.x - cx, oy = o.y - cy;
    float Y = l < n_op ? oy : (l == 62 ? -P.half_goal_w - cy : P.half_goal_w - cy);
    float X = l < n_op ? ox : dxg;
    float ang = atan2f(Y, X);
    float lo = readlane_f(ang, 62);
    float hi = readlane_f(ang, 63);
    bool valid = l < n_op && o.x < P.goal_x;
    float rho2 = fmaf(ox, ox, oy * oy);
    bool inside = valid && rho2 <= P.R * P.R;
    if (__ballot(inside)) return 0.0f;
    float al = asinf(fminf(P.R * rsq(fmaxf(rho2, 1e-30f)), 1.0f));
    float s = fmaxf(ang - al, lo);
    float e = fminf(ang + al, hi);
    bool has = valid && e > s;
    // union length: each interval contributes what the intervals sorted
    // before it (by start, then index) have not already covered
    const unsigned long long hm = __ballot(has);
    float M = -INFINITY;
    for (unsigned long long m = hm; m; m &= m - 1) {
        int k = __builtin_ctzll(m);
        float sk = readlane_f(s, k);
        float ek = readlane_f(e, k);
        bool before = sk < s || (sk == s && k < l);
        M = before ? fmaxf(M, ek) : M;
    }
    float contrib = has ? fmaxf(e - fmaxf(s, M), 0.0f) : 0.0f;
    float blocked = 0.0f;
    for (unsigned long long m = hm; m; m &= m - 1) blocked += readlane_f(contrib, __builtin_ctzll(m));
    return (hi - lo) - blocked;
}

// Passing power (Sec. 4.1, Eq. 1-2) for a pass over d64 metres whose
// receiver arrives after t_recv seconds: the ball should arrive t_recv +
// buffer; ignoring the sliding phase, the speed after it is (d + a t^2/2) / t
// while the ball still rolls at t, else the slowest ball that reaches the
// point, sqrt(2 a d); the kick speed is that over the slide ratio, clamped to
// [vmin, vmax]; 0 when no teammate can receive.
__device__ __forceinline__ double pass_power(const DevParams &P, double d64, float t_recv,
                                             double buffer, double vmin, double vmax)
{
    if (!(t_recv < INFINITY)) return 0.0;
    const double t = (double)t_recv + buffer;
    const double a = P.bp.a_r;
    const double v1 = d64 >= 0.5 * a * t * t ? (d64 + 0.5 * a * t * t) / t : sqrt(2.0 * a * d64);
    return fmin(fmax(v1 / P.bp.ratio, vmin), vmax);
}

// SBIP of every staged variant along one path of length d (metres; LA = d
// scaled by amax) whose path frame is in pr: robot stage over the lane's
// samples (lanes = samples, K/64 consecutive samples per lane), critical
// speeds, first crossings (pm: this wave's LDS block of 4 K floats).  On
// return lane v (a staged variant) holds its first team / opponent crossing
// samples (K: none).  With POWER the frame's variants are replaced by one
// flat pass at the power of Eq. 1-2 (lane 0), whose receiver is the first
// teammate at the last sample, the point itself; its speed is returned in v0.
template <int KPL, bool POWER>
__device__ __forceinline__ void sbip_crossings(const StageLDS &S, const DevParams &P,
                                               const float4 *pr, float *pm, float myv0,
                                               int mytype, float d, float LA, int &my_kt,
                                               int &my_ko, double d64 = 0.0, double buffer = 0.0,
                                               double vmin = 0.0, double vmax = 0.0,
                                               double *v0 = nullptr)
{
    const int l = lane_id();
    const int K = KPL * 64;
    const int n_tm = uni(S.n_tm), n_op = uni(S.n_op);
    const float invK = 1.0f / (float)K;

    float fs[KPL], sk[KPL], Tt[KPL], To[KPL];
#pragma unroll
    for (int q = 0; q < KPL; ++q) {
        fs[q] = (float)(l * KPL + q + 1) * invK;
        sk[q] = fs[q] * d;
        Tt[q] = INFINITY;
        To[q] = INFINITY;
    }
    // 1. robot stage, in the path frame
    if (uni(S.vel_ok)) {
        robot_stage_bounded<KPL, false>(pr, P, 0, n_tm, 0u, fs, LA, Tt);
        robot_stage_bounded<KPL, false>(pr, P, n_tm, n_op, 0x80000000u, fs, LA, To);
    } else {
        robot_stage_bounded<KPL, true>(pr, P, 0, n_tm, 0u, fs, LA, Tt);
        robot_stage_bounded<KPL, true>(pr, P, n_tm, n_op, 0x80000000u, fs, LA, To);
    }
    // 2-3. critical kick speeds per sample, then the first crossing of each
    // lane's variant (a side with no robot never intercepts: critical speed 0)
#pragma unroll
    for (int q = 0; q < KPL; ++q) {
        Tt[q] *= P.invA2;  // seconds
        To[q] *= P.invA2;
    }
    if (POWER) {
        const float t_recv = readlane_f(Tt[KPL - 1], 63);
        const double v = pass_power(P, d64, t_recv, buffer, vmin, vmax);
        *v0 = v;
        myv0 = (float)v;
        mytype = (l == 0 && v > 0.0) ? DPPS_FLAT : -1;
    }
    const unsigned long long flat_m = __ballot(mytype == DPPS_FLAT);
    const unsigned long long chip_m = __ballot(mytype == DPPS_CHIP);
    float *const pf = pm, *const pc = pm + 2 * K;  // flat rows, chip rows
    wave_lds_sync();  // the previous path's searches are done with the rows
    if (flat_m) {
        float vt[KPL], vo[KPL];
        const SampleTerms<KPL, false> st(P, sk);
        side_vcrit<KPL, false>(P, n_tm, Tt, sk, st, sk, vt);
        side_vcrit<KPL, false>(P, n_op, To, sk, st, sk, vo);
        store_running_max<KPL>(vt, pf);
        store_running_max<KPL>(vo, pf + K);
    }
    if (chip_m) {
        float vt[KPL], vo[KPL], vair[KPL];
#pragma unroll
        for (int q = 0; q < KPL; ++q) vair[q] = hsqrt(sk[q] * P.lam1_inv);
        const SampleTerms<KPL, true> st(P, sk);
        side_vcrit<KPL, true>(P, n_tm, Tt, sk, st, vair, vt);
        side_vcrit<KPL, true>(P, n_op, To, sk, st, vair, vo);
        store_running_max<KPL>(vt, pc);
        store_running_max<KPL>(vo, pc + K);
    }
    wave_lds_sync();
    my_kt = K;
    my_ko = K;
    if ((mytype == DPPS_FLAT) | (mytype == DPPS_CHIP)) {
        const float *r = mytype == DPPS_CHIP ? pc : pf;
        count_below<KPL>(r, r + K, myv0, my_kt, my_ko);
    }
}

// Evaluate candidate point (cx, cy) for every staged variant, its path
// frame already in pr (LA: |c - ball| A).  myv0 / mytype hold lane v's
// variant (lanes >= n_var: type -1).  On return lane v (< n_var) holds that
// variant's results.  With POWER the point has one flat variant at its own
// passing power (returned in o_v0), computed from the launch's buffer and
// kick range.
template <int KPL, bool POWER>
__device__ void eval_point(const StageLDS &S, const DevParams &P, const float4 *pr, float *pm,
                           float myv0, int mytype, float cx, float cy, double cx64,
                           double cy64, float LA, float &o_score, int &o_feas, float &o_tt,
                           float &o_to, float &o_v0, const LaunchArgs &a)
{
    const int l = lane_id();
    const int K = KPL * 64;
    const int n_tm = uni(S.n_tm), n_op = uni(S.n_op), n_var = uni(S.n_var);
    const float bx = unif(S.bx), by = unif(S.by);
    const float ex = cx - bx, ey = cy - by;
    const float d = hsqrt(fmaf(ex, ex, ey * ey));
    const double ex64 = cx64 - (double)bx, ey64 = cy64 - (double)by;
    const double d64 = sqrt64(ex64 * ex64 + ey64 * ey64);
    int my_kt, my_ko;
    double v0 = 0.0;
    sbip_crossings<KPL, POWER>(S, P, pr, pm, myv0, mytype, d, LA, my_kt, my_ko, d64,
                               (double)a.p_buffer, (double)a.p_vmin, (double)a.p_vmax, &v0);
    o_v0 = (float)v0;
    // 4. finish: lanes = variants
    o_score = -INFINITY;
    o_feas = 0;
    o_tt = INFINITY;
    o_to = INFINITY;
    bool feas = false;
    double m = -INFINITY;
    if (l < n_var && (!POWER || v0 > 0.0)) {
        const VarConst c = POWER ? var_const(P.bp, DPPS_FLAT, (float)v0) : S.vc[l];
        bool reach = d64 >= 1e-9 && d64 <= c.D && d64 >= c.sf_reach;
        double tt = INFINITY, to = INFINITY;
        if (reach) {
            if (my_kt < K) tt = ball_time64(c, (double)(my_kt + 1) * P.invK_d * d64);
            if (my_ko < K) to = ball_time64(c, (double)(my_ko + 1) * P.invK_d * d64);
        }
        bool tfin = tt < INFINITY;
        m = !tfin ? -INFINITY : (to < INFINITY ? to - tt : INFINITY);
        feas = reach && tfin && m >= P.margin_d;
        o_feas = feas;
        o_tt = (float)tt;
        o_to = (float)to;
    }
    // the open goal angle (lanes = opponents) enters only feasible scores
    if (__ballot(feas)) {
        const float ang = open_angle(S, P, cx, cy, n_op, n_tm);
        if (feas) {
            float gx = cx - P.goal_x;
            float dg = hsqrt(fmaf(gx, gx, cy * cy));
            float mc = fminf(fmaxf((float)m, 0.0f), P.margin_cap);
            o_score = fmaf(P.w_ang_pi, ang, fmaf(P.w_dist, fmaf(-dg, P.inv_dist_norm, 1.0f),
                                                 P.w_margin * mc));
        }
    }
}

// At most 128 VGPRs, so four waves fit on each SIMD.  POWER: one flat pass
// per point at the point's own passing power (Eq. 1-2).
template <int KPL, bool POWER>
__global__ void __launch_bounds__(512, 4) search_kernel(LaunchArgs a)
{
    __shared__ StageLDS S;
    __shared__ OutLDS O;
    // dynamic: each wave's running maxima (4 rows of K), its path frames of
    // two points, the tile's staged score and mask maps
    extern __shared__ float PMX[];
    __shared__ int s_tile;
    const DevParams &P = a.P;
    const int nw = blockDim.x >> 6;
    const int w = threadIdx.x >> 6;
    const int l = lane_id();
    const int TP = a.tile_points;
    float4 *const PR = (float4 *)(PMX + nw * PM_ROWS * KPL * 64);
    float *const OS = (float *)(PR + nw * 2 * PR_ENTRIES);
    uint8_t *const OM = (uint8_t *)(OS + MAX_VAR * TP);
    const bool reduced = (P.out_flags & DPPS_OUT_REDUCED) != 0;
    int iter = 0;
    int cur_frame = -1;
    float myv0 = 0.0f;
    int mytype = -1;
    int myvid = 0;  // the caller's index of lane l's variant
    // Persistent workgroups take the tiles round-robin (no atomics; tiles of
    // differing cost spread evenly) for all but the last one or two rounds,
    // whose tiles they then pull from the work counter as they finish, so
    // that the last tiles go to the workgroups that are free.
    const int G = (int)gridDim.x;
    const int n_tiles = a.n_frames_dev ? *a.n_frames_dev * a.tiles_per_frame : a.n_tiles;
    const int n_static = a.persistent ? max(n_tiles / G - 1, 0) * G : 0;
    if (threadIdx.x == 0) {  // read after the loop's first barrier
        S.bp = P.bp;
        O.wgbest.key = 0ull;
        O.wgbest.t_team = INFINITY;
        O.wgbest.t_opp = INFINITY;
        O.wgbest.v0 = 0.0f;
        O.wgbest.pad = 0.0f;
    }
    while (true) {
        // the previous tile (its staged results and records) is finished
        __syncthreads();
        int t = (int)blockIdx.x + iter * G;
        if (a.persistent && t >= n_static) {
            // a persistent grid's workgroup b sits on XCD b % 8, and so do
            // its static tiles when the grid is a multiple of 8; its dynamic
            // tiles keep that class too, from one counter per class, so
            // that the tiles an XCD runs together write neighbouring chunks
            // (below) and its L2 merges their lines.  C classes: every class
            // has a workgroup (a grid under 8 workgroups uses G classes).
            const int C = min(G, 8);
            const int x = (int)blockIdx.x % C;
            if (threadIdx.x == 0) s_tile = n_static + C * (int)atomicAdd(a.counter + x, 1u) + x;
            __syncthreads();
            t = s_tile;
        }
        if (t >= n_tiles) break;
        ++iter;
        TileDev tile;
        if (a.tiles_per_frame > 0) {
            tile.win = t / a.tiles_per_frame;
            tile.p0 = (t - tile.win * a.tiles_per_frame) * TP;
        } else {
            tile = a.tiles[t];
        }
        const WinDev W = a.wins[tile.win];
        if (W.frame != cur_frame) {
            stage_frame(a.P, S.bp, a.frames, a.robots, a.variants, W.frame, S);
            __syncthreads();
            cur_frame = W.frame;
            const int nv = S.n_var;
            myv0 = l < nv ? S.v0[l] : 0.0f;
            mytype = l < nv ? S.type[l] : -1;
            myvid = l < nv ? S.vidx[l] : 0;
        }
        const int n_var = S.n_var;
        // the window's points in chunks of CH; tile k of a window cut into T
        // tiles holds chunks pk, pk + T, pk + 2T, ...: every tile samples the
        // whole window, so tiles cost alike (neighbouring points cost alike,
        // distant ones do not) and the last round of tiles ends together,
        // while each chunk's outputs are still written as one 16-byte piece
        // per variant.  pk ranks the tiles by (k % 8, k / 8), so the tiles of
        // one class mod 8 (one XCD's, when the window's tiles start the
        // launch's tile list) hold neighbouring chunks.  Slot s of the tile
        // is point (pk + (s / CH) T) CH + s % CH; only the window's last
        // chunk can be short, and it is the last chunk of its tile.
        constexpr int CH = 4;
        const int tk = tile.p0 / TP;
        const int NC = (W.npts + CH - 1) / CH, cpt = TP / CH;
        const int Tw = max((NC + cpt - 1) / cpt, 1);  // = ceil(npts / TP)
        const int pk = (tk & 7) * (Tw >> 3) + min(tk & 7, Tw & 7) + (tk >> 3);
        const int nch = tk < Tw ? min(cpt, (NC - pk + Tw - 1) / Tw) : 0;
        const int npts =
            nch > 0 ? (nch - 1) * CH + min(CH, W.npts - (pk + (nch - 1) * Tw) * CH) : 0;
        unsigned long long bkey = 0ull;
        float btt = INFINITY, bto = INFINITY, bv0 = 0.0f;
        // the wave's points in pairs, slots s0 and s0 + nw: one pass of the
        // path-frame stage frames both (lanes 0-31 the first point's robots,
        // lanes 32-63 the second's; a lone last point is framed twice)
        for (int s0 = w; s0 < npts; s0 += 2 * nw) {
            const int n_pair = s0 + nw < npts ? 2 : 1;
            const int s1 = n_pair == 2 ? s0 + nw : s0;
            float LA0, LA1;
            {
                const int sl = l < 32 ? s0 : s1;
                const int p = (pk + (sl / CH) * Tw) * CH + (sl & (CH - 1));
                const int j = p / W.nx, i = p - j * W.nx;
                const float mi = (float)(W.i0 + i) - W.halfNx;
                const float mj = (float)(W.j0 + j) - W.halfNy;
                const float LAl = path_frame(S, P, PR + (w * 2 + (l >> 5)) * PR_ENTRIES,
                                             S.n_tm + S.n_op, S.n_tm,
                                             (double)W.h * (double)mi, (double)W.h * (double)mj,
                                             (double)unif(S.bx), (double)unif(S.by), l & 31);
                LA0 = readlane_f(LAl, 0);
                LA1 = readlane_f(LAl, 32);
            }
            for (int g = 0; g < n_pair; ++g) {
            const int slot = g ? s1 : s0;
            const int p = (pk + (slot / CH) * Tw) * CH + (slot & (CH - 1));
            const int j = p / W.nx, i = p - j * W.nx;
            const float mi = (float)(W.i0 + i) - W.halfNx;
            const float mj = (float)(W.j0 + j) - W.halfNy;
            const float cx = W.h * mi, cy = W.h * mj;
            const double cx64 = (double)W.h * (double)mi, cy64 = (double)W.h * (double)mj;
            float sc, tt, to, pv0;
            int fe;
            eval_point<KPL, POWER>(S, P, PR + (w * 2 + g) * PR_ENTRIES, PMX + w * PM_ROWS * KPL * 64,
                                   myv0, mytype, cx,
                                   cy, cx64, cy64, g ? LA1 : LA0, sc, fe, tt, to, pv0, a);
            if (POWER && l == 0 && a.v0_out) a.v0_out[W.out_base + p] = pv0;
            unsigned long long key = 0ull;
            if (fe) {
                uint32_t lin = (uint32_t)(W.elem_base + myvid * W.npts + p);
                key = ((unsigned long long)ordered_bits(sc) << 32) |
                      (unsigned long long)(0xFFFFFFFFu - lin);
            }
            if (key > bkey) {
                bkey = key;
                btt = tt;
                bto = to;
                bv0 = POWER ? pv0 : myv0;
            }
            if (reduced) {
                unsigned long long pk = wave_max_u64(key);
                if (l == 0) {
                    int64_t o = W.out_base + p;
                    if (a.score)
                        a.score[o] = pk ? unordered_bits((uint32_t)(pk >> 32)) : -INFINITY;
                    if (a.mask) {
                        uint32_t lin = 0xFFFFFFFFu - (uint32_t)pk;
                        a.mask[o] = pk ? (uint8_t)((lin - (uint32_t)W.elem_base) / (uint32_t)W.npts)
                                       : (uint8_t)255;
                    }
                }
            } else if (l < n_var) {
                OS[myvid * TP + slot] = sc;
                OM[myvid * TP + slot] = (uint8_t)fe;
                if (a.t_team) a.t_team[W.out_base + (int64_t)myvid * W.npts + p] = tt;
                if (a.t_opp) a.t_opp[W.out_base + (int64_t)myvid * W.npts + p] = to;
            }
            }
        }
        // the wave's best pass (and its times), then the tile's
        const unsigned long long wk = wave_max_u64(bkey);
        const unsigned long long who = __ballot(bkey == wk);
        const int src = who ? __builtin_ctzll(who) : 0;
        const float wtt = readlane_f(btt, src), wto = readlane_f(bto, src);
        const float wv0 = readlane_f(bv0, src);
        if (l == 0) {
            O.wbest[w].key = wk;
            O.wbest[w].t_team = wtt;
            O.wbest[w].t_opp = wto;
            O.wbest[w].v0 = wv0;
            O.wbest[w].pad = 0.0f;
        }
        __syncthreads();
        if (w == 0) {
            // lanes < nw hold the waves' records; the largest key wins (keys
            // of different waves differ unless both are 0)
            const unsigned long long k = l < nw ? O.wbest[l].key : 0ull;
            const unsigned long long tk = wave_max_u64(k);
            const unsigned long long at = __ballot(k == tk && l < nw);
            if (l == (int)__builtin_ctzll(at)) {
                TileRec r = O.wbest[l];
                if (r.key == 0ull) {
                    r.t_team = INFINITY;
                    r.t_opp = INFINITY;
                }
                if (!a.wg_records)
                    a.tile_rec[t] = r;
                else if (r.key > O.wgbest.key)
                    O.wgbest = r;
            }
        }
        if (!reduced) {
            const int tot = n_var * npts;
            for (int e = threadIdx.x; e < tot; e += blockDim.x) {
                const int v = e / npts, slot = e - v * npts;
                const int64_t o = W.out_base + (int64_t)v * W.npts + (pk + (slot / CH) * Tw) * CH +
                                  (slot & (CH - 1));
                if (a.score) a.score[o] = OS[v * TP + slot];
                if (a.mask) a.mask[o] = OM[v * TP + slot];
            }
        }
    }
    // (wave 0 made the last update of the workgroup's best before the barrier
    // that ended the loop)
    if (a.wg_records && threadIdx.x == 0) a.tile_rec[blockIdx.x] = O.wgbest;
}

// One workgroup per frame: reduce the frame's tile records to its best pass;
// block 0 also rearms the persistent work counter for the next launch.
__global__ void __launch_bounds__(256) finalize_kernel(LaunchArgs a)
{
    __shared__ TileRec red[256 / 64];
    __shared__ int s_wi;
    const int f = blockIdx.x;
    const int tid = threadIdx.x;
    if (f == 0 && tid < 8 && a.counter) a.counter[tid] = 0u;  // the search's 8 counters
    if (a.n_frames_dev && f >= *a.n_frames_dev) return;
    const FrameDev F = a.frames[f];
    // the frame's tile records, or one record per workgroup of a one-frame
    // launch
    const int rc = a.wg_records ? a.wg_records : F.tile_count;
    const int rb = a.wg_records ? 0 : F.tile_begin;
    TileRec r;
    r.key = 0ull;
    r.v0 = 0.0f;
    r.pad = 0.0f;
    r.t_team = INFINITY;
    r.t_opp = INFINITY;
    // four records in flight per thread (the keys are unique: order-free)
    for (int k0 = tid; k0 < rc; k0 += 4 * blockDim.x) {
        TileRec x[4];
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int k = k0 + q * blockDim.x;
            x[q].key = 0ull;
            if (k < rc) x[q] = a.tile_rec[rb + k];
        }
#pragma unroll
        for (int q = 0; q < 4; ++q)
            if (x[q].key > r.key) r = x[q];
    }
    // each wave's largest key by DPP, the waves' winners through LDS
    const unsigned long long wk = wave_max_u64(r.key);
    const unsigned long long who = __ballot(r.key == wk);
    if ((tid & 63) == (int)__builtin_ctzll(who)) red[tid >> 6] = r;
    if (tid == 0) s_wi = 0;
    __syncthreads();
    TileRec bestr = red[0];
    for (int q = 1; q < (int)(blockDim.x >> 6); ++q)
        if (red[q].key > bestr.key) bestr = red[q];
    // the window of the best element: the last window whose element base is
    // not above it (bases increase with the window), searched in parallel
    const uint32_t lin = 0xFFFFFFFFu - (uint32_t)bestr.key;
    if (bestr.key != 0ull)
        for (int k = tid; k < F.n_windows; k += blockDim.x)
            if ((uint32_t)a.wins[F.win_off + k].elem_base <= lin) atomicMax(&s_wi, k);
    __syncthreads();
    if (tid != 0) return;
    dpps_best b;
    b.found = 0; b.window = -1; b.variant = -1; b.i = -1; b.j = -1; b.type = -1;
    b.x = b.y = b.v0 = 0.0f;
    b.score = -INFINITY; b.t_team = INFINITY; b.t_opp = INFINITY; b.t_ball = INFINITY;
    b.pad = 0;
    if (bestr.key != 0ull) {
        const int wi = s_wi;
        const WinDev W = a.wins[F.win_off + wi];
        const uint32_t rel = lin - (uint32_t)W.elem_base;
        const int v = (int)(rel / (uint32_t)W.npts);
        const int p = (int)(rel - (uint32_t)v * (uint32_t)W.npts);
        const int j = p / W.nx, i = p - j * W.nx;
        const float mi = (float)(W.i0 + i) - W.halfNx;
        const float mj = (float)(W.j0 + j) - W.halfNy;
        const dpps_variant var = a.variants[F.variant_off + v];
        // the per-point power search passes one flat kick at the point's power
        const int ptype = a.power ? DPPS_FLAT : var.type;
        const float pv0 = a.power ? bestr.v0 : var.v0;
        const VarConst c = var_const(a.P.bp, ptype, pv0);
        double ex64 = (double)W.h * (double)mi - (double)F.ball_x;
        double ey64 = (double)W.h * (double)mj - (double)F.ball_y;
        b.found = 1;
        b.window = wi;
        b.variant = v;
        b.i = i;
        b.j = j;
        b.type = ptype;
        b.x = W.h * mi;
        b.y = W.h * mj;
        b.v0 = pv0;
        b.score = unordered_bits((uint32_t)(bestr.key >> 32));
        b.t_team = bestr.t_team;
        b.t_opp = bestr.t_opp;
        b.t_ball = (float)ball_time64(c, sqrt(ex64 * ex64 + ey64 * ey64));
    }
    a.best[a.best_map ? a.best_map[f] : f] = b;
    if (a.fb_on && (!b.found || b.score < a.fb.below)) {
        // this frame takes the exact fallback: one window over the whole lattice
        const int slot = atomicAdd(a.fb.count, 1);
        FrameDev G = F;
        G.n_windows = 1;
        G.win_off = slot;
        G.tile_begin = slot * a.fb.tiles_per_frame;
        G.tile_count = a.fb.tiles_per_frame;
        a.fb.frames[slot] = G;
        WinDev V;
        V.h = a.fb.h;
        V.i0 = 0;
        V.j0 = 0;
        V.nx = a.fb.nx;
        V.ny = a.fb.ny;
        V.halfNx = 0.5f * (float)(a.fb.nx - 1);
        V.halfNy = 0.5f * (float)(a.fb.ny - 1);
        V.frame = slot;
        V.npts = a.fb.nx * a.fb.ny;
        V.elem_base = 0;
        V.out_base = 0;
        a.fb.wins[slot] = V;
        a.fb.map[slot] = f;
    }
}


template <int KPL>
static int launch_kpl(const LaunchArgs &a, int waves_per_wg, int grid, hipStream_t st,
                      hipEvent_t e0, hipEvent_t e1)
{
    if (e0) (void)hipEventRecord(e0, st);
    if (a.n_tiles > 0 && grid > 0) {
        const size_t lds = search_lds_bytes(KPL * 64, waves_per_wg, a.tile_points);
        if (a.power)
            hipLaunchKernelGGL((search_kernel<KPL, true>), dim3(grid), dim3(64 * waves_per_wg),
                               lds, st, a);
        else
            hipLaunchKernelGGL((search_kernel<KPL, false>), dim3(grid), dim3(64 * waves_per_wg),
                               lds, st, a);
    }
    if (e1) (void)hipEventRecord(e1, st);
    if (a.n_frames > 0)
        hipLaunchKernelGGL(finalize_kernel, dim3(a.n_frames), dim3(256), 0, st, a);
    return hipGetLastError() == hipSuccess ? 0 : -1;
}

// ----------------------------------------------------------------------------
// The paper's direction x power form (Sec. 4.2): rays from the ball, the pass
// received at the first teammate's interception, five-feature score.
// ----------------------------------------------------------------------------

// Lane n of each row of 16 lanes, broadcast to its row (DPP row_newbcast).
template <int N>
__device__ __forceinline__ float row_newbcast(float v)
{
    return __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(v), 0x150 + N, 0xf, 0xf, true));
}

// Lane l ^ m within each group of 4 lanes (m = 1, 2, 3; DPP quad_perm; every
// source lane exists, so no old value is needed).
template <int M>
__device__ __forceinline__ float quad_xor(float v)
{
    constexpr int ctrl = M == 1 ? 0xB1 : M == 2 ? 0x4E : 0x1B;
    return __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(v), ctrl, 0xf, 0xf, true));
}

// Lane l ^ 7 within each group of 8 lanes (DPP row_half_mirror).
__device__ __forceinline__ float half_mirror(float v)
{
    return __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(v), 0x141, 0xf, 0xf, true));
}

// Lane l ^ 15 within each row of 16 lanes (DPP row_mirror).
__device__ __forceinline__ float row_mirror(float v)
{
    return __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(v), 0x140, 0xf, 0xf, true));
}

// Sum over each group of GS (8 or 16) lanes, on every lane of the group:
// pairs, then quads, then halves (each partner holds the same partial sum,
// so every lane gets the same bits).
template <int GS>
__device__ __forceinline__ float group_sum(float c)
{
    c += quad_xor<1>(c);
    c += quad_xor<2>(c);
    c += half_mirror(c);
    if (GS == 16) c += row_mirror(c);
    return c;
}

// Least / greatest value over the wave (DPP within each row of 16 lanes,
// then the four rows), on every lane.
__device__ __forceinline__ float wave_min_dpp(float x)
{
    x = fminf(x, quad_xor<1>(x));
    x = fminf(x, quad_xor<2>(x));
    x = fminf(x, half_mirror(x));
    x = fminf(x, row_mirror(x));
    return fminf(fminf(readlane_f(x, 0), readlane_f(x, 16)),
                 fminf(readlane_f(x, 32), readlane_f(x, 48)));
}
__device__ __forceinline__ float wave_max_dpp(float x)
{
    x = fmaxf(x, quad_xor<1>(x));
    x = fmaxf(x, quad_xor<2>(x));
    x = fmaxf(x, half_mirror(x));
    x = fmaxf(x, row_mirror(x));
    return fmaxf(fmaxf(readlane_f(x, 0), readlane_f(x, 16)),
                 fmaxf(readlane_f(x, 32), readlane_f(x, 48)));
}

// Covered length of the union of the intervals [s, e] held by the lanes of
// each group of GS lanes (GS = 8, or 16 for up to n <= 16 intervals; lane o of
// a group holds interval o, has marks a real interval, no end exceeds hi), on
// every lane of the group: each interval adds what the group's intervals
// sorted before it (by start, then index) have not covered.  M, the largest
// end among those, is formed with a median against hi, which needs no NaN
// quieting.
template <int GS>
__device__ __forceinline__ float group_cover(float s, float e, bool has, float hi, int o, int n)
{
    const float sh = has ? s : INFINITY;  // a start of +inf marks no interval
    float M = -INFINITY;
    if (GS == 8) {
        // interval of lane o ^ m of the group for m = 1..7 by DPP lane swaps
        // (l ^ m = l ^ 7 ^ (m ^ 7) for m >= 4); that lane sorts before this
        // one on equal starts when o has the highest bit of m set
        const float hs = half_mirror(sh), he = half_mirror(e);
        const bool hb1 = (o & 1) != 0, hb2 = (o & 2) != 0, hb4 = (o & 4) != 0;
#define GC_UNION(SJ, EJ, HB)                                             \
    {                                                                    \
        const float sj = (SJ), ej = (EJ);                                \
        const bool before = (sj < sh) || ((sj == sh) && (HB));           \
        M = before ? __builtin_amdgcn_fmed3f(M, ej, hi) : M;             \
    }
        GC_UNION(quad_xor<1>(sh), quad_xor<1>(e), hb1)
        GC_UNION(quad_xor<2>(sh), quad_xor<2>(e), hb2)
        GC_UNION(quad_xor<3>(sh), quad_xor<3>(e), hb2)
        GC_UNION(quad_xor<3>(hs), quad_xor<3>(he), hb4)
        GC_UNION(quad_xor<2>(hs), quad_xor<2>(he), hb4)
        GC_UNION(quad_xor<1>(hs), quad_xor<1>(he), hb4)
        GC_UNION(hs, he, hb4)
#undef GC_UNION
    } else {
        // interval j of the group by a row broadcast of lane j
#define GC_STEP(J)                                                                    \
    if (J < n) {                                                                      \
        const float sj = row_newbcast<J>(sh), ej = row_newbcast<J>(e);                \
        const bool before = (sj < sh) || ((sj == sh) && (J < o));                     \
        M = before ? __builtin_amdgcn_fmed3f(M, ej, hi) : M;                          \
    }
        GC_STEP(0) GC_STEP(1) GC_STEP(2) GC_STEP(3)
        GC_STEP(4) GC_STEP(5) GC_STEP(6) GC_STEP(7)
        GC_STEP(8) GC_STEP(9) GC_STEP(10) GC_STEP(11)
        GC_STEP(12) GC_STEP(13) GC_STEP(14) GC_STEP(15)
#undef GC_STEP
    }
    return group_sum<GS>(has ? fmaxf(e - fmaxf(s, M), 0.0f) : 0.0f);
}

// Open goal angle at up to 64 / GS points at once: lane GS g + o looks at
// point g (its own cx, cy, and the point's goal-post angles lo, hi) and
// opponent o (GS = 16 for up to 16 opponents, 8 for up to 8).  The same
// construction as open_angle within each group of GS lanes; returns on every
// lane the angle of its group's point.
template <int GS>
__device__ float open_angle_groups(const StageLDS &S, const DevParams &P, float cx, float cy,
                                   float lo, float hi, int n_op, int n_tm)
{
    const int l = lane_id();
    const int o = l & (GS - 1), base = l & (64 - GS);
    const float4 r = S.rob[n_tm + (o < n_op ? o : 0)];
    const float ox = r.x - cx, oy = r.y - cy;
    const bool valid = o < n_op && r.x < P.goal_x;
    const float rho2 = fmaf(ox, ox, oy * oy);
    const bool inside = valid && rho2 <= P.R * P.R;
    const float ang = atan2f(oy, ox);
    const float al = asinf(fminf(P.R * rsq(fmaxf(rho2, 1e-30f)), 1.0f));
    const float s = fmaxf(ang - al, lo);
    const float e = fminf(ang + al, hi);
    const bool has = valid && e > s;
    const float c = group_cover<GS>(s, e, has, hi, o, n_op);
    const unsigned long long gmask = GS == 16 ? 0xFFFFull : 0xFFull;
    const bool gin = ((__ballot(inside) >> base) & gmask) != 0ull;
    return gin ? 0.0f : (hi - lo) - c;
}

// Open goal angles at the passing points of a direction's feasible variants
// (lanes): a feasible lane whose passing sample differs from the previous
// feasible lane's leads.  The leaders write their points and goal-post
// angles, in lane order, to the wave's LDS block scr (64 float4; free once
// the crossings are known), their points go 64 / GS at a time through
// open_angle_groups, each angle goes back to its leader's entry, and every
// feasible lane reads its leader's.
template <int GS>
__device__ float leader_angles(const StageLDS &S, const DevParams &P, float *scr, bool feas,
                               int my_k, float px, float py, int n_op, int n_tm)
{
    constexpr int NG = 64 / GS;
    const int l = lane_id();
    const unsigned long long fm = __ballot(feas);
    const unsigned long long below = fm & ((1ull << l) - 1ull);
    const int prevl = below ? 63 - __builtin_clzll(below) : 0;
    const int kprev = __shfl(my_k, prevl, 64);
    const bool lead = feas && (below == 0ull || kprev != my_k);
    const unsigned long long lm = __ballot(lead);
    const int n_lead = __popcll(lm);
    float4 *const pts = (float4 *)scr;
    wave_lds_sync();  // the crossing searches are done with the block
    if (lead) {
        const float dxg = fmaxf(P.goal_x - px, P.goal_eps);
        pts[__popcll(lm & ((1ull << l) - 1ull))] =
            make_float4(px, py, atan2f(-P.half_goal_w - py, dxg), atan2f(P.half_goal_w - py, dxg));
    }
    wave_lds_sync();
    for (int c0 = 0; c0 < n_lead; c0 += NG) {
        const int idx = c0 + l / GS;
        const float4 q = pts[min(idx, n_lead - 1)];
        const float a = open_angle_groups<GS>(S, P, q.x, q.y, q.z, q.w, n_op, n_tm);
        if ((l & (GS - 1)) == 0 && idx < n_lead) scr[4 * idx + 2] = a;
    }
    wave_lds_sync();
    // a feasible lane's leader is the last leader at or below it
    const unsigned long long upto = l == 63 ? lm : lm & ((2ull << l) - 1ull);
    const float la = feas ? scr[4 * (__popcll(upto) - 1) + 2] : 0.0f;
    return la;
}

// Distance from the ball along (ux, uy) to the edge of the field (0 when the
// ray leaves at once).
__device__ __forceinline__ double ray_length(const DevParams &P, double bx, double by,
                                             double ux, double uy)
{
    const double hl = 0.5 * (double)P.field_len, hw = 0.5 * (double)P.field_wid;
    double L = INFINITY;
    if (ux > 0.0) L = fmin(L, (hl - bx) / ux);
    if (ux < 0.0) L = fmin(L, (-hl - bx) / ux);
    if (uy > 0.0) L = fmin(L, (hw - by) / uy);
    if (uy < 0.0) L = fmin(L, (-hw - by) / uy);
    return L > 0.0 ? L : 0.0;
}

struct RayOut {
    unsigned long long key;  // 0: not feasible
    float score, t_team, t_opp, s_recv, open_angle, refract;
    int feas;
};

// Every staged variant (lanes) for direction d of the staged frame.
// Unit vector of each kick direction, theta_d = 2 pi d / n from +x
// (computed once per direction count, read by every ray).
__global__ void __launch_bounds__(256) ray_dirs_kernel(double2 *dirs, int n)
{
    const int d = blockIdx.x * blockDim.x + threadIdx.x;
    if (d >= n) return;
    const double xd = 2.0 * (double)d / (double)n;  // theta_d / pi
    dirs[d] = make_double2(cospi(xd), sinpi(xd));
}

int launch_ray_dirs(double2 *dirs, int n, void *stream)
{
    hipLaunchKernelGGL(ray_dirs_kernel, dim3((n + 255) / 256), dim3(256), 0, (hipStream_t)stream,
                       dirs, n);
    return hipGetLastError() == hipSuccess ? 0 : -1;
}

template <int KPL>
__device__ RayOut ray_direction(const StageLDS &S, const DevParams &P, float4 *pr, float *pm,
                                float myv0, int mytype, int myvid, int d, const double2 *dirs,
                                float w_time, float w_refract)
{
    const int l = lane_id();
    const int K = KPL * 64;
    const int n_tm = uni(S.n_tm), n_op = uni(S.n_op), n_var = uni(S.n_var);
    const double bx = (double)unif(S.bx), by = (double)unif(S.by);
    const double2 u = dirs[d];
    const double ux = u.x, uy = u.y;
    const double L = ray_length(P, bx, by, ux, uy);
    path_frame_dir<true>(S, P, pr, n_tm + n_op, n_tm, L * (double)P.A, ux, uy, bx, by, l);
    int my_kt, my_ko;
    sbip_crossings<KPL, false>(S, P, pr, pm, myv0, mytype, (float)L, (float)(L * (double)P.A), my_kt,
                        my_ko);

    RayOut o;
    o.key = 0ull;
    o.score = -INFINITY;
    o.t_team = INFINITY;
    o.t_opp = INFINITY;
    o.s_recv = INFINITY;
    o.open_angle = 0.0f;
    o.refract = 0.0f;
    o.feas = 0;
    double px = 0.0, py = 0.0, m = -INFINITY;
    if (l < n_var) {
        // a crossing counts only where the ball gets to (within its stop)
        const VarConst c = S.vc[l];
        const double st = (double)(my_kt + 1) * P.invK_d * L;
        const double so = (double)(my_ko + 1) * P.invK_d * L;
        const double tt = (my_kt < K && st <= c.D) ? ball_time64(c, st) : INFINITY;
        const double to = (my_ko < K && so <= c.D) ? ball_time64(c, so) : INFINITY;
        const bool tfin = tt < INFINITY;
        m = !tfin ? -INFINITY : (to < INFINITY ? to - tt : INFINITY);
        o.feas = tfin && m >= P.margin_d;
        o.t_team = (float)tt;
        o.t_opp = (float)to;
        o.s_recv = tfin ? (float)st : INFINITY;
        px = bx + st * ux;
        py = by + st * uy;
    }
    // open goal angle at each feasible passing point
    const float my_ang = n_op <= 8 ? leader_angles<8>(S, P, pm, o.feas != 0, my_kt, (float)px,
                                                      (float)py, n_op, n_tm)
                                   : leader_angles<16>(S, P, pm, o.feas != 0, my_kt, (float)px,
                                                       (float)py, n_op, n_tm);
    if (o.feas) {
        const double gx = (double)P.goal_x - px, gy = -py;
        const float dg = (float)sqrt(gx * gx + gy * gy);
        const float refr = dg > 0.0f ? atan2f((float)fabs(ux * gy - uy * gx), (float)(ux * gx + uy * gy))
                                     : 0.0f;
        const float mc = fminf(fmaxf((float)m, 0.0f), P.margin_cap);
        const float sc = fmaf(P.w_ang_pi, my_ang,
                              fmaf(P.w_dist, fmaf(-dg, P.inv_dist_norm, 1.0f),
                                   fmaf(P.w_margin, mc,
                                        fmaf(-w_time, o.t_team, -w_refract * refr * 0.318309886183790672f))));
        o.score = sc;
        o.open_angle = my_ang;
        o.refract = refr;
        const uint32_t lin = (uint32_t)(d * n_var + myvid);
        o.key = ((unsigned long long)ordered_bits(sc) << 32) | (unsigned long long)(0xFFFFFFFFu - lin);
    }
    return o;
}

template <int KPL>
__global__ void __launch_bounds__(512, 4) ray_kernel(RayArgs a)
{
    __shared__ StageLDS S;
    __shared__ float4 PR[MAX_WAVES][PR_ENTRIES];
    extern __shared__ float PMX[];
    __shared__ RayRec WB[MAX_WAVES];
    __shared__ int s_tile;
    __shared__ int s_dir;  // next unclaimed direction slot of the tile
    const DevParams &P = a.P;
    const int nw = blockDim.x >> 6;
    const int w = threadIdx.x >> 6;
    const int l = lane_id();
    int cur_frame = -1;
    float myv0 = 0.0f;
    int mytype = -1, myvid = 0;
    // a contiguous run of tiles per workgroup (consecutive tiles share a
    // frame, so it is staged once per run) for all but the last one or two
    // rounds' worth, then the work counter
    const int G = (int)gridDim.x;
    const int R = max(a.n_tiles / G - 1, 0);
    const int n_static = R * G;
    int iter = 0;
    if (threadIdx.x == 0) {  // read after the loop's first barrier
        S.bp = P.bp;
        s_dir = nw;
    }
    while (true) {
        __syncthreads();  // the previous tile is finished
        int t = iter < R ? (int)blockIdx.x * R + iter : n_static;
        if (t >= n_static) {
            if (threadIdx.x == 0) s_tile = n_static + (int)atomicAdd(a.counter, 1u);
            __syncthreads();
            t = s_tile;
        }
        if (t >= a.n_tiles) break;
        ++iter;
        const TileDev tile = a.tiles[t];
        const int f = tile.win;
        if (f != cur_frame) {
            stage_frame(a.P, S.bp, a.frames, a.robots, a.variants, f, S);
            __syncthreads();
            cur_frame = f;
            const int nv = S.n_var;
            myv0 = l < nv ? S.v0[l] : 0.0f;
            mytype = l < nv ? S.type[l] : -1;
            myvid = l < nv ? S.vidx[l] : 0;
        }
        const int n_var = S.n_var;
        const int64_t base = a.frames[f].ray_base;
        const int nd = min(a.tile_dirs, a.n_dirs - tile.p0);
        // the wave's best so far: its key in a uniform register, its record
        // in the wave's LDS slot (written by the lane that holds it)
        unsigned long long wbk = 0ull;
        if (l == 0) {
            WB[w].key = 0ull;
            WB[w].t_team = WB[w].t_opp = WB[w].s_recv = INFINITY;
            WB[w].open_angle = WB[w].refract = WB[w].pad = 0.0f;
        }
        // each wave takes slot w, then claims the tile's next free slot as it
        // finishes one (directions differ in cost: the waves end together)
        for (int slot = w; slot < nd;) {
            const int d = tile.p0 + slot;
            const RayOut o = ray_direction<KPL>(S, P, PR[w], PMX + w * PM_ROWS * KPL * 64, myv0,
                                                mytype, myvid, d, a.dirs, a.w_time,
                                                a.w_refract);
            if (l < n_var) {
                const int64_t e = base + (int64_t)d * n_var + myvid;
                if (a.mask) a.mask[e] = (uint8_t)o.feas;
                if (a.score) a.score[e] = o.score;
                if (a.t_team) a.t_team[e] = o.t_team;
                if (a.t_opp) a.t_opp[e] = o.t_opp;
                if (a.s_recv) a.s_recv[e] = o.s_recv;
            }
            const unsigned long long dk = wave_max_u64(o.key);
            if (dk > wbk) {
                wbk = dk;
                const int src = __builtin_ctzll(__ballot(o.key == dk));
                if (l == src) {
                    WB[w].key = dk;
                    WB[w].t_team = o.t_team;
                    WB[w].t_opp = o.t_opp;
                    WB[w].s_recv = o.s_recv;
                    WB[w].open_angle = o.open_angle;
                    WB[w].refract = o.refract;
                }
            }
            int nx = 0;
            if (l == 0) nx = atomicAdd(&s_dir, 1);
            slot = uni(nx);
        }
        // the tile's best of the waves' records (keys of different waves
        // differ unless both are 0); the slot counter is rearmed for the
        // next tile, whose first barrier orders it before any claim
        __syncthreads();
        if (threadIdx.x == 0) s_dir = nw;
        if (w == 0) {
            const unsigned long long k = l < nw ? WB[l].key : 0ull;
            const unsigned long long tk = wave_max_u64(k);
            const unsigned long long at = __ballot(k == tk && l < nw);
            if (l == (int)__builtin_ctzll(at)) a.tile_rec[t] = WB[l];
        }
    }
}

// One workgroup per frame: reduce the frame's tile records into its best
// pass; block 0 also rearms the persistent work counter.
__global__ void __launch_bounds__(256) ray_finalize_kernel(RayArgs a)
{
    __shared__ RayRec red[256];
    const int f = blockIdx.x;
    const int tid = threadIdx.x;
    if (f == 0 && tid == 0) *a.counter = 0u;
    const FrameDev F = a.frames[f];
    RayRec r;
    r.key = 0ull;
    r.t_team = r.t_opp = r.s_recv = INFINITY;
    r.open_angle = r.refract = r.pad = 0.0f;
    for (int k = tid; k < F.tile_count; k += blockDim.x) {
        const RayRec x = a.tile_rec[F.tile_begin + k];
        if (x.key > r.key) r = x;
    }
    red[tid] = r;
    __syncthreads();
    for (int s = blockDim.x >> 1; s > 0; s >>= 1) {
        if (tid < s && red[tid + s].key > red[tid].key) red[tid] = red[tid + s];
        __syncthreads();
    }
    if (tid != 0) return;
    const RayRec b = red[0];
    dpps_ray_best o;
    o.found = 0; o.dir = -1; o.variant = -1; o.type = -1;
    o.theta = 0.0f; o.v0 = 0.0f; o.x = 0.0f; o.y = 0.0f;
    o.score = -INFINITY; o.t_team = INFINITY; o.t_opp = INFINITY;
    o.open_angle = 0.0f; o.refract = 0.0f; o.pad = 0;
    if (b.key != 0ull) {
        const uint32_t lin = 0xFFFFFFFFu - (uint32_t)b.key;
        const int d = (int)(lin / (uint32_t)F.n_variants);
        const int v = (int)(lin - (uint32_t)d * (uint32_t)F.n_variants);
        const dpps_variant var = a.variants[F.variant_off + v];
        const double th = 6.283185307179586476925 * (double)d / (double)a.n_dirs;
        const double xd = 2.0 * (double)d / (double)a.n_dirs;
        const double ux = cospi(xd), uy = sinpi(xd);
        o.found = 1;
        o.dir = d;
        o.variant = v;
        o.type = var.type;
        o.theta = (float)th;
        o.v0 = var.v0;
        o.x = (float)((double)F.ball_x + (double)b.s_recv * ux);
        o.y = (float)((double)F.ball_y + (double)b.s_recv * uy);
        o.score = unordered_bits((uint32_t)(b.key >> 32));
        o.t_team = b.t_team;
        o.t_opp = b.t_opp;
        o.open_angle = b.open_angle;
        o.refract = b.refract;
    }
    a.best[f] = o;
}

template <int KPL>
static int launch_ray_kpl(const RayArgs &a, int waves_per_wg, int grid, hipStream_t st,
                          hipEvent_t e0, hipEvent_t e1)
{
    if (e0) (void)hipEventRecord(e0, st);
    if (a.n_tiles > 0 && grid > 0)
        hipLaunchKernelGGL(ray_kernel<KPL>, dim3(grid), dim3(64 * waves_per_wg),
                           pm_bytes(KPL * 64, waves_per_wg), st, a);
    if (e1) (void)hipEventRecord(e1, st);
    if (a.n_frames > 0)
        hipLaunchKernelGGL(ray_finalize_kernel, dim3(a.n_frames), dim3(256), 0, st, a);
    return hipGetLastError() == hipSuccess ? 0 : -1;
}

int launch_ray(const RayArgs &a, int waves_per_wg, int grid, void *stream, void *ev_start,
               void *ev_stop)
{
    hipStream_t st = (hipStream_t)stream;
    hipEvent_t e0 = (hipEvent_t)ev_start, e1 = (hipEvent_t)ev_stop;
    switch (a.P.K / 64) {
    case 1: return launch_ray_kpl<1>(a, waves_per_wg, grid, st, e0, e1);
    case 2: return launch_ray_kpl<2>(a, waves_per_wg, grid, st, e0, e1);
    case 3: return launch_ray_kpl<3>(a, waves_per_wg, grid, st, e0, e1);
    case 4: return launch_ray_kpl<4>(a, waves_per_wg, grid, st, e0, e1);
    default: return -2;
    }
}

int ray_occupancy(int K, int waves_per_wg)
{
    int n = 0;
    hipError_t e = hipErrorInvalidValue;
    const int bs = 64 * waves_per_wg;
    switch (K / 64) {
    case 1: e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, ray_kernel<1>, bs, pm_bytes(1 * 64, waves_per_wg)); break;
    case 2: e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, ray_kernel<2>, bs, pm_bytes(2 * 64, waves_per_wg)); break;
    case 3: e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, ray_kernel<3>, bs, pm_bytes(3 * 64, waves_per_wg)); break;
    case 4: e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, ray_kernel<4>, bs, pm_bytes(4 * 64, waves_per_wg)); break;
    default: break;
    }
    return e == hipSuccess && n > 0 ? n : 1;
}

// ----------------------------------------------------------------------------
// Shooting decision (Sec. 4.4): the widest open gap of the goal mouth, then
// the opponents' interception along a flat shot through its centre.
// ----------------------------------------------------------------------------

// Ball time (float32) to distance s of a staged variant.
__device__ __forceinline__ float ball_time32(const VarConst &c, float s)
{
    const bool ph1 = s <= (float)c.split;
    const float va = ph1 ? (float)c.va1 : (float)c.va2;
    const float ac = ph1 ? (float)c.a1 : (float)c.a2;
    const float x = s - (ph1 ? 0.0f : (float)c.soff2);
    const float to = ph1 ? 0.0f : (float)c.toff2;
    const float q = fmaxf(fmaf(-2.0f * ac, x, va * va), 0.0f);
    return fmaf(2.0f * x, hrcp(va + hsqrt(q)), to);
}

// Earliest arrival (A T / 2), at each of the lane's samples, of the
// opponents [n_tm, n_tm + n_op) of a shot's path frame, sorted by ascending
// lower bound on their arrival over the path -- for the shot's least slack
// only.  After the first two opponents, and again after the next two, the
// slack so far is taken: the least, over the samples the ball reaches
// (sk <= D), of the arrival less the ball's time tb there; tbm is the latest
// of those ball times.  An opponent whose bound less tbm is not below that
// slack cannot lower it at any sample (its arrival is at least the bound, the
// ball's time at most tbm, and both roundings are monotone; the bound is
// shaved by 2^-16 and tbm raised by 2^-18 to cover the two forms'
// roundings), nor can the opponents after it in the sorted order: they are
// left out.  The minima can then differ at some samples; the least slack
// cannot.
template <int KPL>
__device__ __forceinline__ void shot_opponents(const float4 *pr, const DevParams &P, int n_tm,
                                               int n_op, const float (&fs)[KPL],
                                               const float (&sk)[KPL], const float (&tb)[KPL],
                                               float D, float LA, float tbm, float (&T)[KPL])
{
    const float tbh = tbm * (1.0f + 1.0f / 262144.0f);
    int need = n_op;
    int j = 0;
    for (; j + 1 < need; j += 2) {
        const float4 ra = pr[n_tm + j], rb = pr[n_tm + j + 1];
#pragma unroll
        for (int q = 0; q < KPL; ++q)
            T[q] = fminf(T[q], fminf(robot_time_h<true>(ra, fs[q], LA, P),
                                     robot_time_h<true>(rb, fs[q], LA, P)));
        if (j < 4 && need > j + 2) {
            float m = INFINITY;
#pragma unroll
            for (int q = 0; q < KPL; ++q) {
                const float d = T[q] * P.invA2 - tb[q];
                m = sk[q] <= D ? fminf(m, d) : m;
            }
            m = wave_min_dpp(m);
            const int l = lane_id();
            const uint32_t k = l < MAX_ROB ? bound_keys(pr)[l] : 0xFFFFFFFFu;
            const float kv = __uint_as_float(k & 0x7FFFFFFFu & ~(uint32_t)(MAX_ROB - 1));
            const bool opp = k != 0xFFFFFFFFu && (k & 0x80000000u) != 0u;
            const bool out = fmaf(kv * (1.0f - 1.0f / 65536.0f), P.invA2, -tbh) >= m;
            need = min(max((int)__builtin_popcountll(__ballot(opp && !out)), j + 2), need);
        }
    }
    if (j < need) {
        const float4 r = pr[n_tm + j];
#pragma unroll
        for (int q = 0; q < KPL; ++q) T[q] = fminf(T[q], robot_time_h<true>(r, fs[q], LA, P));
    }
}

// Open gaps of the goal mouth seen from (cx, cy); lanes are opponents, lane 62
// the lower post.  A gap starts at the lower post or at the end of a shadow
// that no other shadow covers, and runs to the next shadow start (or the
// upper post).  Returns the widest gap and its start (ties to the lower
// start) and the sum of the gaps; the same values on every lane.
__device__ __forceinline__ void shot_gaps(const StageLDS &S, const DevParams &P, float cx,
                                          float cy, int n_op, int n_tm, float &gap, float &g0,
                                          float &open)
{
    const int l = lane_id();
    const float dxg = fmaxf(P.goal_x - cx, P.goal_eps);
    const float4 o = S.rob[n_tm + (l < n_op ? l : 0)];
    const float ox = o.x - cx, oy = o.y - cy;
    const float Y = l < n_op ? oy : (l == 62 ? -P.half_goal_w - cy : P.half_goal_w - cy);
    const float X = l < n_op ? ox : dxg;
    const float ang = atan2f(Y, X);
    const float lo = readlane_f(ang, 62);
    const float hi = readlane_f(ang, 63);
    const bool valid = l < n_op && o.x < P.goal_x;
    const float rho2 = fmaf(ox, ox, oy * oy);
    gap = 0.0f;
    g0 = lo;
    open = 0.0f;
    if (__ballot(valid && rho2 <= P.R * P.R)) return;
    const float al = asinf(fminf(P.R * rsq(fmaxf(rho2, 1e-30f)), 1.0f));
    const float s = fmaxf(ang - al, lo);
    const float e = fminf(ang + al, hi);
    const bool has = valid && e > s;
    const unsigned long long hm = __ballot(has);
    const bool cand = has || l == 62;
    const float st = l == 62 ? lo : e;
    bool cov = false;
    float nxt = hi;
    for (unsigned long long m = hm; m; m &= m - 1) {
        const int k = __builtin_ctzll(m);
        const float sk = readlane_f(s, k);
        const float ek = readlane_f(e, k);
        cov = cov || (sk <= st && ek > st);
        nxt = sk > st ? fminf(nxt, sk) : nxt;
    }
    const float w = cand && !cov ? fmaxf(nxt - st, 0.0f) : 0.0f;
    const unsigned long long cm = __ballot(cand);
    for (unsigned long long m = cm; m; m &= m - 1) {
        const int k = __builtin_ctzll(m);
        const float wk = readlane_f(w, k);
        const float sk = readlane_f(st, k);
        open += wk;
        if (wk > gap || (wk == gap && wk > 0.0f && sk < g0)) {
            gap = wk;
            g0 = sk;
        }
    }
}

// The decision from shooter position (cx, cy) of the staged frame; lane 0's
// record is the result.
template <int KPL>
__device__ dpps_shot shot_origin(const StageLDS &S, const DevParams &P, float4 *pr, double cx,
                                 double cy, const VarConst &vc, float min_angle, float margin)
{
    const int l = lane_id();
    const int K = KPL * 64;
    const int n_tm = uni(S.n_tm), n_op = uni(S.n_op);
    const float fx = (float)cx, fy = (float)cy;
    float gap, g0, open;
    shot_gaps(S, P, fx, fy, n_op, n_tm, gap, g0, open);
    const double dxg = fmax((double)P.goal_x - cx, (double)P.goal_eps);
    const float aim = gap > 0.0f ? fmaf(0.5f, gap, g0) : atan2f(-fy, (float)dxg);
    const double ux = (double)cosf(aim), uy = (double)sinf(aim);
    const double L = dxg / ux;
    path_frame_dir<true>(S, P, pr, n_tm + n_op, n_tm, L * (double)P.A, ux, uy, cx, cy, l);
    const float Lf = (float)L, LA = (float)(L * (double)P.A);
    const float D = (float)vc.D;
    float fs[KPL], sk[KPL], tb[KPL], T[KPL];
    float tbm = -INFINITY;
#pragma unroll
    for (int q = 0; q < KPL; ++q) {
        fs[q] = (float)(q * 64 + l + 1) * (1.0f / (float)K);
        sk[q] = fs[q] * Lf;
        tb[q] = ball_time32(vc, sk[q]);
        T[q] = INFINITY;
        tbm = sk[q] <= D ? fmaxf(tbm, tb[q]) : tbm;
    }
    shot_opponents<KPL>(pr, P, n_tm, n_op, fs, sk, tb, D, LA, wave_max_dpp(tbm), T);
    float m = INFINITY;
#pragma unroll
    for (int q = 0; q < KPL; ++q) {
        const float d = T[q] * P.invA2 - tb[q];
        m = sk[q] <= D ? fminf(m, d) : m;
    }
    m = wave_min_dpp(m);
    dpps_shot r;
    r.reachable = L <= vc.D;
    r.aim = aim;
    r.gap = gap;
    r.open_angle = open;
    r.length = Lf;
    r.t_goal = r.reachable ? (float)ball_time64(vc, L) : INFINITY;
    r.slack = m;
    r.shoot = gap >= min_angle && r.reachable && m > margin;
    return r;
}

// BALL: one single-wave workgroup per frame, from the frame's ball.  MAP:
// one workgroup per tile of window points, each wave one point at a time.
template <int KPL, bool MAP>
__global__ void __launch_bounds__(512) shot_kernel(ShotArgs a)
{
    __shared__ StageLDS S;
    __shared__ float4 PR[MAX_WAVES][PR_ENTRIES];
    const DevParams &P = a.P;
    const int w = threadIdx.x >> 6;
    const int l = lane_id();
    const int t = blockIdx.x;
    const TileDev tile = MAP ? a.tiles[t] : TileDev{0, 0};
    const WinDev W = MAP ? a.wins[tile.win] : WinDev{};
    const int f = MAP ? W.frame : t;
    stage_frame(P, P.bp, a.frames, a.robots, a.variants, f, S);
    __syncthreads();
    const VarConst vc = var_const(P.bp, DPPS_FLAT, a.v_shot);
    if (!MAP) {
        const dpps_shot r = shot_origin<KPL>(S, P, PR[0], (double)S.bx, (double)S.by, vc,
                                             a.min_angle, a.margin);
        if (l == 0) a.ball[f] = r;
        return;
    }
    const int np = min(a.tile_points, W.npts - tile.p0);
    const int nw = blockDim.x >> 6;
    for (int slot = w; slot < np; slot += nw) {
        const int p = tile.p0 + slot;
        const int j = p / W.nx, i = p - j * W.nx;
        const double cx = (double)W.h * ((double)(W.i0 + i) - (double)W.halfNx);
        const double cy = (double)W.h * ((double)(W.j0 + j) - (double)W.halfNy);
        const dpps_shot r = shot_origin<KPL>(S, P, PR[w], cx, cy, vc, a.min_angle, a.margin);
        if (l == 0) a.map[W.out_base + p] = r;
    }
}

template <int KPL>
static int launch_shot_kpl(const ShotArgs &a, int waves_per_wg, hipStream_t st)
{
    if (a.n_frames > 0)
        hipLaunchKernelGGL((shot_kernel<KPL, false>), dim3(a.n_frames), dim3(64), 0, st, a);
    if (a.map && a.n_tiles > 0)
        hipLaunchKernelGGL((shot_kernel<KPL, true>), dim3(a.n_tiles), dim3(64 * waves_per_wg), 0,
                           st, a);
    return hipGetLastError() == hipSuccess ? 0 : -1;
}

int launch_shot(const ShotArgs &a, int waves_per_wg, void *stream)
{
    hipStream_t st = (hipStream_t)stream;
    if (waves_per_wg < 1 || waves_per_wg > MAX_WAVES) return -2;
    switch (a.P.K / 64) {
    case 1: return launch_shot_kpl<1>(a, waves_per_wg, st);
    case 2: return launch_shot_kpl<2>(a, waves_per_wg, st);
    case 3: return launch_shot_kpl<3>(a, waves_per_wg, st);
    case 4: return launch_shot_kpl<4>(a, waves_per_wg, st);
    default: return -2;
    }
}

// ----------------------------------------------------------------------------
// Running points (Sec. 5.2): five criteria per zone vertex, weighted (Eq. 4);
// lanes are points, the opponents are looped over from LDS.
// ----------------------------------------------------------------------------

// Arrival time (seconds) of staged robot r = (x, y, vx, vy) at (px, py): the
// scaled model of robot_time_h with the offset taken directly.
__device__ __forceinline__ float robot_time_pt(const DevParams &P, float4 r, float px, float py)
{
    const float dx = (px - r.x) * P.A, dy = (py - r.y) * P.A;
    const float r2 = fmaf(dx, dx, fmaf(dy, dy, 1e-30f));
    const float inv = rsq(r2);
    const float del = fmaxf(fmaf(r2, inv, -P.RA), 0.0f);
    float u = fmaf(dx, r.z, dy * r.w) * (0.70710678118654752f * inv);
    u = med3(u, -P.Vh, P.Vh);
    const float ss = u * fabsf(u);  // its magnitude is u^2 (the add's abs modifier)
    const bool over = ss >= del;
    const float Dp = fabsf(ss) + (over ? -del : del);
    const float sg = over ? u : -u;
    const float rh = Dp > P.V2 ? fmaf(Dp, P.inv2V, P.halfV) : hsqrt(Dp);
    return fmaf(sg, 0.70710678118654752f, rh) * P.invA2;
}

// Entry parameter of the segment from c along (dx, dy) into the rectangle
// [x0, x1] x [y0, y1] that holds its end point (slab form, FP64: a segment
// that grazes an edge must be decided as the oracle decides it).
__device__ __forceinline__ double slab_enter(double cx, double cy, double dx, double dy,
                                             double x0, double x1, double y0, double y1)
{
    // the slab's near side chosen before the one division per axis (the
    // same quotients; lanes whose dy signs differ share one division)
    double t = 0.0;
    if (dx != 0.0) t = fmax(t, ((dx > 0.0 ? x0 : x1) - cx) / dx);
    if (dy != 0.0) t = fmax(t, ((dy > 0.0 ? y0 : y1) - cy) / dy);
    return fmin(t, 1.0);
}

// The five criteria and the score at (cx, cy); returns -inf inside the
// defense area (crit untouched).
__device__ float run_eval(const StageLDS &S, const DevParams &P, const dpps_run_params &R,
                          double cx, double cy, int n_tm, int n_op, float (&crit)[5])
{
    const double x0d = (double)P.goal_x - (double)R.def_depth;
    const double hwd = 0.5 * (double)R.def_width;
    if (cx > x0d && cx < (double)P.goal_x && cy > -hwd && cy < hwd) return -INFINITY;
    const float fx = (float)cx, fy = (float)cy;
    // the offset to the goal centre in FP64, then rounded once: its sign
    // decides the bearing's branch for points on the goal line
    const float gx = (float)((double)P.goal_x - cx), gy = (float)(-cy);
    crit[0] = fmaf(-sqrtf(fmaf(gx, gx, gy * gy)), P.inv_dist_norm, 1.0f);
    const double bx = cx - (double)S.bx, by = cy - (double)S.by;
    const double db2 = bx * bx + by * by;
    crit[1] = fminf(sqrtf((float)db2) / R.ball_norm, 1.0f);
    const float phi = fabsf(atan2f(gy, gx));
    const float off = phi < R.ang_lo ? R.ang_lo - phi : (phi > R.ang_hi ? phi - R.ang_hi : 0.0f);
    crit[2] = fmaxf(1.0f - off / R.ang_fall, 0.0f);
    const double gxd = (double)P.goal_x - cx, hwg = (double)P.half_goal_w;
    const double dpy = hwg - cy, dqy = -hwg - cy;
    const double tp_ = slab_enter(cx, cy, gxd, dpy, x0d, (double)P.goal_x, -hwd, hwd);
    const double tq_ = slab_enter(cx, cy, gxd, dqy, x0d, (double)P.goal_x, -hwd, hwd);
    const float px = (float)(cx + tp_ * gxd), py = (float)(cy + tp_ * dpy);
    const float qx = (float)(cx + tq_ * gxd), qy = (float)(cy + tq_ * dqy);
    float tP = INFINITY, tQ = INFINITY, mark = 0.0f;
    for (int o = 0; o < n_op; ++o) {
        const float4 r = S.rob[n_tm + o];
        tP = fminf(tP, robot_time_pt(P, r, px, py));
        tQ = fminf(tQ, robot_time_pt(P, r, qx, qy));
        const double ox = (double)r.x - (double)S.bx, oy = (double)r.y - (double)S.by;
        const float ex = r.x - fx, ey = r.y - fy;
        const float wgt = fmaxf(1.0f - sqrtf(fmaf(ex, ex, ey * ey)) / R.mark_radius, 0.0f);
        mark = (ox * ox + oy * oy < db2) ? fmaxf(mark, wgt) : mark;
    }
    crit[3] = n_op > 0 ? fminf((tP + tQ) / R.guard_norm, 1.0f) : 1.0f;
    crit[4] = 1.0f - mark;
    return fmaf(R.w_goal, crit[0],
                fmaf(R.w_ball, crit[1],
                     fmaf(R.w_angle, crit[2], fmaf(R.w_guard, crit[3], R.w_defense * crit[4]))));
}

__global__ void __launch_bounds__(256) run_kernel(RunArgs a)
{
    __shared__ StageLDS S;
    __shared__ unsigned long long red[4];
    const DevParams &P = a.P;
    const WinDev W = a.wins[blockIdx.x];
    stage_frame(P, P.bp, a.frames, a.robots, a.variants, W.frame, S);
    __syncthreads();
    const int n_tm = S.n_tm, n_op = S.n_op;
    unsigned long long best = 0ull;
    for (int p = threadIdx.x; p < W.npts; p += blockDim.x) {
        const int j = p / W.nx, i = p - j * W.nx;
        const double cx = (double)W.h * ((double)(W.i0 + i) - (double)W.halfNx);
        const double cy = (double)W.h * ((double)(W.j0 + j) - (double)W.halfNy);
        float crit[5];
        const float sc = run_eval(S, P, a.R, cx, cy, n_tm, n_op, crit);
        if (a.score) a.score[W.out_base + p] = sc;
        if (sc > -INFINITY) {
            const unsigned long long k = ((unsigned long long)ordered_bits(sc) << 32) |
                                         (unsigned long long)(0xFFFFFFFFu - (uint32_t)p);
            best = k > best ? k : best;
        }
    }
    best = wave_max_u64(best);
    if (lane_id() == 0) red[threadIdx.x >> 6] = best;
    __syncthreads();
    if (threadIdx.x != 0) return;
    for (int w = 1; w < (int)(blockDim.x >> 6); ++w) best = red[w] > best ? red[w] : best;
    dpps_run_best r;
    r.found = 0; r.i = -1; r.j = -1; r.reserved = 0;
    r.x = 0.0f; r.y = 0.0f; r.score = -INFINITY;
    r.goal = r.ball = r.angle = r.guard = r.defense = 0.0f;
    if (best != 0ull) {
        const int p = (int)(0xFFFFFFFFu - (uint32_t)best);
        const int j = p / W.nx, i = p - j * W.nx;
        const double cx = (double)W.h * ((double)(W.i0 + i) - (double)W.halfNx);
        const double cy = (double)W.h * ((double)(W.j0 + j) - (double)W.halfNy);
        float crit[5];
        r.score = run_eval(S, P, a.R, cx, cy, n_tm, n_op, crit);
        r.found = 1; r.i = i; r.j = j;
        r.x = (float)cx; r.y = (float)cy;
        r.goal = crit[0]; r.ball = crit[1]; r.angle = crit[2]; r.guard = crit[3];
        r.defense = crit[4];
    }
    a.best[blockIdx.x] = r;
}

int launch_run(const RunArgs &a, void *stream)
{
    if (a.n_wins > 0)
        hipLaunchKernelGGL(run_kernel, dim3(a.n_wins), dim3(256), 0, (hipStream_t)stream, a);
    return hipGetLastError() == hipSuccess ? 0 : -1;
}

// Clears n words (one thread each): a kernel rather than a memset node, so
// that a caller may capture it in a graph.
__global__ void __launch_bounds__(64) zero_words_kernel(uint32_t *p, int n)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = 0u;
}

int launch_zero_words(uint32_t *p, int n, void *stream)
{
    if (n <= 0) return 0;
    hipLaunchKernelGGL(zero_words_kernel, dim3((n + 63) / 64), dim3(64), 0, (hipStream_t)stream,
                       p, n);
    return hipGetLastError() == hipSuccess ? 0 : -1;
}

int launch_search(const LaunchArgs &a, int waves_per_wg, int grid, void *stream, void *ev_start,
                  void *ev_stop)
{
    hipStream_t st = (hipStream_t)stream;
    hipEvent_t e0 = (hipEvent_t)ev_start, e1 = (hipEvent_t)ev_stop;
    switch (a.P.K / 64) {
    case 1: return launch_kpl<1>(a, waves_per_wg, grid, st, e0, e1);
    case 2: return launch_kpl<2>(a, waves_per_wg, grid, st, e0, e1);
    case 3: return launch_kpl<3>(a, waves_per_wg, grid, st, e0, e1);
    case 4: return launch_kpl<4>(a, waves_per_wg, grid, st, e0, e1);
    default: return -2;
    }
}

int search_occupancy(int K, int waves_per_wg, int tile_points)
{
    int n = 0;
    hipError_t e = hipErrorInvalidValue;
    const int bs = 64 * waves_per_wg;
    const size_t lds = search_lds_bytes(K, waves_per_wg, tile_points);
    switch (K / 64) {
    case 1: e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, search_kernel<1, false>, bs, lds); break;
    case 2: e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, search_kernel<2, false>, bs, lds); break;
    case 3: e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, search_kernel<3, false>, bs, lds); break;
    case 4: e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, search_kernel<4, false>, bs, lds); break;
    default: break;
    }
    return e == hipSuccess && n > 0 ? n : 1;
}

}  // namespace dpps
