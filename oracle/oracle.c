/*
 * oracle.c -- plain, slow FP64 reference of the SBIP-DPPS passing-point search
 * (arXiv 1909.07717, Sec. 4.1-4.4) and the running-point criteria of Sec. 5.2.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product library links, includes
 * or calls this file; only the test suite, the smoke check and the CPU
 * baseline leg of the benchmark load it.  It shares no code, header, table or
 * constant with the HIP path: every formula below is written out again from
 * the paper and from the readings listed with each function.
 *
 * What it computes, per candidate point c and pass variant (type, v0):
 *   - the ideal ball model's travel time to each of K path samples
 *     (Sec. 4.1: slide down to 5/7 of the kick speed, then roll to rest);
 *   - for every robot except the passer, its earliest interception along the
 *     sampled path (SBIP, Sec. 4.2): the ball time at the first sample the
 *     robot reaches no later than the ball;
 *   - the first-teammate and first-opponent interception times, the margin
 *     between them and the feasibility filter (Sec. 4.3, last feature);
 *   - the weighted-sum score of Eq. (3) with lengths and angles divided by
 *     their upper bound (Sec. 4.3);
 *   - the argmax over everything (Sec. 4.3, best pass line).
 * The per-robot interception times are computed robot by robot, with no
 * factorisation across robots or variants.
 *
 * Readings where the paper is silent (the paper's own figure of the ball
 * model and its interception predictor are not available):
 *   ball deceleration values, chip model, path sampling, robot arrival time,
 *   the open goal angle and the lattice follow the configuration constants
 *   passed in orc_params; each function states the reading it implements.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define ORC_FLAT 0
#define ORC_CHIP 1

/* ambiguity flags (parity bands) */
#define ORC_AMB_REACH 1   /* |d - D| or |d - s_f| below eps_reach           */
#define ORC_AMB_LAND 2    /* chip sample within eps_land of the landing point */
#define ORC_AMB_CROSS 4   /* a robot's arrival within the crossing band       */
#define ORC_AMB_MARGIN 8  /* margin within eps_margin of the threshold        */

typedef struct {
    double field_len, field_wid, goal_x, goal_width;
    double robot_radius, vmax, amax;
    double slide_decel, roll_decel, slide_ratio;
    double chip_angle, gravity;
    double margin_s, margin_cap_s;
    double w_angle, w_dist, w_margin, dist_norm;
    double goal_eps;
    int32_t n_samples;
    int32_t n_threads;
    /* parity bands, used only when bands are requested */
    double eps_reach, eps_land, eps_cross_t, eps_cross_s, eps_margin;
} orc_params;

typedef struct {
    int32_t n_team, n_opp, passer, pad;
    const double *team; /* n_team x (x, y, vx, vy) */
    const double *opp;  /* n_opp  x (x, y, vx, vy) */
    double ball_x, ball_y;
} orc_world;

typedef struct {
    int32_t reachable, feasible, ambig, pad;
    double t_team, t_opp, margin, score, open_angle;
} orc_result;

/* ------------------------------------------------------------------------ */
/* Ball model (Sec. 4.1).                                                    */
/* ------------------------------------------------------------------------ */

/* Stopping distance D and, for chips, the carry s_f (flat: s_f = 0).
 * Flat: the ball slides from v0 down to v1 = ratio * v0 at the sliding
 * deceleration, covering (v0^2 - v1^2) / (2 a_s), then rolls from v1 to rest,
 * covering v1^2 / (2 a_r).  The forward model keeps the sliding distance.
 * Chip (no model in the paper; reading): launched at v0 and the chip angle with
 * no drag, it lands after s_f = v_h * 2 v_z / g and then rolls from the
 * horizontal speed v_h to rest at the rolling deceleration. */
void orc_ball_range(const orc_params *P, int type, double v0, double *D, double *s_f)
{
    if (type == ORC_CHIP) {
        double vh = v0 * cos(P->chip_angle), vz = v0 * sin(P->chip_angle);
        double tf = 2.0 * vz / P->gravity;
        double sf = vh * tf;
        *s_f = sf;
        *D = sf + vh * vh / (2.0 * P->roll_decel);
    } else {
        double v1 = P->slide_ratio * v0;
        double d1 = (v0 * v0 - v1 * v1) / (2.0 * P->slide_decel);
        *s_f = 0.0;
        *D = d1 + v1 * v1 / (2.0 * P->roll_decel);
    }
}

/* Time for the ball to travel distance s along its path; +inf beyond the
 * stopping distance.  Under constant deceleration a from speed v, the time to
 * cover x is the smaller root of x = v t - a t^2 / 2, written here in the
 * cancellation-free form 2x / (v + sqrt(v^2 - 2 a x)). */
static double phase_time(double v, double a, double x)
{
    double q = v * v - 2.0 * a * x;
    if (q < 0.0) q = 0.0;
    return 2.0 * x / (v + sqrt(q));
}

double orc_ball_time(const orc_params *P, int type, double v0, double s)
{
    double D, sf;
    orc_ball_range(P, type, v0, &D, &sf);
    if (s > D) return INFINITY;
    if (type == ORC_CHIP) {
        double vh = v0 * cos(P->chip_angle), vz = v0 * sin(P->chip_angle);
        double tf = 2.0 * vz / P->gravity;
        if (s <= sf) return s / vh; /* in the air: horizontal speed is constant */
        return tf + phase_time(vh, P->roll_decel, s - sf);
    } else {
        double v1 = P->slide_ratio * v0;
        double t1 = (v0 - v1) / P->slide_decel;
        double d1 = (v0 * v0 - v1 * v1) / (2.0 * P->slide_decel);
        if (s <= d1) return phase_time(v0, P->slide_decel, s);
        return t1 + phase_time(v1, P->roll_decel, s - d1);
    }
}

/* Distance travelled by the ball at time t (the forward model; only used for
 * the parity bands). */
double orc_ball_dist(const orc_params *P, int type, double v0, double t)
{
    double D, sf;
    orc_ball_range(P, type, v0, &D, &sf);
    if (type == ORC_CHIP) {
        double vh = v0 * cos(P->chip_angle), vz = v0 * sin(P->chip_angle);
        double tf = 2.0 * vz / P->gravity;
        if (t <= tf) return vh * t;
        double tau = t - tf, tr = vh / P->roll_decel;
        if (tau >= tr) return D;
        return sf + vh * tau - 0.5 * P->roll_decel * tau * tau;
    } else {
        double v1 = P->slide_ratio * v0;
        double t1 = (v0 - v1) / P->slide_decel;
        double d1 = (v0 * v0 - v1 * v1) / (2.0 * P->slide_decel);
        if (t <= t1) return v0 * t - 0.5 * P->slide_decel * t * t;
        double tau = t - t1, tr = v1 / P->roll_decel;
        if (tau >= tr) return D;
        return d1 + v1 * tau - 0.5 * P->roll_decel * tau * tau;
    }
}

/* ------------------------------------------------------------------------ */
/* Robot arrival time (reading: the cited predictor is not available).       */
/* Straight-line 1-D motion with |a| <= A and |v| <= V that ends at rest at   */
/* the point.  delta is the distance left to cover (centre distance minus the */
/* robot radius, floored at 0); u is the initial speed along the line toward  */
/* the point (negative: moving away).                                        */
/* ------------------------------------------------------------------------ */

/* From rest to rest over distance D: triangular if D < V^2/A, else
 * accelerate, cruise at V, decelerate. */
static double rest_to_rest(double D, double A, double V)
{
    if (D >= V * V / A) return D / V + V / A;
    return 2.0 * sqrt(D / A);
}

double orc_robot_time(const orc_params *P, double delta, double u)
{
    double A = P->amax, V = P->vmax;
    if (u < 0.0) {
        /* stop first (time -u/A, drifting u^2/2A further away), then go */
        return -u / A + rest_to_rest(delta + u * u / (2.0 * A), A, V);
    }
    double stop = u * u / (2.0 * A);
    if (stop >= delta) {
        /* cannot stop in time: overshoot, stop, come back */
        return u / A + rest_to_rest(stop - delta, A, V);
    }
    /* accelerate from u to a peak speed, then decelerate to rest */
    double d_acc = (V * V - u * u) / (2.0 * A) + V * V / (2.0 * A);
    if (delta >= d_acc) return (V - u) / A + V / A + (delta - d_acc) / V;
    double vp = sqrt(A * delta + 0.5 * u * u);
    return (2.0 * vp - u) / A;
}

/* Arrival time of robot (x, y, vx, vy) at point (px, py). */
static double robot_time_to(const orc_params *P, const double *rb, double px, double py)
{
    double dx = px - rb[0], dy = py - rb[1];
    double rho = sqrt(dx * dx + dy * dy);
    double delta = rho - P->robot_radius;
    if (delta < 0.0) delta = 0.0;
    double u = 0.0;
    if (rho > 0.0) u = (rb[2] * dx + rb[3] * dy) / rho;
    if (u > P->vmax) u = P->vmax;
    if (u < -P->vmax) u = -P->vmax;
    return orc_robot_time(P, delta, u);
}

double orc_robot_time_to(const orc_params *P, double x, double y, double vx, double vy,
                         double px, double py)
{
    double rb[4] = {x, y, vx, vy};
    return robot_time_to(P, rb, px, py);
}

/* ------------------------------------------------------------------------ */
/* SBIP for one robot (Sec. 4.2).                                            */
/* K samples uniform in distance along the segment from the ball b to c:     */
/* f_k = (k+1)/K, so the kick point is excluded and the target included.     */
/* The robot intercepts at sample k when its arrival time there does not     */
/* exceed the ball's; its interception time is the ball time at the first    */
/* such sample.  Chip samples still in the air cannot be intercepted.        */
/* ------------------------------------------------------------------------ */
typedef struct {
    double bx, by, cx, cy, d, D, sf, v0;
    int type;
} orc_path;

static double sbip_robot(const orc_params *P, const orc_path *pa, const double *rb, int *k_hit)
{
    int K = P->n_samples;
    for (int k = 0; k < K; ++k) {
        double f = (double)(k + 1) / (double)K;
        double s = f * pa->d;
        if (pa->type == ORC_CHIP && s < pa->sf) continue;
        double tb = orc_ball_time(P, pa->type, pa->v0, s);
        double px = pa->bx + f * (pa->cx - pa->bx);
        double py = pa->by + f * (pa->cy - pa->by);
        double tr = robot_time_to(P, rb, px, py);
        if (tr <= tb) {
            if (k_hit) *k_hit = k;
            return tb;
        }
    }
    if (k_hit) *k_hit = K;
    return INFINITY;
}

double orc_sbip_robot(const orc_params *P, double bx, double by, double cx, double cy,
                      int type, double v0, double x, double y, double vx, double vy, int *k_hit)
{
    orc_path pa;
    pa.bx = bx; pa.by = by; pa.cx = cx; pa.cy = cy;
    pa.d = sqrt((cx - bx) * (cx - bx) + (cy - by) * (cy - by));
    pa.type = type; pa.v0 = v0;
    orc_ball_range(P, type, v0, &pa.D, &pa.sf);
    double rb[4] = {x, y, vx, vy};
    return sbip_robot(P, &pa, rb, k_hit);
}

/* ------------------------------------------------------------------------ */
/* Open goal angle (Sec. 4.3 shoot-angle feature, Sec. 4.4 valid angle).     */
/* Directions from c to the goal mouth [goal_x] x [-w/2, w/2] not shadowed   */
/* by an opponent disc of the robot radius; opponents at or beyond the goal  */
/* line do not block; a point inside an opponent disc has angle 0.           */
/* The depth to the goal line is floored at goal_eps.                        */
/* ------------------------------------------------------------------------ */
double orc_open_angle(const orc_params *P, double cx, double cy, int n_opp, const double *opp)
{
    double dx = P->goal_x - cx;
    if (dx < P->goal_eps) dx = P->goal_eps;
    double lo = atan2(-0.5 * P->goal_width - cy, dx);
    double hi = atan2(0.5 * P->goal_width - cy, dx);
    double a[32], b[32];
    int n = 0;
    for (int o = 0; o < n_opp; ++o) {
        const double *r = opp + 4 * o;
        if (r[0] >= P->goal_x) continue;
        double ox = r[0] - cx, oy = r[1] - cy;
        double rho = sqrt(ox * ox + oy * oy);
        if (rho <= P->robot_radius) return 0.0;
        double phi = atan2(oy, ox);
        double al = asin(P->robot_radius / rho);
        double s = phi - al, e = phi + al;
        if (s < lo) s = lo;
        if (e > hi) e = hi;
        if (e > s && n < 32) {
            a[n] = s; b[n] = e; ++n;
        }
    }
    /* sort the blocked intervals by start, then merge */
    for (int i = 1; i < n; ++i) {
        double sa = a[i], sb = b[i];
        int j = i - 1;
        while (j >= 0 && a[j] > sa) {
            a[j + 1] = a[j]; b[j + 1] = b[j]; --j;
        }
        a[j + 1] = sa; b[j + 1] = sb;
    }
    double blocked = 0.0, cs = 0.0, ce = 0.0;
    int open = 0;
    for (int i = 0; i < n; ++i) {
        if (!open) { cs = a[i]; ce = b[i]; open = 1; continue; }
        if (a[i] <= ce) { if (b[i] > ce) ce = b[i]; }
        else { blocked += ce - cs; cs = a[i]; ce = b[i]; }
    }
    if (open) blocked += ce - cs;
    return (hi - lo) - blocked;
}

/* ------------------------------------------------------------------------ */
/* One (point, variant): interception times, feasibility, score.            */
/* ------------------------------------------------------------------------ */
/* Parity bands of one side (not part of the search): at every sample up to
 * and including the side's first interception, the side's earliest arrival
 * (minimum over its robots) is compared with the ball; a sample whose
 * decision lies within eps_cross_t in time, or within eps_cross_s in ball
 * position, marks the entry ambiguous, and so does a chip sample within
 * eps_land of the landing point that the side could reach. */
static void side_bands(const orc_params *P, const orc_path *pa, const double *robots,
                       int n, int skip, int k_side, int *amb)
{
    int K = P->n_samples;
    int klim = k_side < K ? k_side : K - 1;
    for (int k = 0; k <= klim; ++k) {
        double f = (double)(k + 1) / (double)K;
        double s = f * pa->d;
        double px = pa->bx + f * (pa->cx - pa->bx);
        double py = pa->by + f * (pa->cy - pa->by);
        double tmin = INFINITY;
        for (int j = 0; j < n; ++j) {
            if (j == skip) continue;
            double tr = robot_time_to(P, robots + 4 * j, px, py);
            if (tr < tmin) tmin = tr;
        }
        if (!isfinite(tmin)) return;
        if (pa->type == ORC_CHIP && fabs(s - pa->sf) < P->eps_land) {
            double tb_land = s / (pa->v0 * cos(P->chip_angle));
            if (tmin <= tb_land + P->eps_cross_t) *amb |= ORC_AMB_LAND;
        }
        if (pa->type == ORC_CHIP && s < pa->sf) continue;
        double tb = orc_ball_time(P, pa->type, pa->v0, s);
        if (fabs(tmin - tb) < P->eps_cross_t) *amb |= ORC_AMB_CROSS;
        double sb = orc_ball_dist(P, pa->type, pa->v0, tmin);
        if (fabs(sb - s) < P->eps_cross_s) *amb |= ORC_AMB_CROSS;
    }
}

void orc_eval(const orc_params *P, const orc_world *W, int type, double v0,
              double cx, double cy, int bands, orc_result *out)
{
    orc_path pa;
    pa.bx = W->ball_x; pa.by = W->ball_y; pa.cx = cx; pa.cy = cy;
    pa.d = sqrt((cx - pa.bx) * (cx - pa.bx) + (cy - pa.by) * (cy - pa.by));
    pa.type = type; pa.v0 = v0;
    orc_ball_range(P, type, v0, &pa.D, &pa.sf);

    memset(out, 0, sizeof(*out));
    out->open_angle = orc_open_angle(P, cx, cy, W->n_opp, W->opp);
    int amb = 0;
    if (bands) {
        if (fabs(pa.d - pa.D) < P->eps_reach) amb |= ORC_AMB_REACH;
        if (type == ORC_CHIP && fabs(pa.d - pa.sf) < P->eps_reach) amb |= ORC_AMB_REACH;
    }
    /* a point at the ball cannot be passed to; beyond the stopping distance
     * (or, for a chip, short of the landing point) it is not reachable */
    int reachable = pa.d >= 1e-9 && pa.d <= pa.D && (type != ORC_CHIP || pa.d >= pa.sf);
    out->reachable = reachable;
    if (!reachable) {
        out->t_team = INFINITY;
        out->t_opp = INFINITY;
        out->margin = -INFINITY;
        out->score = -INFINITY;
        out->feasible = 0;
        out->ambig = amb;
        return;
    }
    double t_team = INFINITY, t_opp = INFINITY;
    int k_team = P->n_samples, k_opp = P->n_samples;
    for (int j = 0; j < W->n_team; ++j) {
        if (j == W->passer) continue;
        int kh;
        double tau = sbip_robot(P, &pa, W->team + 4 * j, &kh);
        if (tau < t_team) t_team = tau;
        if (kh < k_team) k_team = kh;
    }
    for (int j = 0; j < W->n_opp; ++j) {
        int kh;
        double tau = sbip_robot(P, &pa, W->opp + 4 * j, &kh);
        if (tau < t_opp) t_opp = tau;
        if (kh < k_opp) k_opp = kh;
    }
    double m;
    if (!isfinite(t_team)) m = -INFINITY;
    else if (!isfinite(t_opp)) m = INFINITY;
    else m = t_opp - t_team;
    int feasible = isfinite(t_team) && m >= P->margin_s;
    out->t_team = t_team;
    out->t_opp = t_opp;
    out->margin = m;
    out->feasible = feasible;
    if (feasible) {
        double gx = cx - P->goal_x, gy = cy;
        double dg = sqrt(gx * gx + gy * gy);
        double mc = m < 0.0 ? 0.0 : (m > P->margin_cap_s ? P->margin_cap_s : m);
        out->score = P->w_angle * out->open_angle / M_PI + P->w_dist * (1.0 - dg / P->dist_norm)
                   + P->w_margin * mc;
    } else {
        out->score = -INFINITY;
    }
    if (bands) {
        side_bands(P, &pa, W->team, W->n_team, W->passer, k_team, &amb);
        side_bands(P, &pa, W->opp, W->n_opp, -1, k_opp, &amb);
        if (isfinite(t_team) && isfinite(m) && fabs(m - P->margin_s) < P->eps_margin)
            amb |= ORC_AMB_MARGIN;
    }
    out->ambig = amb;
}

/* ------------------------------------------------------------------------ */
/* Lattice (reading): field-centred, endpoints included.  At spacing h the   */
/* lattice has Nx = round(L/h) + 1 by Ny = round(W/h) + 1 points and point   */
/* (I, J) sits at (h (I - (Nx-1)/2), h (J - (Ny-1)/2)).  A window (h, i0, j0,*/
/* nx, ny) holds the points I = i0 + i, J = j0 + j.                          */
/* ------------------------------------------------------------------------ */
void orc_point(const orc_params *P, double h, int I, int J, double *x, double *y)
{
    int Nx = (int)lround(P->field_len / h) + 1;
    int Ny = (int)lround(P->field_wid / h) + 1;
    *x = h * ((double)I - 0.5 * (double)(Nx - 1));
    *y = h * ((double)J - 0.5 * (double)(Ny - 1));
}

/* Whole frame.  Windows are (h, i0, j0, nx, ny) with h given as a double and
 * the integers in win_int[4*w ..].  Outputs are laid out window-major, then
 * variant-major, then row-major [ny][nx]; any output pointer may be NULL.
 * Returns the number of evaluations. */
int64_t orc_search(const orc_params *P, const orc_world *W,
                   int n_win, const double *win_h, const int32_t *win_int,
                   int n_var, const int32_t *var_type, const double *var_v0,
                   int bands,
                   uint8_t *mask, double *score, double *t_team, double *t_opp,
                   double *margin, uint8_t *ambig)
{
    int64_t base = 0;
    for (int w = 0; w < n_win; ++w) {
        double h = win_h[w];
        int i0 = win_int[4 * w], j0 = win_int[4 * w + 1];
        int nx = win_int[4 * w + 2], ny = win_int[4 * w + 3];
        int64_t npts = (int64_t)nx * ny;
#ifdef _OPENMP
        int nt = P->n_threads > 0 ? P->n_threads : omp_get_max_threads();
#pragma omp parallel for schedule(dynamic, 8) num_threads(nt)
#endif
        for (int64_t p = 0; p < npts; ++p) {
            int i = (int)(p % nx), j = (int)(p / nx);
            double cx, cy;
            orc_point(P, h, i0 + i, j0 + j, &cx, &cy);
            for (int v = 0; v < n_var; ++v) {
                orc_result r;
                orc_eval(P, W, var_type[v], var_v0[v], cx, cy, bands, &r);
                int64_t o = base + (int64_t)v * npts + p;
                if (mask) mask[o] = (uint8_t)r.feasible;
                if (score) score[o] = r.score;
                if (t_team) t_team[o] = r.t_team;
                if (t_opp) t_opp[o] = r.t_opp;
                if (margin) margin[o] = r.margin;
                if (ambig) ambig[o] = (uint8_t)r.ambig;
            }
        }
        base += npts * n_var;
    }
    return base;
}

/* A list of points given by coordinates; outputs are [point][variant]. */
void orc_search_points(const orc_params *P, const orc_world *W, int64_t n_pts, const double *xy,
                       int n_var, const int32_t *var_type, const double *var_v0, int bands,
                       uint8_t *mask, double *score, double *t_team, double *t_opp,
                       double *margin, uint8_t *ambig)
{
#ifdef _OPENMP
    int nt = P->n_threads > 0 ? P->n_threads : omp_get_max_threads();
#pragma omp parallel for schedule(dynamic, 4) num_threads(nt)
#endif
    for (int64_t p = 0; p < n_pts; ++p) {
        for (int v = 0; v < n_var; ++v) {
            orc_result r;
            orc_eval(P, W, var_type[v], var_v0[v], xy[2 * p], xy[2 * p + 1], bands, &r);
            int64_t o = p * n_var + v;
            if (mask) mask[o] = (uint8_t)r.feasible;
            if (score) score[o] = r.score;
            if (t_team) t_team[o] = r.t_team;
            if (t_opp) t_opp[o] = r.t_opp;
            if (margin) margin[o] = r.margin;
            if (ambig) ambig[o] = (uint8_t)r.ambig;
        }
    }
}

/* Best entry of a score array: largest score, ties to the lowest index.
 * Returns the index, or -1 when no entry is finite (no feasible pass). */
int64_t orc_argmax(int64_t n, const double *score)
{
    int64_t best = -1;
    double bs = -INFINITY;
    for (int64_t i = 0; i < n; ++i) {
        if (score[i] > bs) { bs = score[i]; best = i; }
    }
    return best;
}

/* ------------------------------------------------------------------------ */
/* The paper's own DPPS form (Sec. 4.2, Fig. "dynamic passing points         */
/* searching process"): from the passer's point of view, every kick          */
/* direction and every kick power.                                           */
/*                                                                           */
/* Readings (the paper gives the sweep sizes but not these details):         */
/*   - directions theta_d = 2 pi d / n_dirs from +x, counterclockwise;        */
/*   - the ball path runs along the direction from the ball until the ball    */
/*     stops (D of the power) or leaves the field; the K samples are uniform  */
/*     in distance over the part inside the field, s_k = (k+1) L / K, shared  */
/*     by all powers, and a power only uses the samples its ball reaches      */
/*     (s_k <= D; chips also only samples at or past the landing point);      */
/*   - SBIP per robot as above; the pass is received at the first teammate's  */
/*     interception (the passer excluded), which is the passing point;        */
/*   - feasible when a teammate intercepts and the first opponent comes at    */
/*     least margin_s later (or never);                                       */
/*   - score (Eq. 3 with the five features of Sec. 4.3): open goal angle at   */
/*     the passing point / pi, 1 - its distance to the goal centre /          */
/*     dist_norm, the margin clipped to [0, margin_cap_s], minus w_time times */
/*     the teammate's interception time (seconds, not normalised) and minus   */
/*     w_refract times the refraction angle / pi, the angle between the       */
/*     ball's direction and the shot from the passing point to the goal       */
/*     centre (0 when the ball already heads there);                          */
/*   - best: largest score, ties to the lowest (direction, variant) index.    */
/* ------------------------------------------------------------------------ */

typedef struct {
    int32_t n_dirs, pad;
    double w_time, w_refract;
} orc_ray_params;

typedef struct {
    int32_t feasible, k_team, k_opp, ambig;
    double t_team, t_opp, margin, score, s_recv, x, y, open_angle, refract, length;
} orc_ray_result;

/* Distance from (bx, by) along (ux, uy) to the edge of the field rectangle
 * (0 when the ball is on or outside the edge and the ray leaves). */
double orc_ray_length(const orc_params *P, double bx, double by, double ux, double uy)
{
    double hl = 0.5 * P->field_len, hw = 0.5 * P->field_wid;
    double L = INFINITY;
    if (ux > 0.0) L = fmin(L, (hl - bx) / ux);
    if (ux < 0.0) L = fmin(L, (-hl - bx) / ux);
    if (uy > 0.0) L = fmin(L, (hw - by) / uy);
    if (uy < 0.0) L = fmin(L, (-hw - by) / uy);
    return L > 0.0 ? L : 0.0;
}

/* First interception of one robot along the ray (sample index, or K). */
static int ray_sbip_robot(const orc_params *P, int type, double v0, double D, double sf,
                          double bx, double by, double ux, double uy, double L,
                          const double *rb)
{
    int K = P->n_samples;
    for (int k = 0; k < K; ++k) {
        double s = (double)(k + 1) / (double)K * L;
        if (s > D) break; /* the ball never gets there */
        if (type == ORC_CHIP && s < sf) continue; /* still in the air */
        double tb = orc_ball_time(P, type, v0, s);
        double tr = robot_time_to(P, rb, bx + s * ux, by + s * uy);
        if (tr <= tb) return k;
    }
    return K;
}

/* Bands of one side along the ray (parity tests only): at each sample the
 * ball reaches, up to the side's first interception, the side's earliest
 * arrival within eps_cross_t of the ball or the ball's position at that
 * arrival within eps_cross_s of the sample; a sample within eps_reach of the
 * stopping distance or within eps_land of a chip's landing point. */
static void ray_side_bands(const orc_params *P, int type, double v0, double D, double sf,
                           double bx, double by, double ux, double uy, double L,
                           const double *robots, int n, int skip, int k_side, int *amb)
{
    int K = P->n_samples;
    int klim = k_side < K ? k_side : K - 1;
    for (int k = 0; k <= klim; ++k) {
        double s = (double)(k + 1) / (double)K * L;
        if (fabs(s - D) < P->eps_reach) *amb |= ORC_AMB_REACH;
        if (s > D) break;
        double tmin = INFINITY;
        for (int j = 0; j < n; ++j) {
            if (j == skip) continue;
            double tr = robot_time_to(P, robots + 4 * j, bx + s * ux, by + s * uy);
            if (tr < tmin) tmin = tr;
        }
        if (!isfinite(tmin)) return;
        if (type == ORC_CHIP && fabs(s - sf) < P->eps_land) {
            double tb_land = s / (v0 * cos(P->chip_angle));
            if (tmin <= tb_land + P->eps_cross_t) *amb |= ORC_AMB_LAND;
        }
        if (type == ORC_CHIP && s < sf) continue;
        double tb = orc_ball_time(P, type, v0, s);
        if (fabs(tmin - tb) < P->eps_cross_t) *amb |= ORC_AMB_CROSS;
        double sb = orc_ball_dist(P, type, v0, tmin);
        if (fabs(sb - s) < P->eps_cross_s) *amb |= ORC_AMB_CROSS;
    }
}

void orc_ray_eval(const orc_params *P, const orc_ray_params *R, const orc_world *W, int dir,
                  int type, double v0, int bands, orc_ray_result *out)
{
    int K = P->n_samples;
    double th = 2.0 * M_PI * (double)dir / (double)R->n_dirs;
    double ux = cos(th), uy = sin(th);
    double bx = W->ball_x, by = W->ball_y;
    double L = orc_ray_length(P, bx, by, ux, uy);
    double D, sf;
    orc_ball_range(P, type, v0, &D, &sf);
    memset(out, 0, sizeof(*out));
    out->length = L;

    int k_team = K, k_opp = K;
    for (int j = 0; j < W->n_team; ++j) {
        if (j == W->passer) continue;
        int k = ray_sbip_robot(P, type, v0, D, sf, bx, by, ux, uy, L, W->team + 4 * j);
        if (k < k_team) k_team = k;
    }
    for (int j = 0; j < W->n_opp; ++j) {
        int k = ray_sbip_robot(P, type, v0, D, sf, bx, by, ux, uy, L, W->opp + 4 * j);
        if (k < k_opp) k_opp = k;
    }
    double s_team = (double)(k_team + 1) / (double)K * L;
    double s_opp = (double)(k_opp + 1) / (double)K * L;
    double t_team = k_team < K ? orc_ball_time(P, type, v0, s_team) : INFINITY;
    double t_opp = k_opp < K ? orc_ball_time(P, type, v0, s_opp) : INFINITY;
    double m;
    if (!isfinite(t_team)) m = -INFINITY;
    else if (!isfinite(t_opp)) m = INFINITY;
    else m = t_opp - t_team;
    int feasible = isfinite(t_team) && m >= P->margin_s;
    out->k_team = k_team;
    out->k_opp = k_opp;
    out->t_team = t_team;
    out->t_opp = t_opp;
    out->margin = m;
    out->feasible = feasible;
    out->s_recv = isfinite(t_team) ? s_team : INFINITY;
    out->score = -INFINITY;
    if (feasible) {
        double px = bx + s_team * ux, py = by + s_team * uy;
        double gx = P->goal_x - px, gy = -py;
        double dg = sqrt(gx * gx + gy * gy);
        double ang = orc_open_angle(P, px, py, W->n_opp, W->opp);
        double refr = dg > 0.0 ? atan2(fabs(ux * gy - uy * gx), ux * gx + uy * gy) : 0.0;
        double mc = m < 0.0 ? 0.0 : (m > P->margin_cap_s ? P->margin_cap_s : m);
        out->x = px;
        out->y = py;
        out->open_angle = ang;
        out->refract = refr;
        out->score = P->w_angle * ang / M_PI + P->w_dist * (1.0 - dg / P->dist_norm)
                   + P->w_margin * mc - R->w_time * t_team - R->w_refract * refr / M_PI;
    }
    int amb = 0;
    if (bands) {
        ray_side_bands(P, type, v0, D, sf, bx, by, ux, uy, L, W->team, W->n_team, W->passer,
                       k_team, &amb);
        ray_side_bands(P, type, v0, D, sf, bx, by, ux, uy, L, W->opp, W->n_opp, -1, k_opp,
                       &amb);
        if (isfinite(t_team) && isfinite(m) && fabs(m - P->margin_s) < P->eps_margin)
            amb |= ORC_AMB_MARGIN;
    }
    out->ambig = amb;
}

/* Every (direction, variant) of one frame, outputs [dir][variant]; any output
 * pointer may be NULL.  Returns the number of evaluations. */
int64_t orc_ray_search(const orc_params *P, const orc_ray_params *R, const orc_world *W,
                       int n_var, const int32_t *var_type, const double *var_v0, int bands,
                       uint8_t *mask, double *score, double *t_team, double *t_opp,
                       double *s_recv, uint8_t *ambig)
{
#ifdef _OPENMP
    int nt = P->n_threads > 0 ? P->n_threads : omp_get_max_threads();
#pragma omp parallel for schedule(dynamic, 1) num_threads(nt)
#endif
    for (int d = 0; d < R->n_dirs; ++d) {
        for (int v = 0; v < n_var; ++v) {
            orc_ray_result r;
            orc_ray_eval(P, R, W, d, var_type[v], var_v0[v], bands, &r);
            int64_t o = (int64_t)d * n_var + v;
            if (mask) mask[o] = (uint8_t)r.feasible;
            if (score) score[o] = r.score;
            if (t_team) t_team[o] = r.t_team;
            if (t_opp) t_opp[o] = r.t_opp;
            if (s_recv) s_recv[o] = r.s_recv;
            if (ambig) ambig[o] = (uint8_t)r.ambig;
        }
    }
    return (int64_t)R->n_dirs * n_var;
}

/* ------------------------------------------------------------------------ */
/* Passing power (Sec. 4.1, Eq. 1-2): the kick speed for a pass to point c.  */
/* Readings: the receiver B is the teammate (passer excluded) that reaches c */
/* first (arrival-time predictor above); the ball should arrive when B does  */
/* plus a buffer (0.3 s in the paper); Eq. 1, as the paper simplifies it,    */
/* ignores the sliding phase, so over distance d and time t at the rolling    */
/* deceleration a the speed after the slide is v1 = (d + a t^2 / 2) / t      */
/* while the ball still rolls at t (d >= a t^2 / 2); when t is longer than a  */
/* rolling ball can take, the slowest ball that still reaches c,             */
/* v1 = sqrt(2 a d); Eq. 2 gives the kick speed v0 = v1 / slide_ratio (the   */
/* ball slides down to 5/7 of v0); the result is clamped to the robots'      */
/* kick range [v_min, v_max].  Returns 0 when no teammate can receive.       */
/* ------------------------------------------------------------------------ */
double orc_power_speed(const orc_params *P, const orc_world *W, double cx, double cy,
                       double buffer_s, double v_min, double v_max, double *t_recv)
{
    double tb = INFINITY;
    for (int j = 0; j < W->n_team; ++j) {
        if (j == W->passer) continue;
        double t = robot_time_to(P, W->team + 4 * j, cx, cy);
        if (t < tb) tb = t;
    }
    if (t_recv) *t_recv = tb;
    if (!isfinite(tb)) return 0.0;
    double dx = cx - W->ball_x, dy = cy - W->ball_y;
    double d = sqrt(dx * dx + dy * dy);
    double t = tb + buffer_s;
    double a = P->roll_decel;
    double v1 = d >= 0.5 * a * t * t ? (d + 0.5 * a * t * t) / t : sqrt(2.0 * a * d);
    double v0 = v1 / P->slide_ratio;
    if (v0 < v_min) v0 = v_min;
    if (v0 > v_max) v0 = v_max;
    return v0;
}

/* Every point of the windows with one flat pass at the point's own power;
 * outputs as orc_search with one variant, plus the power per point. */
int64_t orc_power_search(const orc_params *P, const orc_world *W, int n_win, const double *win_h,
                         const int32_t *win_int, double buffer_s, double v_min, double v_max,
                         int bands, uint8_t *mask, double *score, double *t_team, double *t_opp,
                         double *v0_out, uint8_t *ambig)
{
    int64_t base = 0;
    for (int w = 0; w < n_win; ++w) {
        double h = win_h[w];
        int i0 = win_int[4 * w], j0 = win_int[4 * w + 1];
        int nx = win_int[4 * w + 2], ny = win_int[4 * w + 3];
        int64_t npts = (int64_t)nx * ny;
#ifdef _OPENMP
        int nt = P->n_threads > 0 ? P->n_threads : omp_get_max_threads();
#pragma omp parallel for schedule(dynamic, 8) num_threads(nt)
#endif
        for (int64_t p = 0; p < npts; ++p) {
            int i = (int)(p % nx), j = (int)(p / nx);
            double cx, cy;
            orc_point(P, h, i0 + i, j0 + j, &cx, &cy);
            double v0 = orc_power_speed(P, W, cx, cy, buffer_s, v_min, v_max, NULL);
            orc_result r;
            if (v0 > 0.0) {
                orc_eval(P, W, ORC_FLAT, v0, cx, cy, bands, &r);
            } else {
                memset(&r, 0, sizeof r);
                r.t_team = INFINITY;
                r.t_opp = INFINITY;
                r.score = -INFINITY;
            }
            int64_t o = base + p;
            if (mask) mask[o] = (uint8_t)r.feasible;
            if (score) score[o] = r.score;
            if (t_team) t_team[o] = r.t_team;
            if (t_opp) t_opp[o] = r.t_opp;
            if (v0_out) v0_out[o] = v0;
            if (ambig) ambig[o] = (uint8_t)r.ambig;
        }
        base += npts;
    }
    return base;
}

/* ------------------------------------------------------------------------ */
/* Shooting decision (Sec. 4.4): the shot-angle test fused with the         */
/* interception prediction along the shot.  Readings (the paper gives no    */
/* numbers or construction details):                                        */
/*  - the goal mouth as seen from the shooter c spans the directions         */
/*    [lo, hi] to the posts (depth to the goal line floored at goal_eps, as  */
/*    for the open angle); opponent discs of the robot radius in front of    */
/*    the goal line shadow directions, exactly as for the open goal angle;   */
/*    a shooter inside an opponent disc has no open direction;              */
/*  - the "valid angle" of a shot is the width of the widest open gap of    */
/*    the mouth, and the shot aims at that gap's centre (ties go to the gap  */
/*    with the lower angle); with no open direction the shot aims at the     */
/*    goal centre;                                                          */
/*  - the shot is a flat kick at v_shot along the aim to the goal line,     */
/*    sampled like a pass (K samples uniform in distance, the kick point     */
/*    excluded, the goal line included); an opponent intercepts at a sample  */
/*    it reaches no later than the ball (teammates never block a shot);      */
/*  - slack = the smallest (opponent arrival - ball time) over the samples  */
/*    the ball gets to, +inf with no opponents; the shot is intercepted      */
/*    exactly when slack <= 0;                                               */
/*  - shoot = (widest gap >= min_angle) and (the ball reaches the goal line) */
/*    and (slack > margin_s).                                                */
/* ------------------------------------------------------------------------ */
#define ORC_AMB_ANGLE 16  /* gap-width decision or aim within the angle band */

typedef struct {
    double v_shot, min_angle, margin_s, eps_angle, eps_aim;
} orc_shot_params;

typedef struct {
    int32_t shoot, reachable, ambig, n_gaps;
    double aim, gap, open_angle, length, t_goal, slack, slack_sens, second_gap, length_sens;
} orc_shot_result;

/* Open gaps of the goal mouth seen from c: fills starts/widths in
 * increasing angle (at most n_opp + 1 gaps) and returns their number; -1
 * when c lies inside an opponent disc.  Writes the mouth's ends. */
static int shot_gaps(const orc_params *P, const orc_world *W, double cx, double cy, double *lo,
                     double *hi, double *gs, double *gw)
{
    double dx = P->goal_x - cx;
    if (dx < P->goal_eps) dx = P->goal_eps;
    *lo = atan2(-0.5 * P->goal_width - cy, dx);
    *hi = atan2(0.5 * P->goal_width - cy, dx);
    double a[32], b[32];
    int n = 0;
    for (int o = 0; o < W->n_opp && o < 32; ++o) {
        const double *r = W->opp + 4 * o;
        if (r[0] >= P->goal_x) continue;
        double ox = r[0] - cx, oy = r[1] - cy;
        double rho = sqrt(ox * ox + oy * oy);
        if (rho <= P->robot_radius) return -1;
        double phi = atan2(oy, ox);
        double al = asin(P->robot_radius / rho);
        double s = fmax(phi - al, *lo), e = fmin(phi + al, *hi);
        if (e > s) { a[n] = s; b[n] = e; ++n; }
    }
    /* insertion sort by start */
    for (int i = 1; i < n; ++i) {
        double sa = a[i], sb = b[i];
        int j = i - 1;
        while (j >= 0 && a[j] > sa) { a[j + 1] = a[j]; b[j + 1] = b[j]; --j; }
        a[j + 1] = sa; b[j + 1] = sb;
    }
    /* walk the mouth from lo: a gap runs from the covered edge to the next
     * blocked start */
    int ng = 0;
    double edge = *lo;
    for (int i = 0; i < n; ++i) {
        if (a[i] > edge) { gs[ng] = edge; gw[ng] = a[i] - edge; ++ng; }
        if (b[i] > edge) edge = b[i];
    }
    if (*hi > edge) { gs[ng] = edge; gw[ng] = *hi - edge; ++ng; }
    return ng;
}

/* Along the shot from c in direction aim to the goal line: path length, ball
 * time at the goal line (inf when the ball stops short) and the slack. */
static void shot_path(const orc_params *P, const orc_world *W, double cx, double cy, double aim,
                      double v_shot, double *L_out, double *t_goal, double *slack)
{
    double dx = P->goal_x - cx;
    if (dx < P->goal_eps) dx = P->goal_eps;
    double ux = cos(aim), uy = sin(aim);
    double L = dx / ux;
    double D, sf;
    orc_ball_range(P, ORC_FLAT, v_shot, &D, &sf);
    *L_out = L;
    *t_goal = L <= D ? orc_ball_time(P, ORC_FLAT, v_shot, L) : INFINITY;
    double m = INFINITY;
    int K = P->n_samples;
    for (int k = 0; k < K; ++k) {
        double s = (double)(k + 1) / (double)K * L;
        if (s > D) break;
        double tb = orc_ball_time(P, ORC_FLAT, v_shot, s);
        double px = cx + s * ux, py = cy + s * uy;
        for (int o = 0; o < W->n_opp; ++o) {
            double tr = robot_time_to(P, W->opp + 4 * o, px, py);
            if (tr - tb < m) m = tr - tb;
        }
    }
    *slack = m;
}

void orc_shot(const orc_params *P, const orc_shot_params *S, const orc_world *W, double cx,
              double cy, int bands, orc_shot_result *out)
{
    double lo, hi, gs[40], gw[40];
    int ng = shot_gaps(P, W, cx, cy, &lo, &hi, gs, gw);
    double best = 0.0, start = 0.0, second = 0.0, total = 0.0;
    int have = 0;
    for (int g = 0; g < ng; ++g) {
        total += gw[g];
        if (!have || gw[g] > best) {
            if (have) second = fmax(second, best);
            best = gw[g]; start = gs[g]; have = 1;
        } else {
            second = fmax(second, gw[g]);
        }
    }
    double dx = P->goal_x - cx;
    if (dx < P->goal_eps) dx = P->goal_eps;
    double aim = best > 0.0 ? start + 0.5 * best : atan2(-cy, dx);
    memset(out, 0, sizeof *out);
    out->n_gaps = ng < 0 ? 0 : ng;
    out->gap = best;
    out->second_gap = second;
    out->open_angle = total;
    out->aim = aim;
    shot_path(P, W, cx, cy, aim, S->v_shot, &out->length, &out->t_goal, &out->slack);
    double D, sf;
    orc_ball_range(P, ORC_FLAT, S->v_shot, &D, &sf);
    out->reachable = out->length <= D;
    out->shoot = best >= S->min_angle && out->reachable && out->slack > S->margin_s;
    if (!bands) return;
    int amb = 0;
    if (fabs(best - S->min_angle) < S->eps_angle) amb |= ORC_AMB_ANGLE;  /* decision */
    if (have && best - second < S->eps_angle) amb |= ORC_AMB_ANGLE;      /* which gap */
    if (best > 0.0 && best < S->eps_angle) amb |= ORC_AMB_ANGLE;         /* aim rule */
    for (int o = 0; o < W->n_opp; ++o) {                                  /* inside rule */
        const double *r = W->opp + 4 * o;
        double rho = hypot(r[0] - cx, r[1] - cy);
        if (r[0] < P->goal_x && fabs(rho - P->robot_radius) < P->eps_reach) amb |= ORC_AMB_ANGLE;
    }
    /* how much the slack and the path length move when the aim moves by
     * eps_aim (the float32 rounding of the aim on the device is well inside
     * it); a shooter on the goal line aims almost along it, where the length
     * is ill-conditioned */
    double sens = 0.0, lsens = 0.0;
    for (int sgn = -1; sgn <= 1; sgn += 2) {
        double L2, tg2, s2;
        shot_path(P, W, cx, cy, aim + sgn * S->eps_aim, S->v_shot, &L2, &tg2, &s2);
        double dsl = isinf(s2) && isinf(out->slack) ? 0.0 : fabs(s2 - out->slack);
        if (!(dsl <= sens)) sens = dsl;
        if (!(fabs(L2 - out->length) <= lsens)) lsens = fabs(L2 - out->length);
    }
    out->slack_sens = sens;
    out->length_sens = lsens;
    if (fabs(out->length - D) < P->eps_reach + lsens) amb |= ORC_AMB_REACH;
    if (fabs(out->slack - S->margin_s) < P->eps_cross_t + sens) amb |= ORC_AMB_MARGIN;
    out->ambig = amb;
}

/* The shot decision from every point of the windows (the ball placed there,
 * everything else unchanged). */
int64_t orc_shot_search(const orc_params *P, const orc_shot_params *S, const orc_world *W,
                        int n_win, const double *win_h, const int32_t *win_int, int bands,
                        orc_shot_result *res)
{
    int64_t base = 0;
    for (int w = 0; w < n_win; ++w) {
        double h = win_h[w];
        int i0 = win_int[4 * w], j0 = win_int[4 * w + 1];
        int nx = win_int[4 * w + 2], ny = win_int[4 * w + 3];
        int64_t npts = (int64_t)nx * ny;
#ifdef _OPENMP
        int nt = P->n_threads > 0 ? P->n_threads : omp_get_max_threads();
#pragma omp parallel for schedule(dynamic, 8) num_threads(nt)
#endif
        for (int64_t p = 0; p < npts; ++p) {
            int i = (int)(p % nx), j = (int)(p / nx);
            double cx, cy;
            orc_point(P, h, i0 + i, j0 + j, &cx, &cy);
            orc_shot(P, S, W, cx, cy, bands, res + base + p);
        }
        base += npts;
    }
    return base;
}

/* ------------------------------------------------------------------------ */
/* Running points (Sec. 5.2): every vertex of a zone raster is scored by the */
/* weighted sum of Eq. (4) over five criteria, each mapped to [0, 1] with    */
/* higher better.  Readings (the paper names the criteria but gives no       */
/* formulas, constants or weights; every constant is a parameter):           */
/*  x1 distance to the goal: 1 - |c - goal centre| / dist_norm;              */
/*  x2 distance to the ball: min(|c - ball| / ball_norm, 1) (too close to    */
/*     the ball is bad);                                                     */
/*  x3 angle to the goal: phi = |bearing of the goal centre from c| (0 when  */
/*     it lies straight along +x); 1 inside [ang_lo, ang_hi], falling        */
/*     linearly to 0 over ang_fall outside it;                               */
/*  x4 guard time: the segments from c to the two goal posts first meet the  */
/*     defense area (the rectangle of def_depth x def_width in front of the  */
/*     goal) at P and Q; each is reached first by some opponent after t_P,   */
/*     t_Q (the robot arrival model of the pass search); x4 = min((t_P +     */
/*     t_Q) / guard_norm, 1);                                                */
/*  x5 avoiding the defense: an opponent o nearer to the ball than c is      */
/*     (|o - ball| < |c - ball|, decided in FP64) marks c with weight        */
/*     max(0, 1 - |o - c| / mark_radius); x5 = 1 - the largest such weight;  */
/*  points strictly inside the defense area cannot be used (score -inf);     */
/*  the best point of a zone has the largest score, ties to the lowest       */
/*  row-major index.                                                         */
/* ------------------------------------------------------------------------ */
typedef struct {
    double w_goal, w_ball, w_angle, w_guard, w_defense;
    double ball_norm, ang_lo, ang_hi, ang_fall, guard_norm, def_depth, def_width, mark_radius;
} orc_run_params;

typedef struct {
    int32_t valid, ambig;
    double score, goal, ball, angle, guard, defense, px, py, qx, qy, t_p, t_q;
} orc_run_result;

#define ORC_AMB_RUN 32 /* an opponent within 1e-9 m of the ball-distance tie */

/* First point of the segment from (cx, cy) to (ex, ey) inside the closed
 * rectangle [x0, x1] x [y0, y1], by intersecting the segment with each edge
 * line and keeping the nearest crossing that lies on the edge (the end point
 * is inside by construction). */
static void seg_enter_rect(double cx, double cy, double ex, double ey, double x0, double x1,
                           double y0, double y1, double *px, double *py)
{
    if (cx >= x0 && cx <= x1 && cy >= y0 && cy <= y1) {  /* already on or in it */
        *px = cx;
        *py = cy;
        return;
    }
    double best = 1.0;
    double dx = ex - cx, dy = ey - cy;
    const double xs[2] = {x0, x1}, ys[2] = {y0, y1};
    for (int i = 0; i < 2; ++i) {
        if (dx != 0.0) {
            double t = (xs[i] - cx) / dx;
            double y = cy + t * dy;
            if (t >= 0.0 && t <= best && y >= y0 && y <= y1) best = t;
        }
        if (dy != 0.0) {
            double t = (ys[i] - cy) / dy;
            double x = cx + t * dx;
            if (t >= 0.0 && t <= best && x >= x0 && x <= x1) best = t;
        }
    }
    *px = cx + best * dx;
    *py = cy + best * dy;
}

void orc_run(const orc_params *P, const orc_run_params *R, const orc_world *W, double cx,
             double cy, orc_run_result *out)
{
    memset(out, 0, sizeof *out);
    double x0 = P->goal_x - R->def_depth, x1 = P->goal_x;
    double y0 = -0.5 * R->def_width, y1 = 0.5 * R->def_width;
    if (cx > x0 && cx < x1 && cy > y0 && cy < y1) {
        out->score = -INFINITY;
        return;
    }
    out->valid = 1;
    double gx = P->goal_x - cx, gy = -cy;
    out->goal = 1.0 - sqrt(gx * gx + gy * gy) / P->dist_norm;
    double bx = cx - W->ball_x, by = cy - W->ball_y;
    double db2 = bx * bx + by * by;
    out->ball = fmin(sqrt(db2) / R->ball_norm, 1.0);
    double phi = fabs(atan2(gy, gx));
    double off = phi < R->ang_lo ? R->ang_lo - phi : (phi > R->ang_hi ? phi - R->ang_hi : 0.0);
    out->angle = fmax(0.0, 1.0 - off / R->ang_fall);
    double hw = 0.5 * P->goal_width;
    seg_enter_rect(cx, cy, P->goal_x, hw, x0, x1, y0, y1, &out->px, &out->py);
    seg_enter_rect(cx, cy, P->goal_x, -hw, x0, x1, y0, y1, &out->qx, &out->qy);
    double tp = INFINITY, tq = INFINITY;
    double mark = 0.0;
    int amb = 0;
    for (int o = 0; o < W->n_opp; ++o) {
        const double *r = W->opp + 4 * o;
        double a = robot_time_to(P, r, out->px, out->py);
        double b = robot_time_to(P, r, out->qx, out->qy);
        if (a < tp) tp = a;
        if (b < tq) tq = b;
        double ox = r[0] - W->ball_x, oy = r[1] - W->ball_y;
        double do2 = ox * ox + oy * oy;
        double dc = hypot(r[0] - cx, r[1] - cy);
        double wgt = fmax(0.0, 1.0 - dc / R->mark_radius);
        if (do2 < db2 && wgt > mark) mark = wgt;
        if (fabs(do2 - db2) < 1e-9 && wgt > 0.0) amb |= ORC_AMB_RUN;
    }
    out->t_p = tp;
    out->t_q = tq;
    out->guard = isfinite(tp + tq) ? fmin((tp + tq) / R->guard_norm, 1.0) : 1.0;
    out->defense = 1.0 - mark;
    out->ambig = amb;
    out->score = R->w_goal * out->goal + R->w_ball * out->ball + R->w_angle * out->angle
               + R->w_guard * out->guard + R->w_defense * out->defense;
}

/* Every point of the windows (the zones); res in window-major, row-major
 * order; best[w] = index within window w of its best point, or -1. */
int64_t orc_run_search(const orc_params *P, const orc_run_params *R, const orc_world *W,
                       int n_win, const double *win_h, const int32_t *win_int,
                       orc_run_result *res, int64_t *best)
{
    int64_t base = 0;
    for (int w = 0; w < n_win; ++w) {
        double h = win_h[w];
        int i0 = win_int[4 * w], j0 = win_int[4 * w + 1];
        int nx = win_int[4 * w + 2], ny = win_int[4 * w + 3];
        int64_t npts = (int64_t)nx * ny;
        int64_t bi = -1;
        double bs = -INFINITY;
        for (int64_t p = 0; p < npts; ++p) {
            int i = (int)(p % nx), j = (int)(p / nx);
            double cx, cy;
            orc_point(P, h, i0 + i, j0 + j, &cx, &cy);
            orc_run(P, R, W, cx, cy, res + base + p);
            if (res[base + p].valid && res[base + p].score > bs) {
                bs = res[base + p].score;
                bi = p;
            }
        }
        best[w] = bi;
        base += npts;
    }
    return base;
}

int orc_abi_version(void) { return 5; }
