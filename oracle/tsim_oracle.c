/*
 * tsim_oracle.c -- plain, slow, single-threaded FP64 reference of the
 * per-timestep microscopic vehicle update of arXiv 2406.10661
 * ("A GPU-accelerated Large-scale Simulator for Transportation System
 * Optimization Benchmarking").
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path may load, call or
 * link this file; only the tests, the smoke check and the CPU-baseline leg of
 * the benchmark do.  It shares no code, header, table or helper with the HIP
 * library: it reads the same plain input arrays and is written from the paper
 * alone, with every neighbour query done by brute force over a lane.
 *
 * What one step computes (Section 3.1 two-phase process, Appendix B.2
 * execution process, Appendix B.3 vehicle models):
 *   prepare  P1 signal state of every junction lane (Section 3.2 policies)
 *            P2 departures into lanes of the origin road when it is safe
 *            P3 per-lane order of active vehicles (x descending, id ascending)
 *   update   every active vehicle reads only the snapshot S of the step start:
 *            U1 IDM car following (Appendix B.3 IDM equations, delta = 4)
 *            U2 MOBIL utilities left/right (Appendix B.3 MOBIL utility)
 *            U3 randomized decision (Appendix B.3 u_T and p_LC)
 *            U4 ballistic integration with snapshot bounds
 *            U5 lane-end transfer, feeder priority, trip completion
 *            U6 metrics (Section 3.3)
 *   commit   state <- next state, t <- t + 1
 * Between steps: routes of least cost under road prices (Section 4
 * congestion pricing), computed in FP32 (osim_shortest_routes).
 * Readings of points the paper leaves open are listed next to the code that
 * implements them (tagged [reading]).
 *
 * Parity pins: IDM closed forms, Philox against rocRAND's host engine,
 * brute-force MOBIL scenes, ring-road equilibrium, red-light stop, the
 * per-step invariants (no overlap, v >= 0, conservation, per-lane order,
 * no entry on red, lane group kept, no lane change on junction lanes), and
 * hand-derived tiny scenes for the departure rules (most room, room >= s0,
 * tau <= t dt, one per lane, blocked head, feeder reach), merge priority,
 * travelling time, mean speed and its horizon average, lane queue length
 * and cooperative yielding, lane restrictions (departures, lane changes,
 * closed junction lanes and the lane group they leave), trip end and start
 * positions (departures from an AOI's connection partway along a lane),
 * each shown to fail under a named mistake; shortest routes against
 * hand-derived routes, brute force over every simple route of small
 * networks with exact costs, and scipy's Dijkstra on a grid.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

enum { WAITING = 0, ACTIVE = 1, FINISHED = 2 };
enum { POL_NONE = 0, POL_FIXED = 1, POL_MANUAL = 2, POL_MAX_PRESSURE = 3 };
enum { EV_TRANSFER = 1, EV_FINISH = 2, EV_FEEDER_BLOCK = 4, EV_CLAMP = 8, EV_DEPART = 16 };

#define NMARGIN 6
#define NMETRIC 16

typedef struct {
    double dt, T, a_max, b_comf, s0, delta, p, a_th, b_safe, p_max, p_min, a_emerg;
    uint64_t seed;
} oparams;

typedef struct {
    int exists;
    double rear; /* leader's rear bumper, in the follower's lane coordinate */
    double v;
} olead;

typedef struct osim {
    oparams P;
    /* network */
    int NJ, R, NRL, NJL, NL;
    int *road_from, *road_to, *road_lane_begin;
    int *lane_road;            /* [NRL] */
    double *lane_len, *lane_lim; /* [NL] */
    unsigned char *restricted;   /* [NL] set_lane_restriction: the lane admits no new vehicle */
    int *jl_in, *jl_out;       /* [NJL] road-lane ids */
    int *jl_junction;          /* [NJL] */
    int *junc_phase_begin, *phase_green_begin, *phase_green_jl;
    double *phase_dur;
    int *policy, *manual_phase;  /* [NJ]; manual_phase is also the phase in force of a MAX_PRESSURE junction */
    int *out_begin, *out_jl;     /* [NRL+1], junction lanes leaving a road lane (global ids) */
    int *feed_begin, *feed_jl;   /* [NRL+1], junction lanes entering a road lane, ascending */
    /* trips */
    int N;
    double *tau, *f, *L;
    int *route_begin, *route;    /* CSR of the routes given at creation */
    int *rstart, *rlen;          /* [N] the route in force: route[rstart, rstart + rlen) */
    double *end_s;               /* [N] trip end position on the last road, < 0: the road's end */
    double *start_s;             /* [N] trip start position on the origin road, <= 0: the road's start */
    long route_n, route_cap;     /* route entries used / allocated (set_vehicle_route appends) */
    int *q_begin, *q_veh;        /* [R+1] departure queue of each origin road, (tau, id) order */
    /* state */
    int64_t t;
    int *status, *lane, *k, *finish_step;
    double *x, *v;
    /* next state */
    int *n_status, *n_lane, *n_k;
    double *n_x, *n_v;
    /* per-step index: lanes front first */
    int *sorted, *lane_start, *lane_cnt;
    unsigned char *green;        /* [NJL] */
    /* metrics */
    double sum_tt, vehicle_steps, speed_acc, speed_steps, mean_speed_last;
    double n_lane_changes, n_transfers, n_clamps, n_feeder_blocks, n_departures, n_finished;
    double *road_sumv;           /* [R] last step */
    int *road_cnt;               /* [R] */
    int *lane_wait;              /* [NL] */
    double *vend;                /* [N] end-of-step speed of the last step (active vehicles) */
    /* diagnostics of the last step */
    double *margin;              /* [N * NMARGIN] */
    double *mobil;               /* [N * 4]: u_L, u_R, u_T, p_LC */
    int *decision;               /* [N]: 0 keep, 1 left, 2 right */
    int *event;                  /* [N]: EV_* bits */
} osim;

/* ------------------------------------------------------------------------ */
/* Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11): ten rounds of the     */
/* multiply-xor round function with a Weyl key schedule.                    */
/* ------------------------------------------------------------------------ */
static void philox4x32_10(uint32_t k0, uint32_t k1, const uint32_t in[4], uint32_t out[4])
{
    uint32_t c0 = in[0], c1 = in[1], c2 = in[2], c3 = in[3];
    for (int round = 0; round < 10; ++round) {
        if (round > 0) {
            k0 += 0x9E3779B9u;
            k1 += 0xBB67AE85u;
        }
        uint64_t p0 = (uint64_t)0xD2511F53u * (uint64_t)c0;
        uint64_t p1 = (uint64_t)0xCD9E8D57u * (uint64_t)c2;
        uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
        uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
        uint32_t n0 = hi1 ^ c1 ^ k0;
        uint32_t n1 = lo1;
        uint32_t n2 = hi0 ^ c3 ^ k1;
        uint32_t n3 = lo0;
        c0 = n0; c1 = n1; c2 = n2; c3 = n3;
    }
    out[0] = c0; out[1] = c1; out[2] = c2; out[3] = c3;
}

void osim_philox(uint64_t seed, const uint32_t ctr[4], uint32_t out[4])
{
    philox4x32_10((uint32_t)seed, (uint32_t)(seed >> 32), ctr, out);
}

/* ------------------------------------------------------------------------ */
/* IDM (Appendix B.3):                                                       */
/*   a = a_max [1 - (v/v0)^delta - (s_star/s)^2]                             */
/*   s_star = s0 + max(0, v T + v dv / (2 sqrt(a_max a_comf)))               */
/* [reading] s is the bumper-to-bumper gap; dv = v - v_leader; s = +inf is   */
/* the free road; s <= 0 gives -inf, and every use floors the result at      */
/* -a_emerg.                                                                 */
/* ------------------------------------------------------------------------ */
static double idm_raw(const oparams *P, double v, double v0, double s, double dv)
{
    double free_term = 1.0 - pow(v / v0, P->delta);
    if (isinf(s) && s > 0) return P->a_max * free_term;
    if (s <= 0.0) return -INFINITY;
    double s_star = P->s0 + fmax(0.0, v * P->T + v * dv / (2.0 * sqrt(P->a_max * P->b_comf)));
    double ratio = s_star / s;
    return P->a_max * (free_term - ratio * ratio);
}

static double idm_acc(const oparams *P, double v, double v0, double s, double dv)
{
    return fmax(idm_raw(P, v, v0, s, dv), -P->a_emerg);
}

static void params_from(oparams *P, const double *pp, uint64_t seed)
{
    P->dt = pp[0]; P->T = pp[1]; P->a_max = pp[2]; P->b_comf = pp[3]; P->s0 = pp[4];
    P->delta = pp[5]; P->p = pp[6]; P->a_th = pp[7]; P->b_safe = pp[8]; P->p_max = pp[9];
    P->p_min = pp[10]; P->a_emerg = pp[11]; P->seed = seed;
}

double osim_idm(const double *params, double v, double v0, double s, double dv)
{
    oparams P;
    params_from(&P, params, 0);
    return idm_raw(&P, v, v0, s, dv);
}

/* ------------------------------------------------------------------------ */
/* construction                                                              */
/* ------------------------------------------------------------------------ */
static void *xcalloc(size_t n, size_t sz) { return calloc(n ? n : 1, sz); }

static const double *g_sort_tau;
static int cmp_queue(const void *a, const void *b)
{
    int i = *(const int *)a, j = *(const int *)b;
    if (g_sort_tau[i] < g_sort_tau[j]) return -1;
    if (g_sort_tau[i] > g_sort_tau[j]) return 1;
    return (i > j) - (i < j);
}

osim *osim_create(int NJ, int R, const int *road_from, const int *road_to, const int *road_lane_begin,
                  const float *road_length, const float *road_limit,
                  int NJL, const int *jl_in, const int *jl_out, const float *jl_length, const float *jl_limit,
                  const int *junc_phase_begin, const float *phase_duration,
                  const int *phase_green_begin, const int *phase_green_jl, const int *junc_policy,
                  int N, const float *depart, const int *route_begin, const int *route_roads,
                  const float *v0_factor, const float *veh_length,
                  const double *params, uint64_t seed)
{
    osim *s = (osim *)xcalloc(1, sizeof(osim));
    params_from(&s->P, params, seed);
    s->NJ = NJ; s->R = R; s->NRL = road_lane_begin[R]; s->NJL = NJL; s->NL = s->NRL + NJL;
    int NRL = s->NRL, NL = s->NL;
    s->road_from = (int *)xcalloc(R, sizeof(int));
    s->road_to = (int *)xcalloc(R, sizeof(int));
    s->road_lane_begin = (int *)xcalloc(R + 1, sizeof(int));
    memcpy(s->road_from, road_from, R * sizeof(int));
    memcpy(s->road_to, road_to, R * sizeof(int));
    memcpy(s->road_lane_begin, road_lane_begin, (R + 1) * sizeof(int));
    s->lane_road = (int *)xcalloc(NRL, sizeof(int));
    s->lane_len = (double *)xcalloc(NL, sizeof(double));
    s->lane_lim = (double *)xcalloc(NL, sizeof(double));
    s->restricted = (unsigned char *)xcalloc(NL, 1);
    for (int r = 0; r < R; ++r)
        for (int l = road_lane_begin[r]; l < road_lane_begin[r + 1]; ++l) {
            s->lane_road[l] = r;
            s->lane_len[l] = road_length[r];
            s->lane_lim[l] = road_limit[r];
        }
    s->jl_in = (int *)xcalloc(NJL, sizeof(int));
    s->jl_out = (int *)xcalloc(NJL, sizeof(int));
    s->jl_junction = (int *)xcalloc(NJL, sizeof(int));
    for (int q = 0; q < NJL; ++q) {
        s->jl_in[q] = jl_in[q];
        s->jl_out[q] = jl_out[q];
        s->jl_junction[q] = road_to[s->lane_road[jl_in[q]]];
        s->lane_len[NRL + q] = jl_length[q];
        s->lane_lim[NRL + q] = jl_limit[q];
    }
    int NP = junc_phase_begin[NJ];
    s->junc_phase_begin = (int *)xcalloc(NJ + 1, sizeof(int));
    memcpy(s->junc_phase_begin, junc_phase_begin, (NJ + 1) * sizeof(int));
    s->phase_dur = (double *)xcalloc(NP, sizeof(double));
    for (int p = 0; p < NP; ++p) s->phase_dur[p] = phase_duration[p];
    s->phase_green_begin = (int *)xcalloc(NP + 1, sizeof(int));
    memcpy(s->phase_green_begin, phase_green_begin, (NP + 1) * sizeof(int));
    int NG = phase_green_begin[NP];
    s->phase_green_jl = (int *)xcalloc(NG, sizeof(int));
    memcpy(s->phase_green_jl, phase_green_jl, NG * sizeof(int));
    s->policy = (int *)xcalloc(NJ, sizeof(int));
    s->manual_phase = (int *)xcalloc(NJ, sizeof(int));
    memcpy(s->policy, junc_policy, NJ * sizeof(int));

    /* junction lanes leaving / entering each road lane (CSR, ascending id) */
    s->out_begin = (int *)xcalloc(NRL + 1, sizeof(int));
    s->feed_begin = (int *)xcalloc(NRL + 1, sizeof(int));
    for (int q = 0; q < NJL; ++q) { s->out_begin[jl_in[q] + 1]++; s->feed_begin[jl_out[q] + 1]++; }
    for (int l = 0; l < NRL; ++l) { s->out_begin[l + 1] += s->out_begin[l]; s->feed_begin[l + 1] += s->feed_begin[l]; }
    s->out_jl = (int *)xcalloc(NJL, sizeof(int));
    s->feed_jl = (int *)xcalloc(NJL, sizeof(int));
    int *fo = (int *)xcalloc(NRL, sizeof(int)), *ff = (int *)xcalloc(NRL, sizeof(int));
    for (int q = 0; q < NJL; ++q) {
        s->out_jl[s->out_begin[jl_in[q]] + fo[jl_in[q]]++] = NRL + q;
        s->feed_jl[s->feed_begin[jl_out[q]] + ff[jl_out[q]]++] = NRL + q;
    }
    free(fo); free(ff);

    /* trips */
    s->N = N;
    s->tau = (double *)xcalloc(N, sizeof(double));
    s->end_s = (double *)xcalloc(N, sizeof(double));
    for (int i = 0; i < N; ++i) s->end_s[i] = -1.0;
    s->start_s = (double *)xcalloc(N, sizeof(double));
    s->f = (double *)xcalloc(N, sizeof(double));
    s->L = (double *)xcalloc(N, sizeof(double));
    s->route_begin = (int *)xcalloc(N + 1, sizeof(int));
    memcpy(s->route_begin, route_begin, (N + 1) * sizeof(int));
    s->route_cap = route_begin[N] > 0 ? route_begin[N] : 1;
    s->route_n = route_begin[N];
    s->route = (int *)xcalloc(s->route_cap, sizeof(int));
    memcpy(s->route, route_roads, (size_t)route_begin[N] * sizeof(int));
    s->rstart = (int *)xcalloc(N, sizeof(int));
    s->rlen = (int *)xcalloc(N, sizeof(int));
    for (int i = 0; i < N; ++i) { s->rstart[i] = route_begin[i]; s->rlen[i] = route_begin[i + 1] - route_begin[i]; }
    for (int i = 0; i < N; ++i) { s->tau[i] = depart[i]; s->f[i] = v0_factor[i]; s->L[i] = veh_length[i]; }
    s->q_begin = (int *)xcalloc(R + 1, sizeof(int));
    s->q_veh = (int *)xcalloc(N, sizeof(int));
    for (int i = 0; i < N; ++i) s->q_begin[s->route[s->route_begin[i]] + 1]++;
    for (int r = 0; r < R; ++r) s->q_begin[r + 1] += s->q_begin[r];
    int *fill = (int *)xcalloc(R, sizeof(int));
    for (int i = 0; i < N; ++i) { int r = s->route[s->route_begin[i]]; s->q_veh[s->q_begin[r] + fill[r]++] = i; }
    free(fill);
    g_sort_tau = s->tau;
    for (int r = 0; r < R; ++r)
        qsort(s->q_veh + s->q_begin[r], s->q_begin[r + 1] - s->q_begin[r], sizeof(int), cmp_queue);

    s->status = (int *)xcalloc(N, sizeof(int));
    s->lane = (int *)xcalloc(N, sizeof(int));
    s->k = (int *)xcalloc(N, sizeof(int));
    s->finish_step = (int *)xcalloc(N, sizeof(int));
    s->x = (double *)xcalloc(N, sizeof(double));
    s->v = (double *)xcalloc(N, sizeof(double));
    s->n_status = (int *)xcalloc(N, sizeof(int));
    s->n_lane = (int *)xcalloc(N, sizeof(int));
    s->n_k = (int *)xcalloc(N, sizeof(int));
    s->n_x = (double *)xcalloc(N, sizeof(double));
    s->n_v = (double *)xcalloc(N, sizeof(double));
    for (int i = 0; i < N; ++i) { s->lane[i] = -1; s->finish_step[i] = -1; }
    s->sorted = (int *)xcalloc(N, sizeof(int));
    s->lane_start = (int *)xcalloc(NL + 1, sizeof(int));
    s->lane_cnt = (int *)xcalloc(NL, sizeof(int));
    s->green = (unsigned char *)xcalloc(NJL, 1);
    s->road_sumv = (double *)xcalloc(R, sizeof(double));
    s->road_cnt = (int *)xcalloc(R, sizeof(int));
    s->lane_wait = (int *)xcalloc(NL, sizeof(int));
    s->vend = (double *)xcalloc(N, sizeof(double));
    s->margin = (double *)xcalloc((size_t)N * NMARGIN, sizeof(double));
    s->mobil = (double *)xcalloc((size_t)N * 4, sizeof(double));
    s->decision = (int *)xcalloc(N, sizeof(int));
    s->event = (int *)xcalloc(N, sizeof(int));
    return s;
}

void osim_destroy(osim *s)
{
    if (!s) return;
    void *ptrs[] = {s->road_from, s->road_to, s->road_lane_begin, s->lane_road, s->lane_len, s->lane_lim, s->restricted, s->end_s, s->start_s,
                    s->jl_in, s->jl_out, s->jl_junction, s->junc_phase_begin, s->phase_green_begin,
                    s->phase_green_jl, s->phase_dur, s->policy, s->manual_phase, s->out_begin, s->out_jl,
                    s->feed_begin, s->feed_jl, s->tau, s->f, s->L, s->route_begin, s->route, s->rstart, s->rlen, s->q_begin,
                    s->q_veh, s->status, s->lane, s->k, s->finish_step, s->x, s->v, s->n_status, s->n_lane,
                    s->n_k, s->n_x, s->n_v, s->sorted, s->lane_start, s->lane_cnt, s->green, s->road_sumv,
                    s->road_cnt, s->lane_wait, s->vend, s->margin, s->mobil, s->decision, s->event};
    for (size_t i = 0; i < sizeof(ptrs) / sizeof(ptrs[0]); ++i) free(ptrs[i]);
    free(s);
}

/* ------------------------------------------------------------------------ */
/* small queries                                                             */
/* ------------------------------------------------------------------------ */

/* [reading] "j ahead of i": larger front-bumper coordinate, ties broken by the
 * smaller vehicle id; a strict total order on the vehicles of one road. */
static int ahead(const osim *s, int a, int b)
{
    return s->x[a] > s->x[b] || (s->x[a] == s->x[b] && a < b);
}

static int route_len(const osim *s, int i) { return s->rlen[i]; }

static int next_road(const osim *s, int i)
{
    return (s->k[i] + 1 < route_len(s, i)) ? s->route[s->rstart[i] + s->k[i] + 1] : -1;
}

/* a junction lane takes new vehicles unless it or the road lane it leads
 * into is restricted (Section 3.2 "Lane" set_lane_restriction; [reading] a
 * restricted lane admits no new vehicle, those already on it, or on a
 * junction lane leading into it, carry on) */
static int jl_open(const osim *s, int g)
{
    return !s->restricted[g] && !s->restricted[s->jl_out[g - s->NRL]];
}

/* open junction lane (global id) from road lane l into road r2, or -1 */
static int jl_to_road(const osim *s, int l, int r2)
{
    for (int e = s->out_begin[l]; e < s->out_begin[l + 1]; ++e) {
        int g = s->out_jl[e];
        if (s->lane_road[s->jl_out[g - s->NRL]] == r2 && jl_open(s, g)) return g;
    }
    return -1;
}

/* lane group G_i on the current road: lanes with a connection to the next
 * road of the route; every lane when the route ends on this road
 * (Appendix B.3: no change away from the lanes that reach the next road). */
static int in_group(const osim *s, int i, int l)
{
    int nr = next_road(s, i);
    return nr < 0 || jl_to_road(s, l, nr) >= 0;
}

static int group_dist(const osim *s, int i, int l)
{
    int r = s->lane_road[l], best = 1 << 30;
    for (int m = s->road_lane_begin[r]; m < s->road_lane_begin[r + 1]; ++m)
        if (in_group(s, i, m)) {
            int d = abs(m - l);
            if (d < best) best = d;
        }
    return best;
}

/* successor lane sigma_i(l): on a road lane the junction lane toward the next
 * road of the route (if l is in the lane group), on a junction lane its out
 * lane, otherwise none */
static int sigma(const osim *s, int i, int l)
{
    if (l >= s->NRL) return s->jl_out[l - s->NRL];
    int nr = next_road(s, i);
    return nr < 0 ? -1 : jl_to_road(s, l, nr);
}

/* stop obstacle at the end of lane l (Appendix B.3 signal rule): the next lane
 * of the route is a red junction lane; [reading] or, with with_wrong_lane, l is
 * a road lane that has no connection to the next road of the route. */
static int stop_at_end(const osim *s, int i, int l, int with_wrong_lane)
{
    if (l >= s->NRL) return 0;
    int nr = next_road(s, i);
    if (nr < 0) return 0;
    int g = jl_to_road(s, l, nr);
    if (g < 0) return with_wrong_lane;
    return !s->green[g - s->NRL];
}

#define LANE(s, m) ((s)->sorted + (s)->lane_start[m])

static int lane_front(const osim *s, int m) { return s->lane_cnt[m] ? LANE(s, m)[0] : -1; }
static int lane_rear(const osim *s, int m) { return s->lane_cnt[m] ? LANE(s, m)[s->lane_cnt[m] - 1] : -1; }

/* rearmost vehicle of lane m that is ahead of vehicle j, with vehicle `skip`
 * taken out of m and vehicle `extra` put into m (either may be -1) */
static int rearmost_ahead(const osim *s, int m, int j, int skip, int extra)
{
    int best = -1;
    for (int c = 0; c < s->lane_cnt[m]; ++c) {
        int z = LANE(s, m)[c];
        if (z == skip || z == j) continue;
        if (ahead(s, z, j) && (best < 0 || ahead(s, best, z))) best = z;
    }
    if (extra >= 0 && extra != j && ahead(s, extra, j) && (best < 0 || ahead(s, best, extra))) best = extra;
    return best;
}

/* frontmost vehicle of lane m that is not ahead of vehicle j (j excluded) */
static int frontmost_behind(const osim *s, int m, int j, int skip)
{
    int best = -1;
    for (int c = 0; c < s->lane_cnt[m]; ++c) {
        int z = LANE(s, m)[c];
        if (z == skip || z == j) continue;
        if (!ahead(s, z, j) && (best < 0 || ahead(s, z, best))) best = z;
    }
    return best;
}

/* lane after sigma_j(m) = g1 along the route: a junction lane leads to its out
 * lane; a road lane of the next road leads to the junction lane toward the
 * road after it (if that lane connects) */
static int sigma2(const osim *s, int j, int g1)
{
    if (g1 >= s->NRL) return s->jl_out[g1 - s->NRL];
    int kk = s->k[j] + 2;
    if (kk >= route_len(s, j)) return -1;
    return jl_to_road(s, g1, s->route[s->rstart[j] + kk]);
}

/* leader of vehicle j if it drives in lane m: the rearmost vehicle of m ahead
 * of it, else (Appendix B.3: no front vehicle in the lane, use the first
 * vehicle of the next lane) the rearmost vehicle of the next lane
 * sigma_j(m); [reading] when that lane is empty too, the rearmost vehicle of
 * the lane after it; else free road */
static olead leader_in(const osim *s, int j, int m, int skip, int extra)
{
    olead ld = {0, INFINITY, 0.0};
    int z = rearmost_ahead(s, m, j, skip, extra);
    if (z >= 0) {
        ld.exists = 1; ld.rear = s->x[z] - s->L[z]; ld.v = s->v[z];
        return ld;
    }
    int g = sigma(s, j, m);
    if (g < 0) return ld;
    if (s->lane_cnt[g] > 0) {
        z = lane_rear(s, g);
        ld.exists = 1; ld.rear = s->lane_len[m] + s->x[z] - s->L[z]; ld.v = s->v[z];
        return ld;
    }
    int g2 = sigma2(s, j, g);
    if (g2 >= 0 && s->lane_cnt[g2] > 0) {
        z = lane_rear(s, g2);
        ld.exists = 1; ld.rear = s->lane_len[m] + s->lane_len[g] + s->x[z] - s->L[z]; ld.v = s->v[z];
    }
    return ld;
}

/* U1: acceleration of vehicle j in lane m behind leader ld, with or without
 * the stationary zero-length obstacle at the lane end */
static double accel_in(const osim *s, int j, int m, olead ld, int stop)
{
    const oparams *P = &s->P;
    double v0 = s->f[j] * s->lane_lim[m];
    double a = ld.exists ? idm_acc(P, s->v[j], v0, ld.rear - s->x[j], s->v[j] - ld.v)
                         : idm_acc(P, s->v[j], v0, INFINITY, 0.0);
    if (stop) a = fmin(a, idm_acc(P, s->v[j], v0, s->lane_len[m] - s->x[j], s->v[j]));
    return a;
}

static double own_accel(const osim *s, int j)
{
    int m = s->lane[j];
    return accel_in(s, j, m, leader_in(s, j, m, -1, -1), stop_at_end(s, j, m, 1));
}

/* [reading] merge target of vehicle m: when m is on a road lane that has no
 * connection to the next road of its route, the adjacent lane one step toward
 * the nearest lane of its lane group (ties to the left); otherwise -1 */
static int merge_target(const osim *s, int m)
{
    int l = s->lane[m];
    if (l >= s->NRL || in_group(s, m, l)) return -1;
    int r = s->lane_road[l], best = -1, bd = 1 << 30;
    for (int g = s->road_lane_begin[r]; g < s->road_lane_begin[r + 1]; ++g)
        if (in_group(s, m, g) && abs(g - l) < bd) { bd = abs(g - l); best = g; }
    if (best < 0) return -1;
    return best < l ? l - 1 : l + 1;
}

/* [reading] cooperative yielding: a vehicle that keeps road lane l treats as
 * a leader (IDM and position bound) the nearest vehicle on lane l-1 or l+1
 * of its road whose merge target is l and whose rear is ahead of its front
 * (smallest rear, ties to the lower id); returns -1 when there is none */
static int yield_leader(const osim *s, int i)
{
    int l = s->lane[i];
    if (l >= s->NRL) return -1;
    int r = s->lane_road[l];
    int best = -1;
    for (int d = -1; d <= 1; d += 2) {
        int m2 = l + d;
        if (m2 < s->road_lane_begin[r] || m2 >= s->road_lane_begin[r + 1]) continue;
        for (int c = 0; c < s->lane_cnt[m2]; ++c) {
            int m = LANE(s, m2)[c];
            if (!(s->x[m] - s->L[m] > s->x[i])) continue;
            if (merge_target(s, m) != l) continue;
            double rm = s->x[m] - s->L[m];
            if (best < 0 || rm < s->x[best] - s->L[best] || (rm == s->x[best] - s->L[best] && m < best)) best = m;
        }
    }
    return best;
}

/* ------------------------------------------------------------------------ */
/* P1 signals (Section 3.2 traffic-signal policies)                          */
/* ------------------------------------------------------------------------ */

static void build_index(osim *s);

/* MAX_PRESSURE (Section 3.2; the maximum-pressure algorithm of Varaiya 2013
 * that the paper cites; Appendix B.2: lane pressures in the prepare phase,
 * the junction's phase update from them) [reading]:
 *   - the pressure of a movement (a junction lane g from road lane in(g) to
 *     road lane out(g)) is n(in(g)) - n(out(g)), n(l) the number of vehicles
 *     on road lane l at the start of the step, before its departures;
 *   - the pressure of a phase is the sum over the movements it makes green;
 *   - the junction takes the phase of largest pressure, ties to the lowest
 *     phase index;
 *   - it decides only at the steps t in which a multiple of the duration of
 *     its first phase falls (floor(t dt / d0) > floor((t - 1) dt / d0), so
 *     at t = 0 and then every d0 seconds) and holds the phase in between. */
static int max_pressure_decides(const osim *s, int j)
{
    double d0 = s->phase_dur[s->junc_phase_begin[j]];
    if (!(d0 > 0.0)) return 1;
    return floor((double)s->t * s->P.dt / d0) > floor((double)(s->t - 1) * s->P.dt / d0);
}

static int max_pressure_phase(const osim *s, int j)
{
    int b = s->junc_phase_begin[j], e = s->junc_phase_begin[j + 1];
    int best = 0;
    long best_p = 0;
    for (int p = b; p < e; ++p) {
        long pr = 0;
        for (int k = s->phase_green_begin[p]; k < s->phase_green_begin[p + 1]; ++k) {
            int g = s->phase_green_jl[k];
            pr += (long)s->lane_cnt[s->jl_in[g]] - (long)s->lane_cnt[s->jl_out[g]];
        }
        if (p == b || pr > best_p) { best_p = pr; best = p - b; }
    }
    return best;
}

/* phase in force at junction j for step t (needs the lane counts of the step
 * start for MAX_PRESSURE junctions, which it may update) */
static int current_phase(osim *s, int j)
{
    int b = s->junc_phase_begin[j], e = s->junc_phase_begin[j + 1];
    if (e == b) return -1;
    if (s->policy[j] == POL_MANUAL) return s->manual_phase[j];
    if (s->policy[j] == POL_MAX_PRESSURE) {
        if (max_pressure_decides(s, j)) s->manual_phase[j] = max_pressure_phase(s, j);
        return s->manual_phase[j];
    }
    /* FIXED_TIME: phases in order, starting with phase 0 at t = 0 */
    double cycle = 0.0;
    for (int p = b; p < e; ++p) cycle += s->phase_dur[p];
    double tt = fmod((double)s->t * s->P.dt, cycle), acc = 0.0;
    for (int p = b; p < e; ++p) {
        acc += s->phase_dur[p];
        if (tt < acc) return p - b;
    }
    return e - b - 1;
}

static void update_signals(osim *s)
{
    memset(s->green, 0, s->NJL);
    for (int j = 0; j < s->NJ; ++j) {
        if (s->policy[j] == POL_NONE) continue;
        int ph = current_phase(s, j);
        if (ph < 0) continue;
        int p = s->junc_phase_begin[j] + ph;
        for (int e = s->phase_green_begin[p]; e < s->phase_green_begin[p + 1]; ++e) s->green[s->phase_green_jl[e]] = 1;
    }
    for (int q = 0; q < s->NJL; ++q)
        if (s->policy[s->jl_junction[q]] == POL_NONE || s->junc_phase_begin[s->jl_junction[q] + 1] == s->junc_phase_begin[s->jl_junction[q]])
            s->green[q] = 1;
}

/* ------------------------------------------------------------------------ */
/* P3 index                                                                  */
/* ------------------------------------------------------------------------ */
static const osim *g_sort_sim;
static int cmp_lane_order(const void *a, const void *b)
{
    int i = *(const int *)a, j = *(const int *)b;
    const osim *s = g_sort_sim;
    if (s->lane[i] != s->lane[j]) return s->lane[i] < s->lane[j] ? -1 : 1;
    if (ahead(s, i, j)) return -1;
    if (ahead(s, j, i)) return 1;
    return 0;
}

static void build_index(osim *s)
{
    int n = 0;
    for (int i = 0; i < s->N; ++i)
        if (s->status[i] == ACTIVE) s->sorted[n++] = i;
    g_sort_sim = s;
    qsort(s->sorted, n, sizeof(int), cmp_lane_order);
    memset(s->lane_cnt, 0, s->NL * sizeof(int));
    for (int c = 0; c < n; ++c) s->lane_cnt[s->lane[s->sorted[c]]]++;
    s->lane_start[0] = 0;
    for (int m = 0; m < s->NL; ++m) s->lane_start[m + 1] = s->lane_start[m] + s->lane_cnt[m];
}

/* ------------------------------------------------------------------------ */
/* P2 departures (Appendix B.2: vehicles whose departure time has come are   */
/* put into lanes when the connection is safe)                               */
/* [reading] per origin road, waiting vehicles leave in (tau, id) order;     */
/* the head takes the lane of its lane group with the most room ahead of it  */
/* (ties to the lower lane index), needs that room >= s0, and needs nothing  */
/* behind it able to reach its rear within the step (reach = x + v dt +      */
/* a_max dt^2/2); at most one insertion per lane per step; the first head    */
/* that cannot enter stops its road's queue for this step.  v = 0.           */
/*  - A trip starting at its origin road's start (start position <= 0)       */
/*    enters at x = 0 behind every vehicle of the lane: room = x - L of the  */
/*    rearmost vehicle (+inf on an empty lane); behind it are the front      */
/*    vehicles h of the feeder junction lanes, whose reach beyond their lane */
/*    end, x_h + v_h dt + a_max dt^2/2 - len(feeder), must be <= -L_head.    */
/*  - A trip starting at an AOI's connection partway along the road          */
/*    (start position p > 0; Appendix B.1: a start may be a position in a    */
/*    lane; Appendix B.2: an AOI puts a due vehicle into the lane when the   */
/*    connection is safe) enters with its front at x = p: room = x - L of    */
/*    the nearest vehicle ahead (x > p, or x = p with a smaller id) minus p; */
/*    behind it is the nearest vehicle of the lane behind, whose reach must  */
/*    be <= p - L_head, or, on a lane with no vehicle behind, the feeder     */
/*    front vehicles, whose reach beyond their lane end must be <= p - L.    */
/* ------------------------------------------------------------------------ */
/* reach of the front vehicles of lane m's feeders past their lane ends must
 * stay <= rear (the entrant's rear bumper); *near collects |margin| */
static int feeders_clear(const osim *s, int m, double rear, double *near)
{
    const oparams *P = &s->P;
    double reach_extra = 0.5 * P->a_max * P->dt * P->dt;
    int safe = 1;
    for (int e = s->feed_begin[m]; e < s->feed_begin[m + 1]; ++e) {
        int fl = s->feed_jl[e];
        int h = lane_front(s, fl);
        if (h < 0) continue;
        double mg = rear - (s->x[h] + s->v[h] * P->dt + reach_extra - s->lane_len[fl]);
        if (fabs(mg) < *near) *near = fabs(mg);
        if (!(mg >= 0.0)) safe = 0;
    }
    return safe;
}

static void departures(osim *s)
{
    const oparams *P = &s->P;
    double now = (double)s->t * P->dt;
    double reach_extra = 0.5 * P->a_max * P->dt * P->dt;
    for (int r = 0; r < s->R; ++r) {
        int lb = s->road_lane_begin[r], le = s->road_lane_begin[r + 1];
        unsigned used = 0;
        for (int c = s->q_begin[r]; c < s->q_begin[r + 1]; ++c) {
            int i = s->q_veh[c];
            if (s->status[i] != WAITING) continue;
            if (!(s->tau[i] <= now)) break;
            double p = s->start_s[i] > 0.0 ? s->start_s[i] : 0.0;
            int best = -1;
            double best_room = -INFINITY;
            double near = INFINITY;
            for (int m = lb; m < le; ++m) {
                if (used & (1u << (m - lb))) continue;
                if (s->restricted[m]) continue;
                s->k[i] = 0;
                if (!in_group(s, i, m)) continue;
                double room;
                int safe;
                if (p == 0.0) {
                    safe = feeders_clear(s, m, -s->L[i], &near);
                    int z = lane_rear(s, m);
                    room = z < 0 ? INFINITY : s->x[z] - s->L[z];
                } else {
                    /* the lane's vehicles front first: the leader is the last
                     * one ahead of the entrant, the follower the first behind */
                    int lead = -1, fol = -1;
                    for (int q = 0; q < s->lane_cnt[m]; ++q) {
                        int z = LANE(s, m)[q];
                        if (s->x[z] > p || (s->x[z] == p && z < i)) lead = z;
                        else { fol = z; break; }
                    }
                    room = lead < 0 ? INFINITY : s->x[lead] - s->L[lead] - p;
                    if (fol >= 0) {
                        double mg = (p - s->L[i]) - (s->x[fol] + s->v[fol] * P->dt + reach_extra);
                        if (fabs(mg) < near) near = fabs(mg);
                        safe = mg >= 0.0;
                    } else {
                        safe = feeders_clear(s, m, p - s->L[i], &near);
                    }
                }
                if (!safe) continue;
                if (room < INFINITY && fabs(room - P->s0) < near) near = fabs(room - P->s0);
                if (room > best_room) { best_room = room; best = m; }
            }
            s->margin[(size_t)i * NMARGIN + 5] = near;
            if (best < 0 || !(best_room >= P->s0)) break;
            used |= 1u << (best - lb);
            s->status[i] = ACTIVE;
            s->lane[i] = best;
            s->k[i] = 0;
            s->x[i] = p;
            s->v[i] = 0.0;
            s->event[i] |= EV_DEPART;
            s->n_departures += 1;
            /* a used lane is not consulted again in this step, so the index of
             * the committed state stays valid for the remaining heads */
        }
    }
}

/* ------------------------------------------------------------------------ */
/* U2 MOBIL for one direction (Appendix B.3 MOBIL utility)                   */
/* u = (a~_ego - a_ego) + p ((a~_new - a_new) + (a~_old - a_old)) - a_th     */
/* [reading] a~ is the acceleration after the prospective change (Kesting et */
/* al. 2007), a_th is subtracted so u > 0 exactly when the gain beats the    */
/* threshold, and the change must be feasible:                               */
/*   F1 the vehicle is on a road lane (no lane change inside junctions)      */
/*   F2 it stays in its lane group, or moves strictly closer to it           */
/*   F3 positive gap to the target leader (side leader, else the target      */
/*      lane's lookahead vehicle)                                            */
/*   F4 the new follower cannot reach the vehicle's rear within one step     */
/*      (v dt + a_max dt^2/2); with no new follower, no feeder junction lane */
/*      front vehicle can reach it                                           */
/*   F5 the new follower's deceleration stays within b_safe                  */
/*   F6 a rightward change yields to any vehicle two lanes right that sits   */
/*      in the same gap of the target lane                                   */
/* The prospective acceleration a~_ego ignores the wrong-lane end obstacle   */
/* (F2 only admits lanes of the group or closer to it) but keeps the red     */
/* signal obstacle.  Absent followers contribute 0.  Returns -inf when       */
/* infeasible; records the smallest margins for the parity report.          */
/* ------------------------------------------------------------------------ */
static double mobil_dir(osim *s, int i, int dir, double *m_pos, double *m_acc, int *target_out)
{
    const oparams *P = &s->P;
    int l = s->lane[i];
    *target_out = -1;
    if (l >= s->NRL) return -INFINITY; /* F1 */
    int r = s->lane_road[l];
    int lb = s->road_lane_begin[r], le = s->road_lane_begin[r + 1];
    int kk = l + dir;
    if (kk < lb || kk >= le) return -INFINITY;
    *target_out = kk;
    if (s->restricted[kk]) return -INFINITY; /* no change into a restricted lane */
    /* F2 */
    if (in_group(s, i, l)) {
        if (!in_group(s, i, kk)) return -INFINITY;
    } else if (!(group_dist(s, i, kk) < group_dist(s, i, l))) {
        return -INFINITY;
    }
    double reach_extra = 0.5 * P->a_max * P->dt * P->dt;
    int tl = rearmost_ahead(s, kk, i, -1, -1);
    int tf = frontmost_behind(s, kk, i, -1);
    /* F6 (discrete): a vehicle j of lane kk+1 is in the same gap of kk as i
     * exactly when tf (if any) is not ahead of j and j is not ahead of tl */
    if (dir > 0 && kk + 1 < le) {
        int m2 = kk + 1;
        for (int c = 0; c < s->lane_cnt[m2]; ++c) {
            int j = LANE(s, m2)[c];
            int above_tf = tf < 0 || ahead(s, j, tf);
            int below_tl = tl < 0 || ahead(s, tl, j);
            if (above_tf && below_tl) return -INFINITY;
        }
    }
    /* continuous checks: record every margin, decide on all of them */
    int feasible = 1;
    double worst_fail = 0.0, min_pass = INFINITY; /* position checks */
    double g;
    {
        /* F3: gap to the target leader (side leader, else target lookahead) */
        olead tg = leader_in(s, i, kk, -1, -1);
        g = tg.exists ? tg.rear - s->x[i] : INFINITY;
    }
    if (!(g > 0.0)) { feasible = 0; if (-g > worst_fail) worst_fail = -g; }
    if (fabs(g) < min_pass) min_pass = fabs(g);
    /* [reading] a new follower whose front is behind the rear of a vehicle
     * merging into its lane already yields to that vehicle (bounded by its
     * rear), so F4 and F5 do not apply to it */
    int tf_yields = tf >= 0 && merge_target(s, i) == kk && s->x[i] - s->L[i] > s->x[tf];
    if (tf >= 0 && !tf_yields) {
        g = s->x[i] - s->L[i] - s->x[tf] - (s->v[tf] * P->dt + reach_extra); /* F4 */
        if (!(g >= 0.0)) { feasible = 0; if (-g > worst_fail) worst_fail = -g; }
        if (fabs(g) < min_pass) min_pass = fabs(g);
    } else if (tf < 0) {
        for (int e = s->feed_begin[kk]; e < s->feed_begin[kk + 1]; ++e) {
            int fl = s->feed_jl[e];
            int h = lane_front(s, fl);
            if (h < 0) continue;
            g = (s->x[i] - s->L[i]) - (s->x[h] + s->v[h] * P->dt + reach_extra - s->lane_len[fl]);
            if (!(g >= 0.0)) { feasible = 0; if (-g > worst_fail) worst_fail = -g; }
            if (fabs(g) < min_pass) min_pass = fabs(g);
        }
    }
    /* accelerations (all from the snapshot) */
    double a_e = own_accel(s, i);
    double ta_e = accel_in(s, i, kk, leader_in(s, i, kk, -1, -1), stop_at_end(s, i, kk, 0));
    double d_new = 0.0, d_old = 0.0;
    double f5 = INFINITY;
    if (tf >= 0) {
        double a_tf = own_accel(s, tf);
        double ta_tf = accel_in(s, tf, kk, leader_in(s, tf, kk, -1, i), stop_at_end(s, tf, kk, 1));
        f5 = ta_tf + P->b_safe;
        d_new = ta_tf - a_tf;
    }
    int of = frontmost_behind(s, l, i, -1);
    if (of >= 0) {
        double a_of = own_accel(s, of);
        double ta_of = accel_in(s, of, l, leader_in(s, of, l, i, -1), stop_at_end(s, of, l, 1));
        d_old = ta_of - a_of;
    }
    int f5_ok = !(tf >= 0) || tf_yields || f5 >= 0.0;
    if (tf_yields) f5 = INFINITY;
    /* position-check robustness: a passing decision is near when its
     * smallest margin is small, a failing one when its largest violation is */
    double pos_rob = feasible ? min_pass : worst_fail;
    double acc_rob = (tf >= 0 && !tf_yields) ? fabs(f5) : INFINITY;
    int overall = feasible && f5_ok;
    /* when the position checks already fail robustly, F5 cannot flip it */
    if (!feasible) acc_rob = INFINITY;
    if (feasible && !f5_ok) pos_rob = INFINITY;
    if (pos_rob < *m_pos) *m_pos = pos_rob;
    if (acc_rob < *m_acc) *m_acc = acc_rob;
    if (!overall) return -INFINITY;
    double da = (ta_e - a_e) + P->p * (d_new + d_old);
    /* [reading] mandatory change: outside its lane group a vehicle takes a
     * feasible move toward the group with utility at least 1, so p_LC reaches
     * its cap */
    if (!in_group(s, i, l)) return fmax(da - P->a_th, 1.0);
    return da - P->a_th;
}

/* ------------------------------------------------------------------------ */
/* one step                                                                  */
/* ------------------------------------------------------------------------ */
static void step_once(osim *s)
{
    const oparams *P = &s->P;
    const int N = s->N, NRL = s->NRL;
    double reach_extra = 0.5 * P->a_max * P->dt * P->dt;
    for (int i = 0; i < N; ++i) {
        for (int c = 0; c < NMARGIN; ++c) s->margin[(size_t)i * NMARGIN + c] = INFINITY;
        s->mobil[i * 4 + 0] = s->mobil[i * 4 + 1] = -INFINITY;
        s->mobil[i * 4 + 2] = s->mobil[i * 4 + 3] = 0.0;
        s->decision[i] = 0;
        s->event[i] = 0;
    }
    /* prepare */
    build_index(s);
    update_signals(s);
    departures(s);
    build_index(s);

    memset(s->road_sumv, 0, s->R * sizeof(double));
    memset(s->road_cnt, 0, s->R * sizeof(int));
    memset(s->lane_wait, 0, s->NL * sizeof(int));
    int n_active = 0;

    /* update: every read below is from the snapshot (x, v, lane, k) */
    for (int i = 0; i < N; ++i) {
        s->n_status[i] = s->status[i];
        s->n_lane[i] = s->lane[i];
        s->n_k[i] = s->k[i];
        s->n_x[i] = s->x[i];
        s->n_v[i] = s->v[i];
        if (s->status[i] != ACTIVE) continue;
        n_active++;
        double *mg = s->margin + (size_t)i * NMARGIN;
        int l = s->lane[i];
        /* U1 */
        double a_e = own_accel(s, i);
        /* U2 */
        double m_pos = INFINITY, m_acc = INFINITY;
        int kL, kR;
        double uL = mobil_dir(s, i, -1, &m_pos, &m_acc, &kL);
        double uR = mobil_dir(s, i, +1, &m_pos, &m_acc, &kR);
        mg[1] = m_pos;
        mg[2] = m_acc;
        double m_u = INFINITY;
        if (uL > -INFINITY) m_u = fmin(m_u, fabs(uL));
        if (uR > -INFINITY) m_u = fmin(m_u, fabs(uR));
        mg[0] = m_u;
        /* U3: u_T = max(0,u_L) + max(0,u_R); p_LC piecewise.
         * [reading] the middle branch is the continuous ramp
         * p_min + (p_max - p_min) u_T; one Philox draw r = word0 * 2^-32 with
         * key = seed and counter = (vehicle id, step, 0, 0) decides; [0, p_LC)
         * is split left-first in proportion u_L+ : u_R+; with u_T = 0 the
         * floor probability p_min is split equally among feasible sides. */
        double uLp = fmax(0.0, uL), uRp = fmax(0.0, uR), uT = uLp + uRp;
        double pLC = uT >= 1.0 ? P->p_max : (uT > 0.0 ? P->p_min + (P->p_max - P->p_min) * uT : P->p_min);
        uint32_t ctr[4] = {(uint32_t)i, (uint32_t)s->t, 0u, 0u}, w[4];
        osim_philox(P->seed, ctr, w);
        double rr = ldexp((double)w[0], -32);
        int dec = 0;
        double m_r = INFINITY;
        if (uT > 0.0) {
            double bL = pLC * uLp / uT;
            /* a side with zero utility owns an empty interval (guarded, since
             * the rounded boundary may sit a hair below p_LC) */
            if (uLp > 0.0 && rr < bL) dec = 1;
            else if (uRp > 0.0 && rr >= bL && rr < pLC) dec = 2;
            m_r = fmin(fabs(rr - bL), fabs(rr - pLC));
        } else {
            int fL = uL > -INFINITY, fR = uR > -INFINITY;
            if (fL && fR) {
                if (rr < 0.5 * P->p_min) dec = 1;
                else if (rr < P->p_min) dec = 2;
                m_r = fmin(fabs(rr - 0.5 * P->p_min), fabs(rr - P->p_min));
            } else if (fL || fR) {
                if (rr < P->p_min) dec = fL ? 1 : 2;
                m_r = fabs(rr - P->p_min);
            }
        }
        mg[3] = m_r;
        s->mobil[i * 4 + 0] = uL;
        s->mobil[i * 4 + 1] = uR;
        s->mobil[i * 4 + 2] = uT;
        s->mobil[i * 4 + 3] = pLC;
        s->decision[i] = dec;
        int ln = dec == 1 ? kL : (dec == 2 ? kR : l);
        double a = a_e;
        int yl = dec ? -1 : yield_leader(s, i);
        if (yl >= 0)
            a = fmin(a, idm_acc(P, s->v[i], s->f[i] * s->lane_lim[l], s->x[yl] - s->L[yl] - s->x[i], s->v[i] - s->v[yl]));
        if (dec) {
            a = accel_in(s, i, ln, leader_in(s, i, ln, -1, -1), stop_at_end(s, i, ln, 0));
            s->n_lane_changes += 1;
        }
        /* U4: ballistic update with in-step stop (Treiber & Kanagaraj 2015) */
        double x = s->x[i], v = s->v[i];
        double vh = v + a * P->dt, xn, vn;
        if (vh >= 0.0) { xn = x + v * P->dt + 0.5 * a * P->dt * P->dt; vn = vh; }
        else { xn = x - v * v / (2.0 * a); vn = 0.0; }
        /* [reading] bound: snapshot rear of the own-lane (or lookahead) leader,
         * after a change also the target leader's rear, and the lane end when
         * the stop obstacle applies in the final lane; a clamped vehicle takes
         * the bounding vehicle's speed (0 at the stop line) if that is lower;
         * nobody moves backwards */
        double B = INFINITY, vcap = INFINITY;
        olead ld = leader_in(s, i, l, -1, -1);
        if (ld.exists) { B = ld.rear; vcap = ld.v; }
        if (dec) {
            olead l2 = leader_in(s, i, ln, -1, -1);
            if (l2.exists) {
                if (l2.rear < B) { B = l2.rear; vcap = l2.v; }
                else if (l2.rear == B) vcap = fmin(vcap, l2.v);
            }
        }
        if (yl >= 0) {
            double by = s->x[yl] - s->L[yl];
            if (by < B) { B = by; vcap = s->v[yl]; }
            else if (by == B) vcap = fmin(vcap, s->v[yl]);
        }
        if (stop_at_end(s, i, ln, 1)) {
            double bl = s->lane_len[ln];
            if (bl < B) { B = bl; vcap = 0.0; }
            else if (bl == B) vcap = 0.0;
        }
        double m_x = fabs(xn - B);
        if (xn > B) {
            xn = fmax(B, x);
            vn = fmin(vn, vcap);
            s->event[i] |= EV_CLAMP;
            s->n_clamps += 1;
        }
        /* U5: lane end, or the trip's end position on its last road
         * ([reading] Section 3.2 set_vehicle_route's end position, an AOI's
         * connection (Appendix B.1) as the trip's end: the trip ends in the step its front
         * passes that position) */
        int nl = ln, nk = s->k[i], nst = ACTIVE;
        double len = s->lane_len[ln];
        const int last = ln < NRL && s->k[i] == route_len(s, i) - 1;
        if (last && s->end_s[i] >= 0.0 && s->end_s[i] < len) len = s->end_s[i];
        m_x = fmin(m_x, fabs(xn - len));
        if (xn > len) {
            if (last) {
                nst = FINISHED;
                s->finish_step[i] = (int)s->t;
                s->sum_tt += (double)(s->t + 1) * P->dt - s->tau[i];
                s->n_finished += 1;
                s->event[i] |= EV_FINISH;
            } else {
                int g = sigma(s, i, ln);
                if (g < 0) abort(); /* the stop obstacle keeps such a vehicle in its lane */
                if (g < NRL) {
                    /* [reading] merges: a road lane fed by several junction
                     * lanes admits an entrant only if no lower-id feeder has a
                     * front vehicle that could cross its end this step */
                    int blocked = 0;
                    for (int e = s->feed_begin[g]; e < s->feed_begin[g + 1]; ++e) {
                        int fl = s->feed_jl[e];
                        if (fl >= ln) break;
                        int h = lane_front(s, fl);
                        if (h < 0) continue;
                        double reach = s->x[h] + s->v[h] * P->dt + reach_extra - s->lane_len[fl];
                        m_x = fmin(m_x, fabs(reach));
                        if (reach > 0.0) blocked = 1;
                    }
                    if (blocked) {
                        xn = len;
                        vn = 0.0;
                        s->event[i] |= EV_FEEDER_BLOCK;
                        s->n_feeder_blocks += 1;
                    } else {
                        nl = g;
                        xn -= len;
                        nk = s->k[i] + 1;
                        s->event[i] |= EV_TRANSFER;
                        s->n_transfers += 1;
                    }
                } else {
                    nl = g;
                    xn -= len;
                    s->event[i] |= EV_TRANSFER;
                    s->n_transfers += 1;
                }
                if (nl != ln && xn > s->lane_len[nl]) abort(); /* one hop per step */
            }
        }
        mg[4] = m_x;
        s->n_status[i] = nst;
        s->n_lane[i] = nst == ACTIVE ? nl : -1;
        s->n_k[i] = nk;
        s->n_x[i] = nst == ACTIVE ? xn : 0.0;
        s->n_v[i] = nst == ACTIVE ? vn : 0.0;
        /* U6 [reading]: a vehicle counts for the lane it occupied in the
         * snapshot, with its end-of-step speed */
        if (l < NRL) {
            s->road_sumv[s->lane_road[l]] += vn;
            s->road_cnt[s->lane_road[l]] += 1;
        }
        s->vend[i] = vn;
    }
    /* U6 lane queue length (Section 3.3: vehicles waiting to be released at
     * the end of the lane) [reading]: the unbroken run of vehicles, counted
     * from the front of the lane in the snapshot order, whose end-of-step
     * speed is below 0.1 m/s; a stopped vehicle behind a moving one is not in
     * the queue at the lane end */
    for (int m = 0; m < s->NL; ++m) {
        int q = 0;
        while (q < s->lane_cnt[m] && s->vend[LANE(s, m)[q]] < 0.1) q++;
        s->lane_wait[m] = q;
    }
    (void)reach_extra;
    /* metrics of the step */
    double sv = 0.0, sc = 0.0;
    for (int r = 0; r < s->R; ++r) { sv += s->road_sumv[r]; sc += s->road_cnt[r]; }
    s->mean_speed_last = sc > 0 ? sv / sc : 0.0;
    if (sc > 0) { s->speed_acc += s->mean_speed_last; s->speed_steps += 1; }
    s->vehicle_steps += n_active;
    /* commit */
    int *ti;
    double *td;
    ti = s->status; s->status = s->n_status; s->n_status = ti;
    ti = s->lane; s->lane = s->n_lane; s->n_lane = ti;
    ti = s->k; s->k = s->n_k; s->n_k = ti;
    td = s->x; s->x = s->n_x; s->n_x = td;
    td = s->v; s->v = s->n_v; s->n_v = td;
    s->t += 1;
}

void osim_step(osim *s, int n)
{
    for (int c = 0; c < n; ++c) step_once(s);
}

/* ------------------------------------------------------------------------ */
/* state and metrics access                                                  */
/* ------------------------------------------------------------------------ */
void osim_get_state(const osim *s, int64_t *t, int *status, int *lane, int *k, double *x, double *v, int *finish_step)
{
    *t = s->t;
    memcpy(status, s->status, s->N * sizeof(int));
    memcpy(lane, s->lane, s->N * sizeof(int));
    memcpy(k, s->k, s->N * sizeof(int));
    memcpy(x, s->x, s->N * sizeof(double));
    memcpy(v, s->v, s->N * sizeof(double));
    memcpy(finish_step, s->finish_step, s->N * sizeof(int));
}

/* Replaces the vehicle state; finished-trip totals are recomputed from the
 * finish steps and the running horizon averages restart from zero. */
void osim_set_state(osim *s, int64_t t, const int *status, const int *lane, const int *k, const double *x,
                    const double *v, const int *finish_step)
{
    s->t = t;
    memcpy(s->status, status, s->N * sizeof(int));
    memcpy(s->lane, lane, s->N * sizeof(int));
    memcpy(s->k, k, s->N * sizeof(int));
    memcpy(s->x, x, s->N * sizeof(double));
    memcpy(s->v, v, s->N * sizeof(double));
    memcpy(s->finish_step, finish_step, s->N * sizeof(int));
    s->sum_tt = 0; s->n_finished = 0;
    for (int i = 0; i < s->N; ++i)
        if (s->status[i] == FINISHED) {
            s->n_finished += 1;
            s->sum_tt += (double)(s->finish_step[i] + 1) * s->P.dt - s->tau[i];
        }
    s->vehicle_steps = s->speed_acc = s->speed_steps = s->mean_speed_last = 0;
    s->n_lane_changes = s->n_transfers = s->n_clamps = s->n_feeder_blocks = s->n_departures = 0;
}

void osim_set_signal_phases(osim *s, int n, const int *junction, const int *phase)
{
    for (int c = 0; c < n; ++c) {
        s->policy[junction[c]] = POL_MANUAL;
        s->manual_phase[junction[c]] = phase[c];
    }
}

void osim_set_policy(osim *s, int n, const int *junction, const int *policy)
{
    for (int c = 0; c < n; ++c) s->policy[junction[c]] = policy[c];
}

/* Section 3.2 "Vehicle" set_vehicle_route: vehicle i follows `route` from
 * now on.  The new route begins with the road the vehicle is on (its origin
 * road while it waits), and, on a junction lane, continues with that lane's
 * road; the vehicle's route position becomes 0.  The trip ends at the end of
 * the new route's last road.  The caller checks the route is connected. */
void osim_set_vehicle_route(osim *s, int i, const int *route, int len, double end_s)
{
    s->end_s[i] = end_s;
    if (s->route_n + len > s->route_cap) {
        while (s->route_n + len > s->route_cap) s->route_cap *= 2;
        s->route = (int *)realloc(s->route, (size_t)s->route_cap * sizeof(int));
    }
    memcpy(s->route + s->route_n, route, (size_t)len * sizeof(int));
    s->rstart[i] = (int)s->route_n;
    s->rlen[i] = len;
    s->route_n += len;
    s->k[i] = 0;
}

void osim_get_route(const osim *s, int i, int *start_pos, int *len, int *out, int max)
{
    *start_pos = s->k[i];
    *len = s->rlen[i];
    for (int c = 0; c < s->rlen[i] && c < max; ++c) out[c] = s->route[s->rstart[i] + c];
}

/* Section 3.2 "Lane" set_lane_max_speed: the speed limit of lanes (road or
 * junction lanes, global lane ids) from the next step on; every vehicle's
 * desired speed on such a lane is its factor times the new limit */
void osim_set_lane_max_speed(osim *s, int n, const int *lanes, const double *speed)
{
    for (int c = 0; c < n; ++c) s->lane_lim[lanes[c]] = speed[c];
}

/* trip start positions (metres along the origin road; <= 0 for its start)
 * of vehicles vids[c], e.g. an AOI's connection on that road */
void osim_set_trip_starts(osim *s, int n, const int *vids, const double *start_s)
{
    for (int c = 0; c < n; ++c) s->start_s[vids[c]] = start_s[c];
}

/* trip end positions (metres along the last road of the route; < 0 for
 * its end) of vehicles vids[c], e.g. an AOI's connection on that road */
void osim_set_trip_ends(osim *s, int n, const int *vids, const double *end_s)
{
    for (int c = 0; c < n; ++c) s->end_s[vids[c]] = end_s[c];
}

/* Section 3.2 "Lane" set_lane_restriction: lanes (global ids) restricted
 * (flag != 0) or released from the next step on */
void osim_set_lane_restriction(osim *s, int n, const int *lanes, const int *flags)
{
    for (int c = 0; c < n; ++c) s->restricted[lanes[c]] = flags[c] != 0;
}

/* policy and phase of every junction (the phase is the MANUAL phase, or the
 * phase in force of a MAX_PRESSURE junction; ignored otherwise) */
void osim_set_junctions(osim *s, const int *policy, const int *phase)
{
    for (int j = 0; j < s->NJ; ++j) {
        s->policy[j] = policy[j];
        s->manual_phase[j] = phase[j];
    }
}

void osim_get_junctions(const osim *s, int *policy, int *phase)
{
    memcpy(policy, s->policy, s->NJ * sizeof(int));
    memcpy(phase, s->manual_phase, s->NJ * sizeof(int));
}

/* out[NMETRIC]: t, waiting, active, finished, sum_tt, att, mean_speed_last,
 * mean_speed_avg, vehicle_steps, lane_changes, transfers, clamps,
 * feeder_blocks, departures, speed_steps, 0 */
void osim_get_metrics(const osim *s, double *out)
{
    double w = 0, a = 0, f = 0;
    for (int i = 0; i < s->N; ++i) {
        if (s->status[i] == WAITING) w += 1;
        else if (s->status[i] == ACTIVE) a += 1;
        else f += 1;
    }
    out[0] = (double)s->t; out[1] = w; out[2] = a; out[3] = f;
    out[4] = s->sum_tt; out[5] = f > 0 ? s->sum_tt / f : 0.0;
    out[6] = s->mean_speed_last;
    out[7] = s->speed_steps > 0 ? s->speed_acc / s->speed_steps : 0.0;
    out[8] = s->vehicle_steps; out[9] = s->n_lane_changes; out[10] = s->n_transfers;
    out[11] = s->n_clamps; out[12] = s->n_feeder_blocks; out[13] = s->n_departures;
    out[14] = s->speed_steps; out[15] = 0.0;
}

void osim_get_road_stats(const osim *s, double *sumv, int *cnt)
{
    memcpy(sumv, s->road_sumv, s->R * sizeof(double));
    memcpy(cnt, s->road_cnt, s->R * sizeof(int));
}

void osim_get_lane_waiting(const osim *s, int *out) { memcpy(out, s->lane_wait, s->NL * sizeof(int)); }

void osim_get_green(const osim *s, unsigned char *out) { memcpy(out, s->green, s->NJL); }

/* signal state for step t without stepping (P1 for the current t) */
void osim_eval_signals(osim *s, unsigned char *out)
{
    build_index(s);
    update_signals(s);
    memcpy(out, s->green, s->NJL);
}

void osim_last_diag(const osim *s, double *margin, double *mobil, int *decision, int *event)
{
    memcpy(margin, s->margin, (size_t)s->N * NMARGIN * sizeof(double));
    memcpy(mobil, s->mobil, (size_t)s->N * 4 * sizeof(double));
    memcpy(decision, s->decision, s->N * sizeof(int));
    memcpy(event, s->event, s->N * sizeof(int));
}

int osim_n_vehicles(const osim *s) { return s->N; }

/* ------------------------------------------------------------------------ */
/* Shortest routes (Section 4 "Congestion Pricing": drivers move to routes  */
/* of lower cost once roads carry prices; Appendix F congestion pricing:    */
/* every road may carry a price; Appendix E travel demand: routes of        */
/* shortest travel time).                                                    */
/* [reading] The cost of a route is the sum, over every road after its      */
/* first, of the road's movement cost: the fastest open junction lane into  */
/* it from the road before (length / limit), plus its own travel time (its  */
/* length over the highest limit of its lanes, or a time the caller gives), */
/* plus its price.  The route is an integer result decided by these sums,   */
/* so it is computed in FP32, the precision the GPU takes it in; the       */
/* cost-to-go of a road is its movement cost plus the cost-to-go of the     */
/* road it enters (the order a tree grown from the destination sums in),    */
/* and of roads with equal candidate costs the smaller id is taken.  A      */
/* route of more roads than the network has counts as unreachable.          */
/* Distances by Dijkstra from the destination over the reversed movements,  */
/* the minimum found by a linear scan.                                       */
/* ------------------------------------------------------------------------ */

typedef struct {
    int R;
    int *fb, *fto;     /* forward movements: [R+1], [E] (ascending target per road) */
    float *fw;         /* [E] movement cost */
    int *rb, *rfrom;   /* reversed: movements entering each road */
    float *rw;
} ograph;

static void ograph_free(ograph *g)
{
    free(g->fb); free(g->fto); free(g->fw); free(g->rb); free(g->rfrom); free(g->rw);
}

/* road travel time: length over the highest limit of its lanes (FP32) */
static float road_time_of(const osim *s, int r, const float *road_time)
{
    if (road_time) return road_time[r];
    float vmax = 0.0f;
    for (int l = s->road_lane_begin[r]; l < s->road_lane_begin[r + 1]; ++l)
        if ((float)s->lane_lim[l] > vmax) vmax = (float)s->lane_lim[l];
    return (float)s->lane_len[s->road_lane_begin[r]] / vmax;
}

static void ograph_build(const osim *s, const float *price, const float *road_time, ograph *g)
{
    int R = s->R;
    g->R = R;
    /* for the road being scanned: cmin[r2], the cheapest junction lane into
     * r2 (seen[r2] == r once one was found), and the list of its targets */
    float *cmin = (float *)xcalloc(R, sizeof(float));
    int *seen = (int *)xcalloc(R, sizeof(int));
    int *tl = (int *)xcalloc(s->NJL, sizeof(int));
    for (int r = 0; r < R; ++r) seen[r] = -1;
    g->fb = (int *)xcalloc(R + 1, sizeof(int));
    int cap = 16, E = 0;
    g->fto = (int *)xcalloc(cap, sizeof(int));
    g->fw = (float *)xcalloc(cap, sizeof(float));
    for (int r = 0; r < R; ++r) {
        g->fb[r] = E;
        int nt = 0;
        for (int l = s->road_lane_begin[r]; l < s->road_lane_begin[r + 1]; ++l)
            for (int e = s->out_begin[l]; e < s->out_begin[l + 1]; ++e) {
                int q = s->out_jl[e];
                if (!jl_open(s, q)) continue;
                int r2 = s->lane_road[s->jl_out[q - s->NRL]];
                float c = (float)s->lane_len[q] / (float)s->lane_lim[q];
                if (seen[r2] != r) { seen[r2] = r; cmin[r2] = c; tl[nt++] = r2; }
                else if (c < cmin[r2]) cmin[r2] = c;
            }
        /* targets of road r in ascending id (insertion sort of a short list) */
        for (int a = 1; a < nt; ++a)
            for (int b = a; b > 0 && tl[b - 1] > tl[b]; --b) { int t = tl[b]; tl[b] = tl[b - 1]; tl[b - 1] = t; }
        for (int c = 0; c < nt; ++c) {
            int r2 = tl[c];
            if (E == cap) {
                cap *= 2;
                g->fto = (int *)realloc(g->fto, cap * sizeof(int));
                g->fw = (float *)realloc(g->fw, cap * sizeof(float));
            }
            float w = cmin[r2] + road_time_of(s, r2, road_time);
            w = w + (price ? price[r2] : 0.0f);
            g->fto[E] = r2;
            g->fw[E] = w;
            ++E;
        }
    }
    g->fb[R] = E;
    /* reversed movements */
    g->rb = (int *)xcalloc(R + 1, sizeof(int));
    g->rfrom = (int *)xcalloc(E, sizeof(int));
    g->rw = (float *)xcalloc(E, sizeof(float));
    for (int e = 0; e < E; ++e) g->rb[g->fto[e] + 1]++;
    for (int r = 0; r < R; ++r) g->rb[r + 1] += g->rb[r];
    int *fill = (int *)xcalloc(R, sizeof(int));
    for (int r = 0; r < R; ++r)
        for (int e = g->fb[r]; e < g->fb[r + 1]; ++e) {
            int t = g->fto[e], k = g->rb[t] + fill[t]++;
            g->rfrom[k] = r;
            g->rw[k] = g->fw[e];
        }
    free(fill); free(cmin); free(seen); free(tl);
}

/* cost-to-go of every road to road d (FP32; +inf where d cannot be reached) */
static void cost_to_go(const ograph *g, int d, float *dist)
{
    int R = g->R;
    unsigned char *done = (unsigned char *)xcalloc(R, 1);
    for (int r = 0; r < R; ++r) dist[r] = INFINITY;
    dist[d] = 0.0f;
    for (;;) {
        int u = -1;
        for (int r = 0; r < R; ++r)
            if (!done[r] && dist[r] < INFINITY && (u < 0 || dist[r] < dist[u])) u = r;
        if (u < 0) break;
        done[u] = 1;
        for (int k = g->rb[u]; k < g->rb[u + 1]; ++k) {
            int r = g->rfrom[k];
            float c = g->rw[k] + dist[u];
            if (c < dist[r]) dist[r] = c;
        }
    }
    free(done);
}

/* Routes for n (origin road, destination road) pairs under the lane limits
 * and restrictions in force, road prices price[R] (NULL: none) and road
 * times road_time[R] (NULL: free-flow).  out_begin[n+1] is a CSR into
 * out_roads (origin first, destination last; empty when the destination
 * cannot be reached).  Returns the number of unreachable pairs, or -1 when
 * more than cap roads would be written. */
int osim_shortest_routes(const osim *s, const float *price, const float *road_time, int n, const int *origin,
                         const int *dest, int *out_begin, int *out_roads, int cap)
{
    ograph g;
    ograph_build(s, price, road_time, &g);
    float *dist = (float *)xcalloc(s->R, sizeof(float));
    int last = -1, bad = 0, pos = 0;
    out_begin[0] = 0;
    for (int p = 0; p < n; ++p) {
        if (dest[p] != last) { cost_to_go(&g, dest[p], dist); last = dest[p]; }
        int r = origin[p], start = pos, ok = dist[r] < INFINITY;
        if (ok) {
            if (pos >= cap) { pos = -1; break; }
            out_roads[pos++] = r;
        }
        while (ok && r != dest[p]) {
            int best = -1;
            float bc = INFINITY;
            for (int e = g.fb[r]; e < g.fb[r + 1]; ++e) {
                float c = g.fw[e] + dist[g.fto[e]];
                if (c < bc) { bc = c; best = g.fto[e]; }
            }
            if (best < 0 || pos - start >= s->R) { ok = 0; break; }
            if (pos >= cap) { pos = -1; break; }
            out_roads[pos++] = best;
            r = best;
        }
        if (pos < 0) break;
        if (!ok) { pos = start; ++bad; }
        out_begin[p + 1] = pos;
    }
    free(dist);
    ograph_free(&g);
    return pos < 0 ? -1 : bad;
}
