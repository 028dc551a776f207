// Host side of the C ABI (include/tsim.h): input validation, internal lane
// numbering by road tile, device arena layout, state import/export and the
// step driver.  All device memory is carved from the caller's arena; the
// library itself never allocates device memory.
#include <algorithm>
#include <array>
#include <cmath>
#include <limits>
#include <cstdio>
#include <cstring>
#include <numeric>
#include <string>
#include <unordered_set>
#include <vector>

#include "../../include/tsim.h"
#include "tsim_internal.h"
#include "tsim_route.h"

namespace tsim {
hipError_t launch_prepare(const DevNet* Dd, const DevNet& H, hipStream_t s);
hipError_t launch_update(const DevNet* Dd, const DevNet& H, hipStream_t s, const PassStreams* ps);
hipError_t launch_fold(const DevNet& H, hipStream_t s);
hipError_t prepare_update_kernels();
hipError_t launch_set_phases(const DevNet* Dd, const DevNet& H, const int32_t* ids, const int32_t* ph, int n, hipStream_t s);
hipError_t launch_export(const DevNet* Dd, const DevNet& H, const int32_t* lane_ext, int32_t* o_lane, float* o_x,
                         float* o_v, int32_t* o_rpos, int32_t* o_rank, hipStream_t s);
hipError_t launch_import(const DevNet* Dd, const DevNet& H, const uint32_t* slots, const VehRec* recs, int n, hipStream_t s);
hipError_t launch_set_all_phases(const DevNet* Dd, const DevNet& H, const int32_t* ph, hipStream_t s);
hipError_t launch_set_policy(const DevNet* Dd, const DevNet& H, const int32_t* ids, const int32_t* pol, int n, hipStream_t s);
hipError_t noalloc_scratch(int32_t** out);
hipError_t launch_set_lane_speed(const DevNet& H, const int32_t* ids, const float* lim, int n, hipStream_t s);
hipError_t launch_record(const DevNet& H, const int32_t* lane_ext, TrajRec* out, long long cap,
                         unsigned long long* count, int every, hipStream_t s);
hipError_t launch_set_end(const DevNet& H, int inst, long long end, hipStream_t s);
hipError_t launch_aoi_counts(const DevNet& H, int v0, int nv, const int32_t* origin, const int32_t* dest, int n_aoi,
                             int32_t* counts, hipStream_t s);
hipError_t launch_apply_routes(const DevNet& H, const int32_t* n_rp, const int32_t* n_rem, const int32_t* n_nr,
                               const uint32_t* n_mask, int n_queue, hipStream_t s);
int update_blocks_per_cu(int sched);
}  // namespace tsim

using namespace tsim;

namespace {

thread_local std::string g_error;

struct Build {
    int R = 0, NJ = 0, NRL = 0, NJL = 0, NL = 0, N = 0;
    std::vector<int32_t> tile_lane_begin, tile_n_road;
    std::vector<float> lane_len, lane_lim;
    std::vector<uint32_t> lane_base;
    std::vector<int32_t> lane_cap, lane_tile, lane_local, jl_out, jl_junc, jl_ext, jl_in_local, jl_out_road;
    std::vector<uint32_t> jl_green_mask;
    std::vector<int32_t> out_begin, out_jl, feed_begin, feed_jl;
    std::vector<int32_t> int_of_ext, ext_of_int;
    std::vector<int32_t> junc_phase_begin, junc_policy;
    std::vector<int32_t> mp_begin, mp_mov;   // movements per junction: (in, out, green mask, 0) internal lanes
    std::vector<float> phase_dur;
    std::vector<double> junc_cycle;
    std::vector<float> tau, vf, vlen;
    std::vector<float> vend;         // per vehicle: trip end position on the last road, < 0: its end
    std::vector<float> vstart;       // per vehicle: trip start position on the origin road, <= 0: its start
    std::vector<int32_t> route_begin, route, q_begin, q_veh;   // route_begin: CSR of the routes given at creation
    std::vector<int32_t> rstart, rlen;   // the route in force of each vehicle: route[rstart, rstart + rlen)
    std::vector<uint32_t> q_mask;    // per queue entry: origin-road lanes that lead to its next road
    std::vector<uint8_t> restricted; // per internal lane (shorter: the rest unrestricted): no new vehicle enters
    uint64_t slots = 0;
    int G = 0;                       // partial slots: max over schedules of GT + GA + GB + GC
    // tile classes by lane count (<= 8, <= 16, <= 32, more); n_le[c] = tiles
    // of classes 0..c
    int n_le[4] = {0, 0, 0, 0};
    // instances of a batch (one for tsim_create)
    int n_inst = 1;
    std::vector<int32_t> tile_inst, junc_inst, inst_vbase;
    std::vector<uint32_t> inst_key;
    std::vector<long long> inst_t0;
    // per-instance offsets into the union: roads, junctions, road lanes,
    // junction lanes, vehicles (n_inst + 1 entries each)
    std::vector<int> road_off, junc_off, rl_off, jl_off, veh_off;
};

// sizes the arena of a handle is laid out for: the network itself, or the
// capacity reserved for a batch that instances join later
struct Caps {
    long long R = 0, NJ = 0, NL = 0, NRL = 0, NJL = 0, N = 0, S = 0, P = 0, E = 0, G = 0, n_inst = 0;
};

struct Region {
    void** ptr;
    size_t bytes;
};

int fail(std::string* err, int code, const std::string& msg)
{
    if (err) *err = msg;
    g_error = msg;
    return code;
}

int tile_class(const Build& B, int r)
{
    const int nl = B.tile_lane_begin[r + 1] - B.tile_lane_begin[r];
    return nl <= 8 ? 0 : (nl <= 16 ? 1 : (nl <= 32 ? 2 : 3));
}

// grids of a schedule: the grouped pass strides over at most nA tiles (those
// with few enough lanes), the wide pass over at most R; each gets no more
// workgroups than the device keeps resident (res_a, res_b; 0 = unknown)
struct SchedGrid {
    int gw, nA, GA, GB, GC, GT, GM, GL;
};

constexpr int kMaxGridA = 8192, kMaxGridB = 8192;

SchedGrid sched_grid(const Build& B, int sched, int res_a = 0, int res_b = 0, int res_c = 0, int res_t = 0)
{
    SchedGrid g{64, 0, 0, 0, 0, 0, 0, 0};
    switch (sched) {
    case kSched8x16: g.gw = 8; g.nA = B.n_le[0]; break;
    case kSched16x32:
    case kSched16x32P:
    case kSched8and16:
    case kSchedFused:
    case kSched16x64: g.gw = 16; g.nA = B.n_le[1]; break;
    case kSched32x64: g.gw = 32; g.nA = B.n_le[2]; break;
    default: g.gw = 64; g.nA = 0; break;
    }
    const int ng = 64 / g.gw;
    const int capA = res_a > 0 ? std::min(res_a, kMaxGridA) : kMaxGridA;
    const int capB = res_b > 0 ? std::min(res_b, kMaxGridB) : kMaxGridB;
    g.GA = g.nA > 0 ? std::max(1, std::min((g.nA + ng - 1) / ng, capA)) : 0;
    g.GB = std::max(1, std::min(B.R, capB));
    const int capC = res_c > 0 ? std::min(res_c, kMaxGridB) : kMaxGridB;
    g.GC = std::max(1, std::min(B.R, capC));
    if ((sched == kSched8and16 || sched == kSchedFused) && B.n_le[0] > 0) {
        // the tiny tiles come last: twice the resident workgroups, so that
        // each does fewer rounds and the launch's tail is shorter (measured
        // 2% faster than once, and four times slower again)
        const int capT = res_t > 0 ? std::min(2 * res_t, kMaxGridA) : kMaxGridA;
        g.GT = std::max(1, std::min((B.n_le[0] + 7) / 8, capT));
    }
    // medium tiles (fused schedule): at most kWideLanes lanes, two per wavefront
    if (sched == kSchedFused && B.n_le[2] > 0) {
        const int capM = res_t > 0 ? std::min(res_t, kMaxGridA) : kMaxGridA;
        g.GM = std::max(1, std::min((B.n_le[2] + 1) / 2, capM));
    }
    // large tiles (fused schedule): one per wavefront, three per workgroup
    if (sched == kSchedFused) {
        const int capL = res_c > 0 ? std::min(res_c, kMaxGridB) : kMaxGridB;
        g.GL = std::max(1, std::min((B.R + 2) / 3, capL));
    }
    return g;
}

// tiles per static size class (n_le: classes 0..c), which bound the grids of
// every schedule, and the partial-sum slots the largest grid needs
void count_tiles(Build& B)
{
    const int R = B.R;
    int cnt[4] = {0, 0, 0, 0};
    for (int r = 0; r < R; ++r) cnt[tile_class(B, r)]++;
    B.n_le[0] = cnt[0];
    for (int c = 1; c < 4; ++c) B.n_le[c] = B.n_le[c - 1] + cnt[c];
    B.G = 1;
    for (int s = 0; s < kNumSched; ++s) {
        const SchedGrid g = sched_grid(B, s);
        B.G = std::max(B.G, g.GA + g.GB + g.GC + g.GT + g.GM + g.GL);
    }
}

// partial-sum slots enough for any tile mix of at most R tiles
long long g_bound(int R)
{
    Build f;
    f.R = R;
    for (int c = 0; c < 4; ++c) f.n_le[c] = R;
    long long G = 1;
    for (int s = 0; s < kNumSched; ++s) {
        const SchedGrid g = sched_grid(f, s, 0, 0, 0, 0);
        G = std::max<long long>(G, g.GA + g.GB + g.GC + g.GT + g.GM + g.GL);
    }
    return G;
}

Caps caps_of(const Build& B)
{
    Caps c;
    c.R = B.R;
    c.NJ = B.NJ;
    c.NL = B.NL;
    c.NRL = B.NRL;
    c.NJL = B.NJL;
    c.N = B.N;
    c.S = (long long)B.slots;
    c.P = (long long)B.phase_dur.size();
    // room for routes changed by tsim_set_vehicle_route (appended)
    c.E = (long long)B.route.size() + (long long)B.route.size() / 4 + 4096;
    c.G = std::max<long long>(B.G, g_bound(B.R));
    c.n_inst = B.n_inst;
    return c;
}


// lane restrictions (Section 3.2 "Lane" set_lane_restriction): a restricted
// lane admits no new vehicle; a junction lane is closed when it or the road
// lane it leads into is restricted (vehicles already on it carry on)
static bool lane_restricted(const Build& B, int m) { return m < (int)B.restricted.size() && B.restricted[m]; }
static bool jl_open(const Build& B, int q) { return !lane_restricted(B, q) && !lane_restricted(B, B.jl_out[q]); }
// the road a junction lane leads to as the device tables hold it: -2 while closed
static int32_t jl_road_eff(const Build& B, int q) { return jl_open(B, q) ? B.jl_out_road[q] : -2; }

// lanes (bits) of origin road r a departing vehicle with next road nr may
// enter: unrestricted, and with an open junction lane toward nr (any lane
// when the route ends on r)
static uint32_t depart_mask(const Build& B, int r, int nr)
{
    const int lb = B.tile_lane_begin[r], nrl = B.tile_n_road[r];
    uint32_t m = 0u;
    for (int li = 0; li < nrl; ++li) {
        if (lane_restricted(B, lb + li)) continue;
        bool ok = nr < 0;
        for (int e = B.out_begin[lb + li]; e < B.out_begin[lb + li + 1] && !ok; ++e)
            ok = B.jl_out_road[B.out_jl[e]] == nr && jl_open(B, B.out_jl[e]);
        if (ok) m |= 1u << li;
    }
    return m;
}

// the next-road word of vehicle v's record on route position rp with rem
// roads after it (the trip's end position on its last road)
static int32_t next_word(const Build& B, int v, int rp, int rem)
{
    if (rem > 0) return B.route[rp + 1];
    const int r = B.route[rp];
    return end_word(B.vend[v], B.lane_len[B.tile_lane_begin[r]]);
}

// the device's static record of lane m
static LaneInfo lane_info_of(const Build& B, int m)
{
    LaneInfo L;
    L.base = B.lane_base[m];
    L.cap = B.lane_cap[m];
    L.len = B.lane_len[m];
    L.lim = B.lane_lim[m];
    L.jl_out = B.jl_out[m];
    L.jl_out_road = B.jl_out[m] >= 0 ? jl_road_eff(B, m) : B.jl_out_road[m];
    L.jl_junc = B.jl_junc[m];
    L.green_mask = B.jl_green_mask[m];
    L.jl_ext = B.jl_ext[m];
    L.jl_in_local = B.jl_in_local[m];
    L.flags = B.jl_out[m] < 0 && lane_restricted(B, m) ? 1 : 0;
    L.pad1 = 0;
    return L;
}

int build_tables(const tsim_network* net, const tsim_trips* tr, const tsim_params* prm, Build& B, std::string* err)
{
    if (!net || !tr || !prm) return fail(err, TSIM_EINVAL, "null network, trips or params");
    const int R = net->n_roads, NJ = net->n_junctions, NJL = net->n_jlanes, N = tr->n_vehicles;
    if (R <= 0 || NJ <= 0 || NJL < 0 || N < 0) return fail(err, TSIM_EINVAL, "bad sizes");
    if (!net->road_from || !net->road_to || !net->road_lane_begin || !net->road_length || !net->road_limit ||
        (NJL && (!net->jl_in_lane || !net->jl_out_lane || !net->jl_length || !net->jl_limit)) ||
        !net->junc_phase_begin || !net->junc_policy || !tr->route_begin || (N && (!tr->depart_time || !tr->route_roads ||
        !tr->v0_factor || !tr->length)))
        return fail(err, TSIM_EINVAL, "null array in network or trips");
    if (!(prm->dt > 0 && prm->a_max > 0 && prm->b_comf > 0 && prm->s0 >= 0 && prm->delta > 0 && prm->a_emerg > 0 &&
          prm->p_max >= prm->p_min && prm->p_min >= 0 && prm->p_max <= 1))
        return fail(err, TSIM_EINVAL, "invalid model parameters");
    B.R = R;
    B.NJ = NJ;
    B.NJL = NJL;
    B.N = N;
    if (net->road_lane_begin[0] != 0) return fail(err, TSIM_EINVAL, "road_lane_begin[0] must be 0");
    for (int r = 0; r < R; ++r) {
        const int nl = net->road_lane_begin[r + 1] - net->road_lane_begin[r];
        if (nl <= 0 || nl > kMaxRoadLanes) return fail(err, TSIM_EINVAL, "road " + std::to_string(r) + ": 1..32 lanes");
        if (net->road_from[r] < 0 || net->road_from[r] >= NJ || net->road_to[r] < 0 || net->road_to[r] >= NJ)
            return fail(err, TSIM_EINVAL, "road junction id out of range");
        if (!(net->road_length[r] > 0) || !(net->road_limit[r] > 0)) return fail(err, TSIM_EINVAL, "road length/limit");
    }
    const int NRL = net->road_lane_begin[R];
    B.NRL = NRL;
    B.NL = NRL + NJL;
    std::vector<int32_t> road_of(NRL);
    for (int r = 0; r < R; ++r)
        for (int l = net->road_lane_begin[r]; l < net->road_lane_begin[r + 1]; ++l) road_of[l] = r;
    std::unordered_set<long long> movement;    // (in road, out road)
    std::unordered_set<long long> lane_target; // (in lane, out road), must be unique
    for (int q = 0; q < NJL; ++q) {
        const int a = net->jl_in_lane[q], b = net->jl_out_lane[q];
        if (a < 0 || a >= NRL || b < 0 || b >= NRL) return fail(err, TSIM_EINVAL, "junction lane endpoints");
        if (net->road_to[road_of[a]] != net->road_from[road_of[b]])
            return fail(err, TSIM_EINVAL, "junction lane " + std::to_string(q) + " does not join its roads at a junction");
        if (!(net->jl_length[q] > 0) || !(net->jl_limit[q] > 0)) return fail(err, TSIM_EINVAL, "junction lane length/limit");
        movement.insert((long long)road_of[a] * R + road_of[b]);
        if (!lane_target.insert((long long)a * R + road_of[b]).second)
            return fail(err, TSIM_EINVAL, "two junction lanes from one lane into one road");
    }
    // trips
    float Lmin = 1e30f, fmax_ = 0.0f;
    if (tr->route_begin[0] != 0) return fail(err, TSIM_EINVAL, "route_begin[0] must be 0");
    for (int i = 0; i < N; ++i) {
        const int b = tr->route_begin[i], e = tr->route_begin[i + 1];
        if (e <= b) return fail(err, TSIM_EINVAL, "empty route of vehicle " + std::to_string(i));
        for (int k = b; k < e; ++k) {
            const int r = tr->route_roads[k];
            if (r < 0 || r >= R) return fail(err, TSIM_EINVAL, "route road out of range");
            if (k + 1 < e && !movement.count((long long)r * R + tr->route_roads[k + 1]))
                return fail(err, TSIM_EINVAL, "vehicle " + std::to_string(i) + ": consecutive route roads not connected");
        }
        if (!(tr->length[i] > 0) || !(tr->v0_factor[i] > 0) || !(tr->depart_time[i] >= 0))
            return fail(err, TSIM_EINVAL, "vehicle length/factor/departure");
        if (tr->end_s && !(tr->end_s[i] < 0.0f) && !(tr->end_s[i] > 0.0f && tr->end_s[i] <= net->road_length[tr->route_roads[e - 1]]))
            return fail(err, TSIM_EINVAL, "vehicle " + std::to_string(i) + ": end position beyond its last road");
        if (tr->start_s && !(tr->start_s[i] < net->road_length[tr->route_roads[b]]))
            return fail(err, TSIM_EINVAL, "vehicle " + std::to_string(i) + ": start position not before its origin road's end");
        Lmin = std::min(Lmin, tr->length[i]);
        fmax_ = std::max(fmax_, tr->v0_factor[i]);
    }
    if (N == 0) Lmin = 1.0f;
    // one lane-end crossing per step: every lane longer than the farthest one-step move
    const double reach = 0.5 * prm->a_max * prm->dt * prm->dt;
    for (int r = 0; r < R; ++r)
        if (net->road_length[r] <= fmax_ * net->road_limit[r] * prm->dt + reach)
            return fail(err, TSIM_EINVAL, "road " + std::to_string(r) + " shorter than one step of travel");
    for (int q = 0; q < NJL; ++q)
        if (net->jl_length[q] <= fmax_ * net->jl_limit[q] * prm->dt + reach)
            return fail(err, TSIM_EINVAL, "junction lane " + std::to_string(q) + " shorter than one step of travel");
    // junctions and phases
    if (net->junc_phase_begin[0] != 0) return fail(err, TSIM_EINVAL, "junc_phase_begin[0] must be 0");
    const int NP = net->junc_phase_begin[NJ];
    if (NP && (!net->phase_duration || !net->phase_green_begin || !net->phase_green_jl))
        return fail(err, TSIM_EINVAL, "null phase arrays");
    std::vector<int32_t> jl_junc_ext(NJL);
    for (int q = 0; q < NJL; ++q) jl_junc_ext[q] = net->road_to[road_of[net->jl_in_lane[q]]];
    std::vector<uint32_t> mask_ext(NJL, 0u);
    B.junc_cycle.assign(NJ, 0.0);
    for (int j = 0; j < NJ; ++j) {
        const int b = net->junc_phase_begin[j], e = net->junc_phase_begin[j + 1];
        if (e < b || e - b > kMaxPhases) return fail(err, TSIM_EINVAL, "junction " + std::to_string(j) + ": 0..32 phases");
        const int pol = net->junc_policy[j];
        if (pol < 0 || pol > 3) return fail(err, TSIM_EINVAL, "bad policy");
        if (pol == TSIM_POLICY_MAX_PRESSURE && e > b && !(net->phase_duration[b] > 0))
            return fail(err, TSIM_EINVAL, "max-pressure junction with a non-positive first phase duration");
        double cyc = 0.0;
        for (int p = b; p < e; ++p) {
            if (pol == TSIM_POLICY_FIXED_TIME && !(net->phase_duration[p] > 0))
                return fail(err, TSIM_EINVAL, "non-positive phase duration");
            cyc += net->phase_duration[p];
            for (int g = net->phase_green_begin[p]; g < net->phase_green_begin[p + 1]; ++g) {
                const int q = net->phase_green_jl[g];
                if (q < 0 || q >= NJL || jl_junc_ext[q] != j)
                    return fail(err, TSIM_EINVAL, "phase lists a junction lane of another junction");
                mask_ext[q] |= 1u << (p - b);
            }
        }
        B.junc_cycle[j] = cyc;
    }
    B.junc_phase_begin.assign(net->junc_phase_begin, net->junc_phase_begin + NJ + 1);
    B.phase_dur.assign(NP, 0.0f);
    for (int p = 0; p < NP; ++p) B.phase_dur[p] = net->phase_duration[p];
    B.junc_policy.assign(net->junc_policy, net->junc_policy + NJ);

    // internal lane numbering: tile r = road lanes of r, then junction lanes
    // leaving r in external order
    std::vector<std::vector<int>> jl_of_road(R);
    for (int q = 0; q < NJL; ++q) jl_of_road[road_of[net->jl_in_lane[q]]].push_back(q);
    B.tile_lane_begin.assign(R + 1, 0);
    B.tile_n_road.assign(R, 0);
    B.int_of_ext.assign(B.NL, -1);
    B.ext_of_int.assign(B.NL, -1);
    int nxt = 0;
    for (int r = 0; r < R; ++r) {
        B.tile_lane_begin[r] = nxt;
        const int nl = net->road_lane_begin[r + 1] - net->road_lane_begin[r];
        B.tile_n_road[r] = nl;
        if (nl + (int)jl_of_road[r].size() > kMaxTileLanes)
            return fail(err, TSIM_EINVAL, "road " + std::to_string(r) + ": more than 64 lanes with its junction lanes");
        for (int l = net->road_lane_begin[r]; l < net->road_lane_begin[r + 1]; ++l) {
            B.int_of_ext[l] = nxt;
            B.ext_of_int[nxt] = l;
            nxt++;
        }
        for (int q : jl_of_road[r]) {
            B.int_of_ext[NRL + q] = nxt;
            B.ext_of_int[nxt] = NRL + q;
            nxt++;
        }
    }
    B.tile_lane_begin[R] = nxt;
    const int NL = B.NL;
    B.lane_len.assign(NL, 0.f);
    B.lane_lim.assign(NL, 0.f);
    B.lane_cap.assign(NL, 0);
    B.lane_base.assign(NL, 0u);
    B.lane_tile.assign(NL, 0);
    B.lane_local.assign(NL, 0);
    B.jl_out.assign(NL, -1);
    B.jl_junc.assign(NL, 0);
    B.jl_ext.assign(NL, -1);
    B.jl_in_local.assign(NL, -1);
    B.jl_out_road.assign(NL, -1);
    B.jl_green_mask.assign(NL, 0u);
    uint64_t slots = 0;
    for (int r = 0; r < R; ++r) {
        for (int m = B.tile_lane_begin[r]; m < B.tile_lane_begin[r + 1]; ++m) {
            const int e = B.ext_of_int[m];
            B.lane_tile[m] = r;
            B.lane_local[m] = m - B.tile_lane_begin[r];
            if (e < NRL) {
                B.lane_len[m] = net->road_length[r];
                B.lane_lim[m] = net->road_limit[r];
            } else {
                const int q = e - NRL;
                B.lane_len[m] = net->jl_length[q];
                B.lane_lim[m] = net->jl_limit[q];
                B.jl_out[m] = B.int_of_ext[net->jl_out_lane[q]];
                B.jl_junc[m] = jl_junc_ext[q];
                B.jl_ext[m] = q;
                B.jl_in_local[m] = net->jl_in_lane[q] - net->road_lane_begin[r];
                B.jl_out_road[m] = road_of[net->jl_out_lane[q]];
                B.jl_green_mask[m] = mask_ext[q];
            }
            const int cap = (int)std::floor(B.lane_len[m] / Lmin) + 2;
            B.lane_cap[m] = cap;
            B.lane_base[m] = (uint32_t)slots;
            slots += (uint64_t)cap;
        }
    }
    if (slots >= (1ull << 31)) return fail(err, TSIM_EINVAL, "network too large for 32-bit slot indices");
    B.slots = slots;
    // connections per internal road lane
    B.out_begin.assign(NL + 1, 0);
    B.feed_begin.assign(NL + 1, 0);
    for (int q = 0; q < NJL; ++q) {
        B.out_begin[B.int_of_ext[net->jl_in_lane[q]] + 1]++;
        B.feed_begin[B.int_of_ext[net->jl_out_lane[q]] + 1]++;
    }
    for (int m = 0; m < NL; ++m) {
        B.out_begin[m + 1] += B.out_begin[m];
        B.feed_begin[m + 1] += B.feed_begin[m];
    }
    B.out_jl.assign(NJL, 0);
    B.feed_jl.assign(NJL, 0);
    {
        std::vector<int> fo(NL, 0), ff(NL, 0);
        for (int q = 0; q < NJL; ++q) {  // external order = feeder priority order
            const int a = B.int_of_ext[net->jl_in_lane[q]], b = B.int_of_ext[net->jl_out_lane[q]];
            B.out_jl[B.out_begin[a] + fo[a]++] = B.int_of_ext[NRL + q];
            B.feed_jl[B.feed_begin[b] + ff[b]++] = B.int_of_ext[NRL + q];
        }
    }
    // movements of each junction for the max-pressure policy
    B.mp_begin.assign(NJ + 1, 0);
    for (int q = 0; q < NJL; ++q) B.mp_begin[jl_junc_ext[q] + 1]++;
    for (int j = 0; j < NJ; ++j) B.mp_begin[j + 1] += B.mp_begin[j];
    B.mp_mov.assign(4 * (size_t)NJL, 0);
    {
        std::vector<int> fill(NJ, 0);
        for (int q = 0; q < NJL; ++q) {
            const int k = B.mp_begin[jl_junc_ext[q]] + fill[jl_junc_ext[q]]++;
            B.mp_mov[4 * k] = B.int_of_ext[net->jl_in_lane[q]];
            B.mp_mov[4 * k + 1] = B.int_of_ext[net->jl_out_lane[q]];
            B.mp_mov[4 * k + 2] = (int32_t)mask_ext[q];
        }
    }
    // vehicles and departure queues (tau, id) per origin road
    B.tau.assign(tr->depart_time, tr->depart_time + N);
    B.vf.assign(tr->v0_factor, tr->v0_factor + N);
    B.vlen.assign(tr->length, tr->length + N);
    if (tr->end_s) B.vend.assign(tr->end_s, tr->end_s + N);
    else B.vend.assign(N, -1.0f);
    B.vstart.assign(N, 0.0f);
    if (tr->start_s)
        for (int i = 0; i < N; ++i) B.vstart[i] = tr->start_s[i] > 0.0f ? tr->start_s[i] : 0.0f;
    B.route_begin.assign(tr->route_begin, tr->route_begin + N + 1);
    B.route.assign(tr->route_roads, tr->route_roads + tr->route_begin[N]);
    B.rstart.assign(B.route_begin.begin(), B.route_begin.begin() + N);
    B.rlen.resize(N);
    for (int i = 0; i < N; ++i) B.rlen[i] = B.route_begin[i + 1] - B.route_begin[i];
    B.q_begin.assign(R + 1, 0);
    for (int i = 0; i < N; ++i) B.q_begin[B.route[B.route_begin[i]] + 1]++;
    for (int r = 0; r < R; ++r) B.q_begin[r + 1] += B.q_begin[r];
    B.q_veh.assign(N, 0);
    {
        std::vector<int> fill(R, 0);
        for (int i = 0; i < N; ++i) {
            const int r = B.route[B.route_begin[i]];
            B.q_veh[B.q_begin[r] + fill[r]++] = i;
        }
        for (int r = 0; r < R; ++r)
            std::sort(B.q_veh.begin() + B.q_begin[r], B.q_veh.begin() + B.q_begin[r + 1], [&](int a, int b) {
                return B.tau[a] < B.tau[b] || (B.tau[a] == B.tau[b] && a < b);
            });
        B.q_mask.assign(N, 0u);
        for (int r = 0; r < R; ++r) {
            for (int k = B.q_begin[r]; k < B.q_begin[r + 1]; ++k) {
                const int v = B.q_veh[k];
                const int rb = B.route_begin[v];
                B.q_mask[k] = depart_mask(B, r, B.route_begin[v + 1] - rb > 1 ? B.route[rb + 1] : -1);
            }
        }
    }
    count_tiles(B);
    return TSIM_OK;
}

// instance metadata for a single network
void single_instance(Build& B, const tsim_params* prm)
{
    B.n_inst = 1;
    B.tile_inst.assign(B.R, 0);
    B.junc_inst.assign(B.NJ, 0);
    B.inst_vbase.assign(1, 0);
    B.inst_key = {(uint32_t)prm->seed, (uint32_t)(prm->seed >> 32)};
    B.inst_t0.assign(1, 0);
    B.road_off = {0, B.R};
    B.junc_off = {0, B.NJ};
    B.rl_off = {0, B.NRL};
    B.jl_off = {0, B.NJL};
    B.veh_off = {0, B.N};
}

// the disjoint union of several instances as one network and trip table
struct Union {
    std::vector<int32_t> road_from, road_to, road_lane_begin, jl_in, jl_out, junc_phase_begin, phase_green_begin,
        phase_green_jl, junc_policy, route_begin, route_roads;
    std::vector<float> road_length, road_limit, jl_length, jl_limit, phase_duration, depart, v0f, vlen, vend, vstart;
    tsim_network net{};
    tsim_trips trips{};
    std::vector<int> road_off, junc_off, rl_off, jl_off, veh_off;
};

int make_union(const tsim_network* nets, const tsim_trips* trips, const tsim_params* prm, int n, Union& U,
               std::string* err)
{
    if (!nets || !trips || !prm || n <= 0) return fail(err, TSIM_EINVAL, "null or empty batch");
    U.road_off.assign(1, 0);
    U.junc_off.assign(1, 0);
    U.rl_off.assign(1, 0);
    U.jl_off.assign(1, 0);
    U.veh_off.assign(1, 0);
    U.road_lane_begin.assign(1, 0);
    U.junc_phase_begin.assign(1, 0);
    U.phase_green_begin.assign(1, 0);
    U.route_begin.assign(1, 0);
    for (int k = 0; k < n; ++k) {
        const tsim_network& N = nets[k];
        const tsim_trips& T = trips[k];
        const tsim_params& P = prm[k];
        const tsim_params& P0 = prm[0];
        if (P.dt != P0.dt || P.T != P0.T || P.a_max != P0.a_max || P.b_comf != P0.b_comf || P.s0 != P0.s0 ||
            P.delta != P0.delta || P.politeness != P0.politeness || P.a_th != P0.a_th || P.b_safe != P0.b_safe ||
            P.p_max != P0.p_max || P.p_min != P0.p_min || P.a_emerg != P0.a_emerg)
            return fail(err, TSIM_EINVAL, "batch instances must share every parameter but the seed");
        if (N.n_roads <= 0 || N.n_junctions <= 0 || !N.road_lane_begin || !N.junc_phase_begin || !T.route_begin ||
            T.n_vehicles < 0 || N.n_jlanes < 0)
            return fail(err, TSIM_EINVAL, "instance " + std::to_string(k) + ": bad sizes");
        const int ro = U.road_off.back(), jo = U.junc_off.back(), lo = U.rl_off.back(), qo = U.jl_off.back(),
                  vo = U.veh_off.back();
        const int nrl = N.road_lane_begin[N.n_roads];
        const int np = N.junc_phase_begin[N.n_junctions];
        const int pgo = (int)U.phase_duration.size();
        const int go = U.phase_green_begin.back();
        for (int r = 0; r < N.n_roads; ++r) {
            U.road_from.push_back(N.road_from[r] + jo);
            U.road_to.push_back(N.road_to[r] + jo);
            U.road_lane_begin.push_back(N.road_lane_begin[r + 1] + lo);
            U.road_length.push_back(N.road_length[r]);
            U.road_limit.push_back(N.road_limit[r]);
        }
        for (int q = 0; q < N.n_jlanes; ++q) {
            U.jl_in.push_back(N.jl_in_lane[q] + lo);
            U.jl_out.push_back(N.jl_out_lane[q] + lo);
            U.jl_length.push_back(N.jl_length[q]);
            U.jl_limit.push_back(N.jl_limit[q]);
        }
        for (int j = 0; j < N.n_junctions; ++j) {
            U.junc_phase_begin.push_back(N.junc_phase_begin[j + 1] + pgo);
            U.junc_policy.push_back(N.junc_policy[j]);
        }
        for (int p = 0; p < np; ++p) {
            U.phase_duration.push_back(N.phase_duration[p]);
            U.phase_green_begin.push_back(N.phase_green_begin[p + 1] + go);
        }
        for (int g = 0; g < (np ? N.phase_green_begin[np] : 0); ++g) U.phase_green_jl.push_back(N.phase_green_jl[g] + qo);
        const int rbo = U.route_begin.back();
        for (int i = 0; i < T.n_vehicles; ++i) {
            U.route_begin.push_back(T.route_begin[i + 1] + rbo);
            U.depart.push_back(T.depart_time[i]);
            U.v0f.push_back(T.v0_factor[i]);
            U.vlen.push_back(T.length[i]);
            U.vend.push_back(T.end_s ? T.end_s[i] : -1.0f);
            U.vstart.push_back(T.start_s ? T.start_s[i] : 0.0f);
        }
        for (int e = 0; e < T.route_begin[T.n_vehicles]; ++e) U.route_roads.push_back(T.route_roads[e] + ro);
        U.road_off.push_back(ro + N.n_roads);
        U.junc_off.push_back(jo + N.n_junctions);
        U.rl_off.push_back(lo + nrl);
        U.jl_off.push_back(qo + N.n_jlanes);
        U.veh_off.push_back(vo + T.n_vehicles);
    }
    tsim_network& N = U.net;
    N.n_junctions = U.junc_off.back();
    N.n_roads = U.road_off.back();
    N.road_from = U.road_from.data();
    N.road_to = U.road_to.data();
    N.road_lane_begin = U.road_lane_begin.data();
    N.road_length = U.road_length.data();
    N.road_limit = U.road_limit.data();
    N.n_jlanes = U.jl_off.back();
    N.jl_in_lane = U.jl_in.data();
    N.jl_out_lane = U.jl_out.data();
    N.jl_length = U.jl_length.data();
    N.jl_limit = U.jl_limit.data();
    N.junc_phase_begin = U.junc_phase_begin.data();
    N.phase_duration = U.phase_duration.data();
    N.phase_green_begin = U.phase_green_begin.data();
    N.phase_green_jl = U.phase_green_jl.data();
    N.junc_policy = U.junc_policy.data();
    tsim_trips& T = U.trips;
    T.n_vehicles = U.veh_off.back();
    T.depart_time = U.depart.data();
    T.route_begin = U.route_begin.data();
    T.route_roads = U.route_roads.data();
    T.v0_factor = U.v0f.data();
    T.length = U.vlen.data();
    T.end_s = U.vend.data();
    T.start_s = U.vstart.data();
    return TSIM_OK;
}

// instance metadata of a batch built from a union
void batch_instances(Build& B, const Union& U, const tsim_params* prm, int n)
{
    B.n_inst = n;
    B.road_off = U.road_off;
    B.junc_off = U.junc_off;
    B.rl_off = U.rl_off;
    B.jl_off = U.jl_off;
    B.veh_off = U.veh_off;
    B.tile_inst.assign(B.R, 0);
    B.junc_inst.assign(B.NJ, 0);
    B.inst_vbase.assign(n, 0);
    B.inst_key.assign(2 * n, 0u);
    B.inst_t0.assign(n, 0);
    for (int k = 0; k < n; ++k) {
        for (int r = U.road_off[k]; r < U.road_off[k + 1]; ++r) B.tile_inst[r] = k;
        for (int j = U.junc_off[k]; j < U.junc_off[k + 1]; ++j) B.junc_inst[j] = k;
        B.inst_vbase[k] = U.veh_off[k];
        B.inst_key[2 * k] = (uint32_t)prm[k].seed;
        B.inst_key[2 * k + 1] = (uint32_t)(prm[k].seed >> 32);
    }
    // tiles grouped by instance within each class (each workgroup takes a
    // contiguous run), larger tiles first within an instance
    count_tiles(B);
}

}  // namespace

struct tsim_handle {
    hipStream_t stream = nullptr;
    char* arena = nullptr;
    size_t arena_bytes = 0;
    DevNet D{};                      // host copy of the device view
    DevNet* d_net = nullptr;         // device copy (kernel argument)
    Build B;
    int32_t* d_lane_ext = nullptr;   // internal -> external lane id
    int32_t* d_io_i0 = nullptr;      // staging: export lane / import slots
    int32_t* d_io_i1 = nullptr;      // staging: export route pos
    int32_t* d_io_i2 = nullptr;      // staging: export rank
    float* d_io_f0 = nullptr;
    float* d_io_f1 = nullptr;
    VehRec* d_io_rec = nullptr;      // staging: import records
    int32_t* d_io_ph = nullptr;      // staging: phase updates (2 slots of 2 x NJ)
    int32_t* d_io_lane = nullptr;    // staging: lane updates (NL ids, then NL values)
    unsigned long long* d_traj_n = nullptr;   // trajectory records appended so far
    // areas of interest (tsim_set_aois), per instance: the caller's buffer
    // (per-vehicle origin and destination AOI ids, then the count slots) and
    // the number of AOIs
    struct AoiSet {
        int32_t* d = nullptr;
        int n = 0;
    };
    std::vector<AoiSet> aois;
    TrajRec* traj = nullptr;         // caller's trajectory buffer (device), traj_cap records
    long long traj_cap = 0;
    int traj_every = 0;              // 0: not recording
    int32_t* h_pin[2] = {nullptr, nullptr};   // pinned host staging of the two slots
    hipEvent_t pin_ev[2] = {nullptr, nullptr};
    bool pin_used[2] = {false, false};
    int pin_slot = 0;
    // kernel timing (tsim_set_profiling)
    bool prof = false;
    std::vector<hipEvent_t> ev[2];   // start/stop pairs per kernel
    int ev_used[2] = {0, 0};
    double ms[2] = {0.0, 0.0};
    long long launches[2] = {0, 0};
    // captured step chunks (tsim_set_graph_steps): one graph of `graph_chunk`
    // steps, replayed; the remainder of a call is launched directly
    int graph_chunk = 0;
    hipGraphExec_t graph = nullptr;
    hipStream_t cap_stream = nullptr;   // capture only (the caller's stream may be the null stream)
    PassStreams ps;                     // tsim_set_concurrency
    int res[kNumSched + 4] = {};        // resident workgroups: grouped pass per schedule, wide, huge, pipelined wide, tiny
    Caps cap;                           // sizes the arena is laid out for
    tsim_params params{};               // model parameters (batches: shared by every instance but the seed)
    int device = 0;                     // GPU the handle was created on
    std::vector<char> removed;          // batches: instances taken out by tsim_batch_remove
    std::string err;
};

namespace {

size_t align_up(size_t x) { return (x + 255) & ~(size_t)255; }

// every device array of a handle, in arena order
std::vector<Region> regions(tsim_handle* h, bool assign)
{
    const Caps& c = h->cap;
    DevNet& D = h->D;
    const size_t NL = c.NL, R = c.R, NJ = c.NJ, N = c.N, S = c.S, NJL = c.NJL;
    std::vector<Region> v;
    auto add = [&](void* field, size_t bytes) { v.push_back({(void**)field, bytes}); };
    (void)assign;
    add(&D.tile_lane_begin, (R + 1) * 4);
    add(&D.tile_n_road, std::max<size_t>(R, 1) * 4);
    add(&D.lane_info, std::max<size_t>(NL, 1) * sizeof(LaneInfo));
    add(&D.lane_len, std::max<size_t>(NL, 1) * 4);
    add(&D.lane_lim, std::max<size_t>(NL, 1) * 4);
    add(&D.lane_base, std::max<size_t>(NL, 1) * 4);
    add(&D.lane_cap, std::max<size_t>(NL, 1) * 4);
    add(&D.lane_tile, std::max<size_t>(NL, 1) * 4);
    add(&D.lane_local, std::max<size_t>(NL, 1) * 4);
    add(&D.jl_out, std::max<size_t>(NL, 1) * 4);
    add(&D.jl_junc, std::max<size_t>(NL, 1) * 4);
    add(&D.jl_green_mask, std::max<size_t>(NL, 1) * 4);
    add(&D.jl_ext, std::max<size_t>(NL, 1) * 4);
    add(&D.jl_in_local, std::max<size_t>(NL, 1) * 4);
    add(&D.jl_out_road, std::max<size_t>(NL, 1) * 4);
    add(&D.out_begin, (NL + 1) * 4);
    add(&D.out_jl, std::max<size_t>(NJL, 1) * 4);
    add(&D.out_pair, std::max<size_t>(NJL, 1) * 8);
    add(&D.feed_begin, (NL + 1) * 4);
    add(&D.feed_jl, std::max<size_t>(NJL, 1) * 4);
    add(&D.junc_phase_begin, (NJ + 1) * 4);
    add(&D.mp_begin, (NJ + 1) * 4);
    add(&D.mp_mov, std::max<size_t>(NJL, 1) * 16);
    add(&D.phase_dur, std::max<size_t>(c.P, 1) * 4);
    add(&D.junc_cycle, std::max<size_t>(NJ, 1) * 8);
    add(&D.junc_policy, std::max<size_t>(NJ, 1) * 4);
    add(&D.junc_manual, std::max<size_t>(NJ, 1) * 4);
    add(&D.junc_cur, std::max<size_t>(NJ, 1) * 4);
    add(&D.tau, std::max<size_t>(N, 1) * 4);
    add(&D.route_begin, (N + 1) * 4);
    add(&D.route, std::max<size_t>(c.E, 1) * 4);
    add(&D.vf, std::max<size_t>(N, 1) * 4);
    add(&D.vlen, std::max<size_t>(N, 1) * 4);
    add(&D.vend, std::max<size_t>(N, 1) * 4);
    add(&D.vstart, std::max<size_t>(N, 1) * 4);
    add(&D.status, std::max<size_t>(N, 1) * 4);
    add(&D.finish_step, std::max<size_t>(N, 1) * 4);
    add(&D.q_begin, (R + 1) * 4);
    add(&D.q_rec, std::max<size_t>(N, 1) * sizeof(QRec));
    add(&D.q_head, std::max<size_t>(R, 1) * 4);
    add(&D.slab0, std::max<size_t>(S, 1) * sizeof(VehRec));
    add(&D.slab1, std::max<size_t>(S, 1) * sizeof(VehRec));
    add(&D.sum0, std::max<size_t>(NL, 1) * sizeof(LaneSum));
    add(&D.sum1, std::max<size_t>(NL, 1) * sizeof(LaneSum));
    add(&D.tile_n0, std::max<size_t>(R, 1) * 4);
    add(&D.tile_n1, std::max<size_t>(R, 1) * 4);
    add(&D.inbox, std::max<size_t>(NL, 1) * sizeof(VehRec));
    add(&D.inbox_flag, std::max<size_t>(NL, 1) * 4);
    add(&D.sh_gmask, std::max<size_t>(S, 1) * 4);
    add(&D.sh_jq, std::max<size_t>(S, 1) * 4);
    add(&D.sh_aown, std::max<size_t>(S, 1) * 4);
    add(&D.sh_merge, std::max<size_t>(S, 1) * 4);
    add(&D.sh_lrear, std::max<size_t>(S, 1) * 4);
    add(&D.sh_lv, std::max<size_t>(S, 1) * 4);
    add(&D.sh_nx, std::max<size_t>(S, 1) * 4);
    add(&D.sh_nv, std::max<size_t>(S, 1) * 4);
    add(&D.sh_kind, std::max<size_t>(S, 1) * 4);
    add(&D.sh_nlane, std::max<size_t>(S, 1) * 4);
    add(&D.sh_pref, std::max<size_t>(S, 1) * 4);
    add(&D.road_speed, std::max<size_t>(R, 1) * 4);
    add(&D.lane_wait, std::max<size_t>(NL, 1) * 4);
    add(&D.list_small, std::max<size_t>(R, 1) * 4);
    add(&D.list_big, std::max<size_t>(R, 1) * 4);
    add(&D.list_huge, std::max<size_t>(R, 1) * 4);
    add(&D.list_tiny, std::max<size_t>(R, 1) * 4);
    add(&D.list_med, std::max<size_t>(R, 1) * 4);
    add(&D.list_large, std::max<size_t>(R, 1) * 4);
    add(&D.list_cnt, 2 * kNumLists * kCntStride * 4);
    add(&D.part, (size_t)std::max<long long>(c.G, 1) * sizeof(WGPartial));
    add(&D.ustep, 8);
    add(&D.fold_flag, 24);
    add(&D.part2, (size_t)kFoldWGs * sizeof(WGPartial));
    add(&D.met, (size_t)std::max<long long>(c.n_inst, 1) * sizeof(DevMetrics));
    add(&D.tile_inst, std::max<size_t>(R, 1) * 4);
    add(&D.junc_inst, std::max<size_t>(NJ, 1) * 4);
    add(&D.inst_vbase, (size_t)std::max<long long>(c.n_inst, 1) * 4);
    add(&D.inst_key, (size_t)std::max<long long>(c.n_inst, 1) * 8);
    add(&D.inst_t0, (size_t)std::max<long long>(c.n_inst, 1) * 8);
    add(&D.inst_end, (size_t)std::max<long long>(c.n_inst, 1) * 8);
    add(&D.inst_acc, (size_t)std::max<long long>(c.n_inst, 1) * sizeof(WGPartial));
    add(&D.gstep, 8);
    add(&h->d_lane_ext, std::max<size_t>(NL, 1) * 4);
    add(&h->d_io_i0, std::max<size_t>(N, 1) * 4);
    add(&h->d_io_i1, std::max<size_t>(N, 1) * 4);
    add(&h->d_io_i2, std::max<size_t>(N, 1) * 4);
    add(&h->d_io_f0, std::max<size_t>(N, 1) * 4);
    add(&h->d_io_f1, std::max<size_t>(N, 1) * 4);
    add(&h->d_io_rec, std::max<size_t>(N, 1) * sizeof(VehRec));
    add(&h->d_io_ph, 4 * std::max<size_t>(NJ, 1) * 4);
    add(&h->d_io_lane, 2 * std::max<size_t>(NL, 1) * 4);
    add(&h->d_traj_n, 8);
    add(&h->d_net, sizeof(DevNet));
    return v;
}

size_t arena_size(tsim_handle* h)
{
    size_t s = 0;
    for (auto& r : regions(h, false)) s += align_up(r.bytes);
    return s;
}

int hip_fail(tsim_handle* h, hipError_t e, const char* what)
{
    std::string m = std::string(what) + ": " + hipGetErrorString(e);
    if (h) h->err = m;
    g_error = m;
    return TSIM_EDEVICE;
}

#define HIPCHK(h, call)                                   \
    do {                                                  \
        hipError_t e_ = (call);                           \
        if (e_ != hipSuccess) return hip_fail(h, e_, #call); \
    } while (0)

template <class T>
hipError_t up(tsim_handle* h, T* dst, const std::vector<T>& src)
{
    if (src.empty()) return hipSuccess;
    return hipMemcpyAsync((void*)dst, src.data(), src.size() * sizeof(T), hipMemcpyHostToDevice, h->stream);
}

void fill_params(KParams& P, const tsim_params* p)
{
    P.dt = (float)p->dt;
    P.T = (float)p->T;
    P.a_max = (float)p->a_max;
    P.s0 = (float)p->s0;
    P.delta = (float)p->delta;
    P.p = (float)p->politeness;
    P.a_th = (float)p->a_th;
    P.b_safe = (float)p->b_safe;
    P.p_max = (float)p->p_max;
    P.p_min = (float)p->p_min;
    P.a_emerg = (float)p->a_emerg;
    P.inv_2sqrt_ab = (float)(1.0 / (2.0 * std::sqrt(p->a_max * p->b_comf)));
    P.reach = (float)(0.5 * p->a_max * p->dt * p->dt);
    P.dt_d = p->dt;
    P.key0 = (uint32_t)p->seed;
    P.key1 = (uint32_t)(p->seed >> 32);
    P.delta_is_4 = p->delta == 4.0 ? 1 : 0;
}

// whether the step launches k_signals (some junction may use MAX_PRESSURE);
// a captured graph that launches otherwise is dropped (recaptured on the next
// step)
void set_mp_any(tsim_handle* h, bool any)
{
    if ((h->D.mp_any != 0) == any) return;
    if (h->graph) {
        (void)hipStreamSynchronize(h->stream);
        (void)hipGraphExecDestroy(h->graph);
        h->graph = nullptr;
    }
    h->D.mp_any = any ? 1 : 0;
}

// index ranges of instance k of a batch inside the union (k = -1: the whole
// handle): roads (= tiles), junctions, vehicles, internal lanes, and the
// external road-lane and junction-lane ranges
struct Ranges {
    int r0, r1, j0, j1, v0, v1, m0, m1, rl0, nrl, jl0, njl;
};

Ranges ranges_of(const Build& B, int k)
{
    if (k < 0) return Ranges{0, B.R, 0, B.NJ, 0, B.N, 0, B.NL, 0, B.NRL, 0, B.NJL};
    Ranges g;
    g.r0 = B.road_off[k];
    g.r1 = B.road_off[k + 1];
    g.j0 = B.junc_off[k];
    g.j1 = B.junc_off[k + 1];
    g.v0 = B.veh_off[k];
    g.v1 = B.veh_off[k + 1];
    g.m0 = B.tile_lane_begin[g.r0];
    g.m1 = B.tile_lane_begin[g.r1];
    g.rl0 = B.rl_off[k];
    g.nrl = B.rl_off[k + 1] - g.rl0;
    g.jl0 = B.jl_off[k];
    g.njl = B.jl_off[k + 1] - g.jl0;
    return g;
}

// external lane id of the union from an instance-local one, and back
int union_lane(const Build& B, const Ranges& g, int l)
{
    return l < g.nrl ? g.rl0 + l : B.NRL + g.jl0 + (l - g.nrl);
}
int local_lane(const Build& B, const Ranges& g, int e)
{
    return e < B.NRL ? e - g.rl0 : (e - B.NRL - g.jl0) + g.nrl;
}

template <class T>
hipError_t up_at(tsim_handle* h, T* dst, const std::vector<T>& src)
{
    if (src.empty()) return hipSuccess;
    return hipMemcpyAsync((void*)dst, src.data(), src.size() * sizeof(T), hipMemcpyHostToDevice, h->stream);
}

// uploads the state of instance k (k = -1: the whole handle) from
// instance-local arrays: per-lane orders are rebuilt on the host.  With
// k = -1 the handle's step counter becomes `step`; otherwise the instance
// joins the batch's running step count with its own local step `step`
// (every array indexed by global step parity keeps working), after the
// pending step of the batch is folded.
int upload_state(tsim_handle* h, int k, int64_t step, const int32_t* status, const int32_t* lane_loc,
                 const int32_t* route_pos, const float* x, const float* v, const int32_t* finish_step,
                 const int32_t* pol, const int32_t* ph)
{
    Build& B = h->B;
    DevNet& D = h->D;
    const Ranges g = ranges_of(B, k);
    const int nv = g.v1 - g.v0, nm = g.m1 - g.m0, nr = g.r1 - g.r0, nj = g.j1 - g.j0;
    std::vector<std::vector<int>> per_lane(nm);
    const int nl_loc = g.nrl + g.njl;
    for (int il = 0; il < nv; ++il) {
        const int i = g.v0 + il;
        const int s = status[il];
        if (s < 0 || s > 2) return fail(&h->err, TSIM_EINVAL, "bad status");
        if (s == TSIM_ACTIVE) {
            const int l = lane_loc[il];
            if (l < 0 || l >= nl_loc) return fail(&h->err, TSIM_EINVAL, "active vehicle without a valid lane");
            const int rl = B.rlen[i];
            const int kk = route_pos[il];
            if (kk < 0 || kk >= rl) return fail(&h->err, TSIM_EINVAL, "route position out of range");
            const int m = B.int_of_ext[union_lane(B, g, l)];
            const int r = B.lane_tile[m];
            if (B.route[B.rstart[i] + kk] != r) return fail(&h->err, TSIM_EINVAL, "lane not on the current road");
            if (B.jl_out[m] >= 0 && (kk + 1 >= rl || B.jl_out_road[m] != B.route[B.rstart[i] + kk + 1]))
                return fail(&h->err, TSIM_EINVAL, "junction lane not toward the next road");
            if (!(x[il] >= 0.0f && x[il] <= B.lane_len[m]) || !(v[il] >= 0.0f))
                return fail(&h->err, TSIM_EINVAL, "position or speed out of range");
            per_lane[m - g.m0].push_back(i);
        }
        if (s == TSIM_FINISHED && finish_step[il] < 0) return fail(&h->err, TSIM_EINVAL, "finished without a finish step");
    }
    // the step from which the state is read: the handle's new step (k = -1)
    // or the batch's current global step
    long long gnow = step;
    if (k >= 0) {
        HIPCHK(h, launch_fold(h->D, h->stream));
        HIPCHK(h, hipMemcpyAsync(&gnow, D.gstep, sizeof(gnow), hipMemcpyDeviceToHost, h->stream));
        HIPCHK(h, hipStreamSynchronize(h->stream));
    }
    auto X = [&](int i) { return x[i - g.v0]; };
    auto V = [&](int i) { return v[i - g.v0]; };
    std::vector<uint32_t> slots;
    std::vector<VehRec> recs;
    const float INF = std::numeric_limits<float>::infinity();
    LaneSum empty;
    empty.cnt = 0;
    empty.rear = INF;
    empty.rear_v = 0.0f;
    empty.front_reach = -INF;
    empty.gate = 0;     // tag 0: stale for every step
    empty.fmax = 0;
    std::vector<LaneSum> sum(nm, empty);
    std::vector<LaneSum> sum_other(sum);
    std::vector<int32_t> tile_n(nr, 0), tile_zero(nr, 0);
    std::vector<float> road_speed(nr, -1.0f);
    std::vector<int32_t> lane_wait(nm, 0), inbox_zero(nm, 0);
    const float dtf = (float)h->D.P.dt, reachf = h->D.P.reach;
    for (int m = g.m0; m < g.m1; ++m) {
        auto& L = per_lane[m - g.m0];
        std::sort(L.begin(), L.end(), [&](int a, int b) { return X(a) > X(b) || (X(a) == X(b) && a < b); });
        if ((int)L.size() > B.lane_cap[m]) return fail(&h->err, TSIM_EINVAL, "lane over capacity (overlapping vehicles)");
        if (!L.empty()) {
            LaneSum& su = sum[m - g.m0];
            su.cnt = (int)L.size();
            const int f = L.front(), b = L.back();
            su.front_reach = X(f) + V(f) * dtf + reachf - B.lane_len[m];
            su.rear = X(b) - B.vlen[b];
            su.rear_v = V(b);
            tile_n[B.lane_tile[m] - g.r0] += su.cnt;
        }
        for (size_t c = 0; c < L.size(); ++c) {
            const int i = L[c];
            VehRec o;
            o.x = X(i);
            o.v = V(i);
            o.vid = i;
            o.len = B.vlen[i];
            o.f = B.vf[i];
            o.rp = B.rstart[i] + route_pos[i - g.v0];
            o.rem = B.rstart[i] + B.rlen[i] - o.rp - 1;
            o.nr = next_word(B, i, o.rp, o.rem);
            slots.push_back(B.lane_base[m] + (uint32_t)c);
            recs.push_back(o);
        }
    }
    // feeder gates of the current step from the junction-lane summaries,
    // tagged for the step that reads them (the other buffer's are written by
    // the update kernels with the next step's tag)
    std::vector<int> gmin(nm, kNoGate), fmx(nm, kNoFeeder);
    for (int q = g.m0; q < g.m1; ++q) {
        const int go = B.jl_out[q];
        if (go < 0 || sum[q - g.m0].cnt == 0) continue;
        const float fr = sum[q - g.m0].front_reach;
        fmx[go - g.m0] = std::max(fmx[go - g.m0], f2o(fr));
        if (fr > 0.0f) gmin[go - g.m0] = std::min(gmin[go - g.m0], B.jl_ext[q]);
    }
    for (int m = 0; m < nm; ++m) {
        if (fmx[m] != kNoFeeder) sum[m].fmax = fmax_key(gnow, fmx[m]);
        if (gmin[m] != kNoGate) sum[m].gate = gate_key(gnow, gmin[m]);
    }
    std::vector<int32_t> qhead(nr);
    for (int r = g.r0; r < g.r1; ++r) {
        int hd = B.q_begin[r];
        while (hd < B.q_begin[r + 1] && status[B.q_veh[hd] - g.v0] != TSIM_WAITING) hd++;
        qhead[r - g.r0] = hd;
    }
    const int k0 = k < 0 ? 0 : k, k1 = k < 0 ? B.n_inst : k + 1;
    std::vector<DevMetrics> Ms(k1 - k0);
    std::vector<long long> t0s(k1 - k0);
    for (int kk = k0; kk < k1; ++kk) {
        DevMetrics& M = Ms[kk - k0];
        std::memset(&M, 0, sizeof(M));
        t0s[kk - k0] = k < 0 ? 0 : gnow - step;
        M.step = step;
        for (int i = B.veh_off[kk]; i < B.veh_off[kk + 1]; ++i) {
            const int st = status[i - g.v0];
            if (st != TSIM_WAITING) M.departed++;
            if (st == TSIM_FINISHED) {
                M.finished++;
                const double tt = (double)(finish_step[i - g.v0] + 1) * h->D.P.dt_d - (double)B.tau[i];
                M.sum_tt_fx += llrint(tt * kTimeFx);
            }
        }
    }
    std::vector<WGPartial> zacc(k1 - k0);
    std::memset(zacc.data(), 0, zacc.size() * sizeof(WGPartial));
    std::vector<int32_t> st(status, status + nv), fs(finish_step, finish_step + nv);
    std::vector<int32_t> jp(pol, pol + nj), jm(ph, ph + nj);
    const bool odd = (gnow & 1) != 0;
    HIPCHK(h, up_at(h, (odd ? D.sum1 : D.sum0) + g.m0, sum));
    HIPCHK(h, up_at(h, (odd ? D.sum0 : D.sum1) + g.m0, sum_other));
    HIPCHK(h, up_at(h, (odd ? D.tile_n1 : D.tile_n0) + g.r0, tile_n));
    HIPCHK(h, up_at(h, (odd ? D.tile_n0 : D.tile_n1) + g.r0, tile_zero));
    HIPCHK(h, up_at(h, D.road_speed + g.r0, road_speed));
    HIPCHK(h, up_at(h, D.lane_wait + g.m0, lane_wait));
    HIPCHK(h, up_at(h, D.inbox_flag + g.m0, inbox_zero));
    HIPCHK(h, up_at(h, D.status + g.v0, st));
    HIPCHK(h, up_at(h, D.finish_step + g.v0, fs));
    HIPCHK(h, up_at(h, D.junc_policy + g.j0, jp));
    HIPCHK(h, up_at(h, D.junc_manual + g.j0, jm));
    const bool any_mp = std::any_of(jp.begin(), jp.end(), [](int32_t p) { return p == TSIM_POLICY_MAX_PRESSURE; });
    if (k < 0) set_mp_any(h, any_mp);
    else if (any_mp) set_mp_any(h, true);
    HIPCHK(h, up_at(h, D.q_head + g.r0, qhead));
    HIPCHK(h, up_at(h, D.met + k0, Ms));
    HIPCHK(h, up_at(h, D.inst_acc + k0, zacc));
    HIPCHK(h, up_at(h, (long long*)D.inst_t0 + k0, t0s));
    if (k < 0) {
        const long long gstep = step;
        const long long ustep = step - 1;   // the last step run (none folded yet)
        HIPCHK(h, hipMemsetAsync(D.fold_flag, 0, 24, h->stream));
        HIPCHK(h, hipMemsetAsync(D.list_cnt, 0, 2 * kNumLists * kCntStride * 4, h->stream));
        HIPCHK(h, hipMemcpyAsync(D.gstep, &gstep, sizeof(gstep), hipMemcpyHostToDevice, h->stream));
        HIPCHK(h, hipMemcpyAsync(D.ustep, &ustep, sizeof(ustep), hipMemcpyHostToDevice, h->stream));
    }
    if (!slots.empty()) {
        HIPCHK(h, hipMemcpyAsync(h->d_io_i0, slots.data(), slots.size() * 4, hipMemcpyHostToDevice, h->stream));
        HIPCHK(h, hipMemcpyAsync(h->d_io_rec, recs.data(), recs.size() * sizeof(VehRec), hipMemcpyHostToDevice, h->stream));
        HIPCHK(h, launch_import(h->d_net, h->D, (const uint32_t*)h->d_io_i0, h->d_io_rec, (int)slots.size(), h->stream));
    }
    HIPCHK(h, hipStreamSynchronize(h->stream));
    return TSIM_OK;
}

}  // namespace

extern "C" {

int tsim_footprint(const tsim_network* net, const tsim_trips* trips, const tsim_params* params, size_t* bytes_out)
{
    if (!bytes_out) return fail(nullptr, TSIM_EINVAL, "null bytes_out");
    tsim_handle tmp;
    int rc = build_tables(net, trips, params, tmp.B, nullptr);
    if (rc) return rc;
    single_instance(tmp.B, params);
    tmp.cap = caps_of(tmp.B);
    *bytes_out = arena_size(&tmp) + 256;
    return TSIM_OK;
}

static int create_impl(tsim_handle* h, const tsim_params* params, void* hip_stream, void* device_arena,
                       size_t arena_bytes, tsim_handle** out);

static void set_sched(tsim_handle* h, int sched)
{
    // the fused launch sizes every range by its own occupancy
    const bool fused = sched == kSchedFused;
    const int res_b = fused ? h->res[sched]
                      : (sched == kSched16x32P || sched == kSched8and16) ? h->res[kNumSched + 2]
                                                                          : h->res[kNumSched];
    const SchedGrid g = sched_grid(h->B, sched, h->res[sched], res_b, fused ? h->res[sched] : h->res[kNumSched + 1],
                                   fused ? h->res[sched] : h->res[kNumSched + 3]);
    h->D.sched = sched;
    h->D.GA = g.GA;
    h->D.GB = g.GB;
    h->D.GC = g.GC;
    h->D.GT = g.GT;
    h->D.GM = g.GM;
    h->D.GL = g.GL;
}

int tsim_create(const tsim_network* net, const tsim_trips* trips, const tsim_params* params, void* hip_stream,
                void* device_arena, size_t arena_bytes, tsim_handle** out)
{
    if (!out) return fail(nullptr, TSIM_EINVAL, "null out");
    *out = nullptr;
    if (!device_arena) return fail(nullptr, TSIM_EINVAL, "null arena");
    tsim_handle* h = new (std::nothrow) tsim_handle();
    if (!h) return fail(nullptr, TSIM_ENOMEM, "host allocation failed");
    int rc = build_tables(net, trips, params, h->B, &h->err);
    if (rc) {
        delete h;
        return rc;
    }
    single_instance(h->B, params);
    h->cap = caps_of(h->B);
    return create_impl(h, params, hip_stream, device_arena, arena_bytes, out);
}

int tsim_batch_footprint(const tsim_network* nets, const tsim_trips* trips, const tsim_params* params, int32_t n,
                         size_t* bytes_out)
{
    if (!bytes_out) return fail(nullptr, TSIM_EINVAL, "null bytes_out");
    Union U;
    int rc = make_union(nets, trips, params, n, U, nullptr);
    if (rc) return rc;
    tsim_handle tmp;
    rc = build_tables(&U.net, &U.trips, params, tmp.B, nullptr);
    if (rc) return rc;
    batch_instances(tmp.B, U, params, n);
    tmp.cap = caps_of(tmp.B);
    *bytes_out = arena_size(&tmp) + 256;
    return TSIM_OK;
}

int tsim_batch_create(const tsim_network* nets, const tsim_trips* trips, const tsim_params* params, int32_t n,
                      void* hip_stream, void* device_arena, size_t arena_bytes, tsim_batch** out)
{
    if (!out) return fail(nullptr, TSIM_EINVAL, "null out");
    *out = nullptr;
    if (!device_arena) return fail(nullptr, TSIM_EINVAL, "null arena");
    Union U;
    int rc = make_union(nets, trips, params, n, U, nullptr);
    if (rc) return rc;
    tsim_handle* h = new (std::nothrow) tsim_handle();
    if (!h) return fail(nullptr, TSIM_ENOMEM, "host allocation failed");
    rc = build_tables(&U.net, &U.trips, params, h->B, &h->err);
    if (rc) {
        delete h;
        return rc;
    }
    batch_instances(h->B, U, params, n);
    h->cap = caps_of(h->B);
    return create_impl(h, params, hip_stream, device_arena, arena_bytes, out);
}

}  // extern "C"

namespace {

// index spans of the host tables whose device copies are (re)written:
// roads, internal lanes, junctions, vehicles, junction-lane CSR entries,
// phases, route entries, instances
struct Span {
    int r0, r1, m0, m1, j0, j1, v0, v1, q0, q1, p0, p1, k0, k1;
    long long e0, e1;
};

Span full_span(const Build& B)
{
    return Span{0, B.R, 0, B.NL, 0, B.NJ, 0, B.N, 0, (int)B.out_jl.size(), 0, (int)B.phase_dur.size(), 0, B.n_inst,
                0, (long long)B.route.size()};
}

// copies src[lo, hi) to dst + lo
template <class T>
hipError_t up_range(tsim_handle* h, T* dst, const std::vector<T>& src, long long lo, long long hi)
{
    if (hi <= lo) return hipSuccess;
    return hipMemcpyAsync((void*)(dst + lo), src.data() + lo, (size_t)(hi - lo) * sizeof(T), hipMemcpyHostToDevice,
                          h->stream);
}

// device copies of the static tables over a span (prefix arrays include
// their end entry); per-instance keys, start steps and horizons of the span's
// instances
int upload_tables(tsim_handle* h, const Span& sp)
{
    Build& B = h->B;
    DevNet& D = h->D;
    auto chk = [&](hipError_t e, const char* what) -> int { return e == hipSuccess ? 0 : hip_fail(h, e, what); };
    int e = 0;
    e = e ? e : chk(up_range(h, (int32_t*)D.tile_lane_begin, B.tile_lane_begin, sp.r0, sp.r1 + 1), "tiles");
    e = e ? e : chk(up_range(h, (int32_t*)D.tile_n_road, B.tile_n_road, sp.r0, sp.r1), "tiles");
    e = e ? e : chk(up_range(h, (float*)D.lane_len, B.lane_len, sp.m0, sp.m1), "lanes");
    {
        std::vector<LaneInfo> li(B.NL);
        for (int m = sp.m0; m < sp.m1; ++m) li[m] = lane_info_of(B, m);
        e = e ? e : chk(up_range(h, (LaneInfo*)D.lane_info, li, sp.m0, sp.m1), "lanes");
    }
    e = e ? e : chk(up_range(h, (float*)D.lane_lim, B.lane_lim, sp.m0, sp.m1), "lanes");
    e = e ? e : chk(up_range(h, (uint32_t*)D.lane_base, B.lane_base, sp.m0, sp.m1), "lanes");
    e = e ? e : chk(up_range(h, (int32_t*)D.lane_cap, B.lane_cap, sp.m0, sp.m1), "lanes");
    e = e ? e : chk(up_range(h, (int32_t*)D.lane_tile, B.lane_tile, sp.m0, sp.m1), "lanes");
    e = e ? e : chk(up_range(h, (int32_t*)D.lane_local, B.lane_local, sp.m0, sp.m1), "lanes");
    e = e ? e : chk(up_range(h, (int32_t*)D.jl_out, B.jl_out, sp.m0, sp.m1), "lanes");
    e = e ? e : chk(up_range(h, (int32_t*)D.jl_junc, B.jl_junc, sp.m0, sp.m1), "lanes");
    e = e ? e : chk(up_range(h, (uint32_t*)D.jl_green_mask, B.jl_green_mask, sp.m0, sp.m1), "lanes");
    e = e ? e : chk(up_range(h, (int32_t*)D.jl_ext, B.jl_ext, sp.m0, sp.m1), "lanes");
    e = e ? e : chk(up_range(h, (int32_t*)D.jl_in_local, B.jl_in_local, sp.m0, sp.m1), "lanes");
    e = e ? e : chk(up_range(h, (int32_t*)D.jl_out_road, B.jl_out_road, sp.m0, sp.m1), "lanes");
    e = e ? e : chk(up_range(h, (int32_t*)D.out_begin, B.out_begin, sp.m0, sp.m1 + 1), "conn");
    e = e ? e : chk(up_range(h, (int32_t*)D.out_jl, B.out_jl, sp.q0, sp.q1), "conn");
    {
        std::vector<int32_t> pairs(2 * B.out_jl.size());
        for (int k = sp.q0; k < sp.q1; ++k) {
            pairs[2 * k] = jl_road_eff(B, B.out_jl[k]);
            pairs[2 * k + 1] = B.out_jl[k];
        }
        e = e ? e : chk(up_range(h, (int32_t*)D.out_pair, pairs, 2LL * sp.q0, 2LL * sp.q1), "conn");
    }
    e = e ? e : chk(up_range(h, (int32_t*)D.feed_begin, B.feed_begin, sp.m0, sp.m1 + 1), "conn");
    e = e ? e : chk(up_range(h, (int32_t*)D.feed_jl, B.feed_jl, sp.q0, sp.q1), "conn");
    e = e ? e : chk(up_range(h, (int32_t*)D.junc_phase_begin, B.junc_phase_begin, sp.j0, sp.j1 + 1), "junctions");
    e = e ? e : chk(up_range(h, (int32_t*)D.mp_begin, B.mp_begin, sp.j0, sp.j1 + 1), "junctions");
    e = e ? e : chk(up_range(h, (int32_t*)D.mp_mov, B.mp_mov, 4LL * sp.q0, 4LL * sp.q1), "junctions");
    e = e ? e : chk(up_range(h, (float*)D.phase_dur, B.phase_dur, sp.p0, sp.p1), "junctions");
    e = e ? e : chk(up_range(h, (double*)D.junc_cycle, B.junc_cycle, sp.j0, sp.j1), "junctions");
    e = e ? e : chk(up_range(h, (float*)D.tau, B.tau, sp.v0, sp.v1), "trips");
    e = e ? e : chk(up_range(h, (int32_t*)D.route_begin, B.rstart, sp.v0, sp.v1), "trips");
    e = e ? e : chk(up_range(h, (int32_t*)D.route, B.route, sp.e0, sp.e1), "trips");
    e = e ? e : chk(up_range(h, (float*)D.vf, B.vf, sp.v0, sp.v1), "trips");
    e = e ? e : chk(up_range(h, (float*)D.vlen, B.vlen, sp.v0, sp.v1), "trips");
    e = e ? e : chk(up_range(h, (float*)D.vend, B.vend, sp.v0, sp.v1), "trips");
    e = e ? e : chk(up_range(h, (float*)D.vstart, B.vstart, sp.v0, sp.v1), "trips");
    e = e ? e : chk(up_range(h, (int32_t*)D.q_begin, B.q_begin, sp.r0, sp.r1 + 1), "queues");
    {
        // queue entries of the span's roads are those of its vehicles
        const int k0 = B.q_begin[sp.r0], k1 = B.q_begin[sp.r1];
        std::vector<QRec> qr(B.q_veh.size());
        for (int k = k0; k < k1; ++k) {
            const int v = B.q_veh[k];
            const int rb = B.rstart[v], rl = B.rlen[v];
            QRec& q = qr[k];
            q.tau = B.tau[v];
            q.mask = B.q_mask[k];
            q.vid = v;
            q.len = B.vlen[v];
            q.f = B.vf[v];
            q.rp = rb;
            q.rem = rl - 1;
            q.nr = next_word(B, v, rb, rl - 1);
        }
        e = e ? e : chk(up_range(h, (QRec*)D.q_rec, qr, k0, k1), "queues");
    }
    e = e ? e : chk(up_range(h, h->d_lane_ext, B.ext_of_int, sp.m0, sp.m1), "lanes");
    e = e ? e : chk(up_range(h, (int32_t*)D.tile_inst, B.tile_inst, sp.r0, sp.r1), "instances");
    e = e ? e : chk(up_range(h, (int32_t*)D.junc_inst, B.junc_inst, sp.j0, sp.j1), "instances");
    e = e ? e : chk(up_range(h, (int32_t*)D.inst_vbase, B.inst_vbase, sp.k0, sp.k1), "instances");
    e = e ? e : chk(up_range(h, (uint32_t*)D.inst_key, B.inst_key, 2LL * sp.k0, 2LL * sp.k1), "instances");
    e = e ? e : chk(up_range(h, (long long*)D.inst_t0, B.inst_t0, sp.k0, sp.k1), "instances");
    {
        std::vector<long long> ends(B.n_inst, std::numeric_limits<long long>::max());
        e = e ? e : chk(up_range(h, (long long*)D.inst_end, ends, sp.k0, sp.k1), "instances");
    }
    return e;
}

// the view's sizes and schedule grids from the host tables (after a create
// or a change of the batch's instances)
void refresh_view(tsim_handle* h)
{
    Build& B = h->B;
    DevNet& D = h->D;
    count_tiles(B);
    D.R = B.R;
    D.NJ = B.NJ;
    D.NL = B.NL;
    D.N = B.N;
    D.G = B.G;
    D.n_inst = B.n_inst;
    set_sched(h, D.sched);
}

}  // namespace

extern "C" {

static int create_impl(tsim_handle* h, const tsim_params* params, void* hip_stream, void* device_arena,
                       size_t arena_bytes, tsim_handle** out)
{
    int rc = 0;
    const size_t need = arena_size(h);
    char* base = (char*)(((uintptr_t)device_arena + 255) & ~(uintptr_t)255);
    const size_t lost = (size_t)(base - (char*)device_arena);
    if (arena_bytes < need + lost) {
        g_error = "arena too small: need " + std::to_string(need + lost) + " bytes";
        delete h;
        return TSIM_ENOMEM;
    }
    h->stream = (hipStream_t)hip_stream;
    h->arena = (char*)device_arena;
    h->arena_bytes = arena_bytes;
    size_t off = 0;
    for (auto& r : regions(h, true)) {
        *r.ptr = base + off;
        off += align_up(r.bytes);
    }
    Build& B = h->B;
    DevNet& D = h->D;
    {
        int dev = 0, cus = 0;
        if (hipGetDevice(&dev) == hipSuccess && hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) == hipSuccess) {
            for (int sc = 0; sc < kNumSched; ++sc) h->res[sc] = cus * update_blocks_per_cu(sc);
            h->res[kNumSched] = cus * update_blocks_per_cu(-1);
            h->res[kNumSched + 1] = cus * update_blocks_per_cu(-2);
            h->res[kNumSched + 2] = cus * update_blocks_per_cu(-3);
            h->res[kNumSched + 3] = cus * update_blocks_per_cu(-4);
        }
    }
    D.sched = kSchedFused;
    refresh_view(h);
    h->removed.assign(B.n_inst, 0);
    {
        // set-up of the no-allocation entry point on this GPU: its scratch
        // address, looked up once per device (a failure is reported by that
        // entry point, which looks again)
        int32_t* sp = nullptr;
        (void)noalloc_scratch(&sp);
        (void)hipGetDevice(&h->device);
    }
    h->params = *params;
    fill_params(D.P, params);
    int e = 0;
    // the fused update kernel's LDS (above the default dynamic limit), set
    // whether or not the occupancy queries above ran
    {
        const hipError_t pe = prepare_update_kernels();
        if (pe != hipSuccess) e = hip_fail(h, pe, "fused update kernel attributes");
    }
    e = e ? e : upload_tables(h, full_span(B));
    if (!e) {
        const hipError_t ce = hipMemcpyAsync(h->d_net, &h->D, sizeof(DevNet), hipMemcpyHostToDevice, h->stream);
        if (ce != hipSuccess) e = hip_fail(h, ce, "view");
    }
    if (e) {
        delete h;
        return e;
    }
    // initial state: every vehicle waiting at t = 0
    std::vector<int32_t> st(B.N, TSIM_WAITING), lane(B.N, -1), rpos(B.N, 0), fs(B.N, -1);
    std::vector<float> xz(B.N, 0.f), vz(B.N, 0.f);
    std::vector<int32_t> zero_nj(B.NJ, 0);
    rc = upload_state(h, -1, 0, st.data(), lane.data(), rpos.data(), xz.data(), vz.data(), fs.data(), B.junc_policy.data(),
                      zero_nj.data());
    if (rc) {
        delete h;
        return rc;
    }
    *out = h;
    return TSIM_OK;
}

namespace {
constexpr int kEventPairs = 4096;

// sums the recorded event pairs of kernel k into h->ms[k]
int flush_events(tsim_handle* h, int k)
{
    if (h->ev_used[k] == 0) return TSIM_OK;
    HIPCHK(h, hipStreamSynchronize(h->stream));
    for (int i = 0; i < h->ev_used[k]; ++i) {
        float t = 0.f;
        HIPCHK(h, hipEventElapsedTime(&t, h->ev[k][2 * i], h->ev[k][2 * i + 1]));
        h->ms[k] += t;
    }
    h->launches[k] += h->ev_used[k];
    h->ev_used[k] = 0;
    return TSIM_OK;
}

int timed_launch(tsim_handle* h, int k)
{
    if (!h->prof) return (k == 0 ? launch_update(h->d_net, h->D, h->stream, &h->ps) : launch_prepare(h->d_net, h->D, h->stream)) == hipSuccess
                             ? TSIM_OK
                             : hip_fail(h, hipGetLastError(), "kernel launch");
    if (h->ev_used[k] == kEventPairs) {
        int rc = flush_events(h, k);
        if (rc) return rc;
    }
    if (h->ev[k].empty()) {
        h->ev[k].resize(2 * kEventPairs);
        for (auto& e : h->ev[k]) HIPCHK(h, hipEventCreate(&e));
    }
    const int i = h->ev_used[k]++;
    HIPCHK(h, hipEventRecord(h->ev[k][2 * i], h->stream));
    HIPCHK(h, k == 0 ? launch_update(h->d_net, h->D, h->stream, &h->ps) : launch_prepare(h->d_net, h->D, h->stream));
    HIPCHK(h, hipEventRecord(h->ev[k][2 * i + 1], h->stream));
    return TSIM_OK;
}
}  // namespace

static int capture_chunk(tsim_handle* h)
{
    hipGraph_t g = nullptr;
    if (!h->cap_stream) HIPCHK(h, hipStreamCreateWithFlags(&h->cap_stream, hipStreamNonBlocking));
    HIPCHK(h, hipStreamBeginCapture(h->cap_stream, hipStreamCaptureModeThreadLocal));
    hipError_t e = hipSuccess;
    for (int s = 0; s < h->graph_chunk && e == hipSuccess; ++s) {
        e = launch_prepare(h->d_net, h->D, h->cap_stream);
        if (e == hipSuccess) e = launch_update(h->d_net, h->D, h->cap_stream, &h->ps);
        if (e == hipSuccess && h->traj_every > 0)
            e = launch_record(h->D, h->d_lane_ext, h->traj, h->traj_cap, h->d_traj_n, h->traj_every, h->cap_stream);
    }
    hipError_t e2 = hipStreamEndCapture(h->cap_stream, &g);
    if (e != hipSuccess || e2 != hipSuccess) {
        if (g) (void)hipGraphDestroy(g);
        return fail(&h->err, TSIM_EDEVICE, std::string("graph capture: ") + hipGetErrorString(e != hipSuccess ? e : e2));
    }
    e = hipGraphInstantiate(&h->graph, g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    if (e != hipSuccess) {
        h->graph = nullptr;
        return fail(&h->err, TSIM_EDEVICE, std::string("graph instantiate: ") + hipGetErrorString(e));
    }
    return TSIM_OK;
}

int tsim_set_graph_steps(tsim_handle* h, int32_t chunk)
{
    if (!h || chunk < 0 || chunk > 4096) return fail(nullptr, TSIM_EINVAL, "bad handle or chunk");
    if (h->graph) {
        HIPCHK(h, hipStreamSynchronize(h->stream));
        (void)hipGraphExecDestroy(h->graph);
        h->graph = nullptr;
    }
    h->graph_chunk = chunk;
    return TSIM_OK;
}

int tsim_set_schedule(tsim_handle* h, int32_t schedule)
{
    if (!h || schedule < 0 || schedule >= kNumSched) return fail(nullptr, TSIM_EINVAL, "bad handle or schedule");
    if (schedule == h->D.sched) return TSIM_OK;
    if (h->graph) {
        HIPCHK(h, hipStreamSynchronize(h->stream));
        (void)hipGraphExecDestroy(h->graph);
        h->graph = nullptr;
    }
    set_sched(h, schedule);
    return TSIM_OK;
}

int tsim_set_concurrency(tsim_handle* h, int32_t enable)
{
    if (!h || enable < 0 || enable > 1) return fail(nullptr, TSIM_EINVAL, "bad handle or flag");
    if ((h->ps.n > 0) == (enable == 1)) return TSIM_OK;
    HIPCHK(h, hipStreamSynchronize(h->stream));
    if (h->graph) {
        (void)hipGraphExecDestroy(h->graph);
        h->graph = nullptr;
    }
    if (enable) {
        if (!h->ps.fork) HIPCHK(h, hipEventCreateWithFlags(&h->ps.fork, hipEventDisableTiming));
        for (int i = 0; i < 3; ++i) {
            if (!h->ps.aux[i]) HIPCHK(h, hipStreamCreateWithFlags(&h->ps.aux[i], hipStreamNonBlocking));
            if (!h->ps.join[i]) HIPCHK(h, hipEventCreateWithFlags(&h->ps.join[i], hipEventDisableTiming));
        }
    }
    h->ps.n = enable ? 3 : 0;
    return TSIM_OK;
}

int tsim_get_schedule(tsim_handle* h, int32_t* schedule)
{
    if (!h || !schedule) return fail(nullptr, TSIM_EINVAL, "bad arguments");
    *schedule = h->D.sched;
    return TSIM_OK;
}

// times `rounds` rounds of `steps` real steps under every schedule in turn,
// with the handle's current pass concurrency; best_ms[sc] receives each
// schedule's best round.  Leaves the schedule as it found it.
static int time_schedules(tsim_handle* h, int32_t steps, int32_t rounds, float* best_ms)
{
    std::vector<hipEvent_t> ev(2 * (size_t)rounds * kNumSched, nullptr);
    int rc = TSIM_OK;
    for (auto& e : ev) {
        if (hipEventCreate(&e) != hipSuccess) {
            rc = fail(&h->err, TSIM_EDEVICE, "event creation failed");
            break;
        }
    }
    const int keep = h->D.sched;
    for (int r = 0; r < rounds && rc == TSIM_OK; ++r) {
        for (int sc = 0; sc < kNumSched && rc == TSIM_OK; ++sc) {
            set_sched(h, sc);
            const size_t k = 2 * ((size_t)r * kNumSched + sc);
            hipError_t e = hipEventRecord(ev[k], h->stream);
            for (int t = 0; t < steps && e == hipSuccess; ++t) {
                e = launch_prepare(h->d_net, h->D, h->stream);
                if (e == hipSuccess) e = launch_update(h->d_net, h->D, h->stream, &h->ps);
            }
            if (e == hipSuccess) e = hipEventRecord(ev[k + 1], h->stream);
            if (e != hipSuccess) rc = hip_fail(h, e, "autotune");
        }
    }
    for (int sc = 0; sc < kNumSched; ++sc) best_ms[sc] = std::numeric_limits<float>::infinity();
    if (rc == TSIM_OK) {
        hipError_t e = hipStreamSynchronize(h->stream);
        for (int r = 0; r < rounds && e == hipSuccess; ++r)
            for (int sc = 0; sc < kNumSched && e == hipSuccess; ++sc) {
                const size_t k = 2 * ((size_t)r * kNumSched + sc);
                float ms = 0.0f;
                e = hipEventElapsedTime(&ms, ev[k], ev[k + 1]);
                best_ms[sc] = std::min(best_ms[sc], ms);
            }
        if (e != hipSuccess) rc = hip_fail(h, e, "autotune timing");
    }
    for (auto& e : ev)
        if (e) (void)hipEventDestroy(e);
    set_sched(h, keep);
    return rc;
}

int tsim_autotune(tsim_handle* h, int32_t steps, int32_t rounds, int32_t* chosen, float* us_per_step)
{
    if (!h || steps < 1 || rounds < 1 || steps > 100000 || rounds > 100)
        return fail(nullptr, TSIM_EINVAL, "bad handle, steps or rounds");
    if (h->D.R + h->D.NJ == 0) return fail(&h->err, TSIM_EINVAL, "autotune of an empty batch");
    float best_ms[kNumSched];
    const int rc = time_schedules(h, steps, rounds, best_ms);
    int pick = h->D.sched;
    if (rc == TSIM_OK) {
        pick = 0;
        for (int sc = 1; sc < kNumSched; ++sc)
            if (best_ms[sc] < best_ms[pick]) pick = sc;
        if (us_per_step)
            for (int sc = 0; sc < kNumSched; ++sc) us_per_step[sc] = best_ms[sc] * 1000.0f / (float)steps;
    }
    const int rc2 = tsim_set_schedule(h, pick);
    if (chosen) *chosen = h->D.sched;
    return rc ? rc : rc2;
}

int tsim_autotune_launch(tsim_handle* h, int32_t steps, int32_t rounds, int32_t* schedule, int32_t* concurrent,
                         float* us_per_step)
{
    if (!h || steps < 1 || rounds < 1 || steps > 100000 || rounds > 100)
        return fail(nullptr, TSIM_EINVAL, "bad handle, steps or rounds");
    if (h->D.R + h->D.NJ == 0) return fail(&h->err, TSIM_EINVAL, "autotune of an empty batch");
    const int keep_conc = h->ps.n > 0 ? 1 : 0;
    float best_ms[2][kNumSched];
    int rc = TSIM_OK;
    for (int c = 0; c < 2 && rc == TSIM_OK; ++c) {
        rc = tsim_set_concurrency(h, c);
        if (rc == TSIM_OK) rc = time_schedules(h, steps, rounds, best_ms[c]);
    }
    int pick_s = h->D.sched, pick_c = keep_conc;
    if (rc == TSIM_OK) {
        pick_s = 0;
        pick_c = 0;
        for (int c = 0; c < 2; ++c)
            for (int sc = 0; sc < kNumSched; ++sc)
                if (best_ms[c][sc] < best_ms[pick_c][pick_s]) {
                    pick_c = c;
                    pick_s = sc;
                }
        if (us_per_step)
            for (int c = 0; c < 2; ++c)
                for (int sc = 0; sc < kNumSched; ++sc)
                    us_per_step[c * kNumSched + sc] = best_ms[c][sc] * 1000.0f / (float)steps;
    }
    int rc2 = tsim_set_concurrency(h, pick_c);
    if (rc2 == TSIM_OK) rc2 = tsim_set_schedule(h, pick_s);
    if (schedule) *schedule = h->D.sched;
    if (concurrent) *concurrent = h->ps.n > 0 ? 1 : 0;
    return rc ? rc : rc2;
}

int tsim_step(tsim_handle* h, int32_t n_steps)
{
    if (!h || n_steps < 0) return fail(nullptr, TSIM_EINVAL, "bad handle or step count");
    if (h->D.R + h->D.NJ == 0) return TSIM_OK;   // an empty batch has nothing to step
    if (h->graph_chunk > 0 && !h->prof) {
        if (!h->graph) {
            int rc = capture_chunk(h);
            if (rc) return rc;
        }
        while (n_steps >= h->graph_chunk) {
            HIPCHK(h, hipGraphLaunch(h->graph, h->stream));
            n_steps -= h->graph_chunk;
        }
    }
    for (int s = 0; s < n_steps; ++s) {
        int rc = timed_launch(h, 1);
        if (rc) return rc;
        rc = timed_launch(h, 0);
        if (rc) return rc;
        if (h->traj_every > 0)
            HIPCHK(h, launch_record(h->D, h->d_lane_ext, h->traj, h->traj_cap, h->d_traj_n, h->traj_every, h->stream));
    }
    return TSIM_OK;
}

int tsim_set_trajectory(tsim_handle* h, void* device_buffer, int64_t capacity, int32_t every)
{
    if (!h || every < 0 || (every > 0 && (!device_buffer || capacity < 0)) || h->B.n_inst != 1)
        return fail(nullptr, TSIM_EINVAL, "bad arguments (single-instance handles only)");
    if (h->graph) {
        HIPCHK(h, hipStreamSynchronize(h->stream));
        (void)hipGraphExecDestroy(h->graph);
        h->graph = nullptr;
    }
    h->traj = (TrajRec*)device_buffer;
    h->traj_cap = every > 0 ? capacity : 0;
    h->traj_every = every;
    HIPCHK(h, hipMemsetAsync(h->d_traj_n, 0, 8, h->stream));
    HIPCHK(h, hipStreamSynchronize(h->stream));
    return TSIM_OK;
}

int tsim_get_trajectory_count(tsim_handle* h, int64_t* n)
{
    if (!h || !n) return fail(nullptr, TSIM_EINVAL, "bad arguments");
    unsigned long long c = 0;
    HIPCHK(h, hipMemcpyAsync(&c, h->d_traj_n, 8, hipMemcpyDeviceToHost, h->stream));
    HIPCHK(h, hipStreamSynchronize(h->stream));
    *n = (int64_t)c;
    return TSIM_OK;
}

// layout of the AOI buffer: origin ids [N], destination ids [N], counts
// [2 n_aoi], each part 256-byte aligned
static size_t aoi_bytes(long long n_veh, long long n_aoi)
{
    auto up = [](size_t b) { return (b + 255) / 256 * 256; };
    return 2 * up((size_t)std::max<long long>(n_veh, 1) * 4) + up((size_t)std::max<long long>(2 * n_aoi, 1) * 4);
}

// instance k of a batch (k >= 0, not removed) or the single instance (k < 0)
static bool instance_ok(const tsim_handle* h, int k)
{
    if (k < 0) return h->B.n_inst == 1;
    return k < h->B.n_inst && !(k < (int)h->removed.size() && h->removed[k]);
}

static int aoi_footprint_impl(tsim_handle* h, int k, int32_t n_aoi, size_t* bytes_out)
{
    if (!h || n_aoi < 0 || !bytes_out || !instance_ok(h, k)) return fail(nullptr, TSIM_EINVAL, "bad arguments");
    const Ranges g = ranges_of(h->B, k);
    *bytes_out = aoi_bytes(g.v1 - g.v0, n_aoi);
    return TSIM_OK;
}

static int set_aois_impl(tsim_handle* h, int k, int32_t n_aoi, const int32_t* conn_begin, const int32_t* conn_road,
                         const float* conn_s, const int32_t* origin_aoi, const int32_t* dest_aoi, void* device_buffer,
                         size_t buffer_bytes)
{
    if (!h || n_aoi < 0 || (n_aoi > 0 && !conn_begin) || !device_buffer || !instance_ok(h, k))
        return fail(nullptr, TSIM_EINVAL, "bad arguments");
    Build& B = h->B;
    DevNet& D = h->D;
    const Ranges g = ranges_of(B, k);
    const int N = g.v1 - g.v0, R = g.r1 - g.r0;
    if ((reinterpret_cast<uintptr_t>(device_buffer) & 255u) != 0 || buffer_bytes < aoi_bytes(N, n_aoi))
        return fail(&h->err, TSIM_EINVAL, "AOI buffer too small or not 256-byte aligned");
    const int n_conn = n_aoi > 0 ? conn_begin[n_aoi] : 0;
    if (n_aoi > 0 && (conn_begin[0] != 0 || (n_conn > 0 && (!conn_road || !conn_s))))
        return fail(&h->err, TSIM_EINVAL, "bad AOI connection table");
    for (int a = 0; a < n_aoi; ++a)
        if (conn_begin[a + 1] < conn_begin[a]) return fail(&h->err, TSIM_EINVAL, "bad AOI connection table");
    for (int c = 0; c < n_conn; ++c) {
        const int r = conn_road[c];
        if (r < 0 || r >= R) return fail(&h->err, TSIM_EINVAL, "AOI connection on a road out of range");
        if (!(conn_s[c] >= 0.0f && conn_s[c] <= B.lane_len[B.tile_lane_begin[g.r0 + r]]))
            return fail(&h->err, TSIM_EINVAL, "AOI connection beyond its road");
    }
    // the AOI's first listed connection on (union) road r, -1 when it has none
    auto conn_on = [&](int a, int r) {
        for (int c = conn_begin[a]; c < conn_begin[a + 1]; ++c)
            if (g.r0 + conn_road[c] == r) return c;
        return -1;
    };
    std::vector<int32_t> st(N);
    if (N > 0) {
        HIPCHK(h, hipMemcpyAsync(st.data(), D.status + g.v0, (size_t)N * 4, hipMemcpyDeviceToHost, h->stream));
        HIPCHK(h, hipStreamSynchronize(h->stream));
    }
    std::vector<int32_t> org(N, -1), dst(N, -1);
    std::vector<float> vstart = B.vstart, vend = B.vend;
    for (int i = 0; i < N; ++i) {
        const int o = origin_aoi ? origin_aoi[i] : -1, d = dest_aoi ? dest_aoi[i] : -1;
        if (o < 0 && d < 0) continue;
        if (o >= n_aoi || d >= n_aoi) return fail(&h->err, TSIM_EINVAL, "AOI id out of range");
        if (st[i] != TSIM_WAITING)
            return fail(&h->err, TSIM_EINVAL, "vehicle " + std::to_string(i) + " has already departed");
        const int v = g.v0 + i;
        const int first = B.route[B.rstart[v]], last = B.route[B.rstart[v] + B.rlen[v] - 1];
        if (o >= 0) {
            const int c = conn_on(o, first);
            if (c < 0)
                return fail(&h->err, TSIM_EINVAL, "vehicle " + std::to_string(i) + ": its origin AOI has no connection on its first road");
            if (!(conn_s[c] < B.lane_len[B.tile_lane_begin[first]]))
                return fail(&h->err, TSIM_EINVAL, "vehicle " + std::to_string(i) + ": its start connection is at the road's end");
            vstart[v] = conn_s[c];
            org[i] = o;
        }
        if (d >= 0) {
            const int c = conn_on(d, last);
            if (c < 0)
                return fail(&h->err, TSIM_EINVAL, "vehicle " + std::to_string(i) + ": its destination AOI has no connection on its last road");
            if (!(conn_s[c] > 0.0f))
                return fail(&h->err, TSIM_EINVAL, "vehicle " + std::to_string(i) + ": its end connection is at the road's start");
            vend[v] = conn_s[c];
            dst[i] = d;
        }
    }
    // every vehicle concerned is still waiting: its start and end positions
    // are read when it departs
    auto up = [](size_t b) { return (b + 255) / 256 * 256; };
    int32_t* base = (int32_t*)device_buffer;
    int32_t* d_org = base;
    int32_t* d_dst = (int32_t*)((char*)device_buffer + up((size_t)std::max(N, 1) * 4));
    if (N > 0) {
        HIPCHK(h, hipMemcpyAsync(d_org, org.data(), (size_t)N * 4, hipMemcpyHostToDevice, h->stream));
        HIPCHK(h, hipMemcpyAsync(d_dst, dst.data(), (size_t)N * 4, hipMemcpyHostToDevice, h->stream));
    }
    B.vstart = vstart;
    B.vend = vend;
    HIPCHK(h, up_range(h, (float*)D.vstart, B.vstart, g.v0, g.v1));
    HIPCHK(h, up_range(h, (float*)D.vend, B.vend, g.v0, g.v1));
    // a one-road trip's departure record carries its end position (its
    // next-road word): the instance's queue records are written again from
    // the tables
    const int q0 = B.q_begin[g.r0], q1 = B.q_begin[g.r1];
    std::vector<QRec> qr(B.q_veh.size());
    for (int q = q0; q < q1; ++q) {
        const int v = B.q_veh[q];
        const int rb = B.rstart[v], rl = B.rlen[v];
        qr[q].tau = B.tau[v];
        qr[q].mask = B.q_mask[q];
        qr[q].vid = v;
        qr[q].len = B.vlen[v];
        qr[q].f = B.vf[v];
        qr[q].rp = rb;
        qr[q].rem = rl - 1;
        qr[q].nr = next_word(B, v, rb, rl - 1);
    }
    HIPCHK(h, up_range(h, (QRec*)D.q_rec, qr, q0, q1));
    HIPCHK(h, hipStreamSynchronize(h->stream));
    const size_t slot = k < 0 ? 0 : (size_t)k;
    if (h->aois.size() <= slot) h->aois.resize(slot + 1);
    h->aois[slot].d = base;
    h->aois[slot].n = n_aoi;
    return TSIM_OK;
}

static int get_aoi_counts_impl(tsim_handle* h, int k, int32_t* waiting, int32_t* arrived, int32_t n_aoi)
{
    if (!h || !instance_ok(h, k)) return fail(nullptr, TSIM_EINVAL, "bad arguments");
    const size_t slot = k < 0 ? 0 : (size_t)k;
    if (slot >= h->aois.size() || !h->aois[slot].d || n_aoi != h->aois[slot].n || (n_aoi > 0 && (!waiting || !arrived)))
        return fail(&h->err, TSIM_EINVAL, "no AOIs set for the instance, or another AOI count");
    if (n_aoi == 0) return TSIM_OK;
    auto up = [](size_t b) { return (b + 255) / 256 * 256; };
    const DevNet& D = h->D;
    const Ranges g = ranges_of(h->B, k);
    const int nv = g.v1 - g.v0;
    int32_t* d = h->aois[slot].d;
    const size_t vb = up((size_t)std::max(nv, 1) * 4);
    const int32_t* d_org = d;
    const int32_t* d_dst = (const int32_t*)((const char*)d + vb);
    int32_t* cnt = (int32_t*)((char*)d + 2 * vb);
    HIPCHK(h, hipMemsetAsync(cnt, 0, (size_t)2 * n_aoi * 4, h->stream));
    HIPCHK(h, launch_aoi_counts(D, g.v0, nv, d_org, d_dst, n_aoi, cnt, h->stream));
    HIPCHK(h, hipMemcpyAsync(waiting, cnt, (size_t)n_aoi * 4, hipMemcpyDeviceToHost, h->stream));
    HIPCHK(h, hipMemcpyAsync(arrived, cnt + n_aoi, (size_t)n_aoi * 4, hipMemcpyDeviceToHost, h->stream));
    HIPCHK(h, hipStreamSynchronize(h->stream));
    return TSIM_OK;
}

int tsim_aoi_footprint(tsim_handle* h, int32_t n_aoi, size_t* bytes_out)
{
    return aoi_footprint_impl(h, -1, n_aoi, bytes_out);
}

int tsim_set_aois(tsim_handle* h, int32_t n_aoi, const int32_t* conn_begin, const int32_t* conn_road,
                  const float* conn_s, const int32_t* origin_aoi, const int32_t* dest_aoi, void* device_buffer,
                  size_t buffer_bytes)
{
    return set_aois_impl(h, -1, n_aoi, conn_begin, conn_road, conn_s, origin_aoi, dest_aoi, device_buffer,
                         buffer_bytes);
}

int tsim_get_aoi_counts(tsim_handle* h, int32_t* waiting, int32_t* arrived, int32_t n_aoi)
{
    return get_aoi_counts_impl(h, -1, waiting, arrived, n_aoi);
}

int tsim_batch_aoi_footprint(tsim_batch* b, int32_t instance, int32_t n_aoi, size_t* bytes_out)
{
    return aoi_footprint_impl(b, instance < 0 ? INT32_MAX : instance, n_aoi, bytes_out);
}

int tsim_batch_set_aois(tsim_batch* b, int32_t instance, int32_t n_aoi, const int32_t* conn_begin,
                        const int32_t* conn_road, const float* conn_s, const int32_t* origin_aoi,
                        const int32_t* dest_aoi, void* device_buffer, size_t buffer_bytes)
{
    return set_aois_impl(b, instance < 0 ? INT32_MAX : instance, n_aoi, conn_begin, conn_road, conn_s, origin_aoi,
                         dest_aoi, device_buffer, buffer_bytes);
}

int tsim_batch_get_aoi_counts(tsim_batch* b, int32_t instance, int32_t* waiting, int32_t* arrived, int32_t n_aoi)
{
    return get_aoi_counts_impl(b, instance < 0 ? INT32_MAX : instance, waiting, arrived, n_aoi);
}

int tsim_set_profiling(tsim_handle* h, int32_t enable)
{
    if (!h) return fail(nullptr, TSIM_EINVAL, "null handle");
    for (int k = 0; k < 2; ++k) {
        int rc = flush_events(h, k);
        if (rc) return rc;
        h->ms[k] = 0.0;
        h->launches[k] = 0;
    }
    h->prof = enable != 0;
    return TSIM_OK;
}

int tsim_get_kernel_times(tsim_handle* h, double* ms, int64_t* launches, int32_t n_kernels)
{
    if (!h || !ms || !launches || n_kernels < 1 || n_kernels > 2) return fail(nullptr, TSIM_EINVAL, "bad arguments");
    for (int k = 0; k < n_kernels; ++k) {
        int rc = flush_events(h, k);
        if (rc) return rc;
        ms[k] = h->ms[k];
        launches[k] = h->launches[k];
    }
    return TSIM_OK;
}

// next pinned/device staging slot for phase updates; waits only for the copy
// that last used the same slot
static int stage_slot(tsim_handle* h, int32_t** hp, int32_t** dp)
{
    const int s = h->pin_slot;
    const size_t bytes = (size_t)2 * h->B.NJ * 4;
    if (!h->h_pin[s]) {
        HIPCHK(h, hipHostMalloc((void**)&h->h_pin[s], bytes, hipHostMallocDefault));
        HIPCHK(h, hipEventCreateWithFlags(&h->pin_ev[s], hipEventDisableTiming));
    }
    if (h->pin_used[s]) HIPCHK(h, hipEventSynchronize(h->pin_ev[s]));
    h->pin_used[s] = true;
    *hp = h->h_pin[s];
    *dp = h->d_io_ph + (size_t)s * 2 * h->B.NJ;
    h->pin_slot = s ^ 1;
    return TSIM_OK;
}

static int set_phases_impl(tsim_handle* h, int inst, const int32_t* junction_ids, const int32_t* phase_index,
                           int32_t n)
{
    if (!h || n < 0 || (n && (!junction_ids || !phase_index))) return fail(nullptr, TSIM_EINVAL, "bad arguments");
    Build& B = h->B;
    if (inst < 0 || inst >= B.n_inst) return fail(&h->err, TSIM_EINVAL, "instance out of range");
    if (n == 0) return TSIM_OK;
    const int jo = B.junc_off[inst], nj = B.junc_off[inst + 1] - jo;
    if (n > nj) return fail(&h->err, TSIM_EINVAL, "more updates than junctions");
    std::vector<int32_t> ids(n), ph(n);
    for (int c = 0; c < n; ++c) {
        const int j = junction_ids[c];
        if (j < 0 || j >= nj) return fail(&h->err, TSIM_EINVAL, "junction id out of range");
        const int np = B.junc_phase_begin[jo + j + 1] - B.junc_phase_begin[jo + j];
        if (phase_index[c] < 0 || phase_index[c] >= np) return fail(&h->err, TSIM_EINVAL, "phase index out of range");
        ids[c] = jo + j;
        ph[c] = phase_index[c];
    }
    int32_t* hp = nullptr;
    int32_t* dp = nullptr;
    int rc = stage_slot(h, &hp, &dp);
    if (rc) return rc;
    std::memcpy(hp, ids.data(), (size_t)n * 4);
    std::memcpy(hp + B.NJ, ph.data(), (size_t)n * 4);
    HIPCHK(h, hipMemcpyAsync(dp, hp, (size_t)2 * B.NJ * 4, hipMemcpyHostToDevice, h->stream));
    HIPCHK(h, launch_set_phases(h->d_net, h->D, dp, dp + B.NJ, n, h->stream));
    HIPCHK(h, hipEventRecord(h->pin_ev[h->pin_slot ^ 1], h->stream));
    return TSIM_OK;
}

int tsim_set_signal_phases(tsim_handle* h, const int32_t* junction_ids, const int32_t* phase_index, int32_t n)
{
    return set_phases_impl(h, 0, junction_ids, phase_index, n);
}

int tsim_set_signal_phases_noalloc(tsim_handle* h, const int32_t* junction_ids, const int32_t* phase_index, int32_t n)
{
    if (!h || n < 0 || (n && (!junction_ids || !phase_index)) || h->B.n_inst != 1)
        return fail(nullptr, TSIM_EINVAL, "bad arguments");
    if (n > kNoAllocMaxUpdates)
        return fail(&h->err, TSIM_EINVAL, "more than " + std::to_string(kNoAllocMaxUpdates) + " junction updates");
    if (n == 0) return TSIM_OK;
    for (int c = 0; c < n; ++c) {
        const int j = junction_ids[c];
        if (j < 0 || j >= h->B.NJ) return fail(&h->err, TSIM_EINVAL, "junction id out of range");
        const int np = h->B.junc_phase_begin[j + 1] - h->B.junc_phase_begin[j];
        if (phase_index[c] < 0 || phase_index[c] >= np) return fail(&h->err, TSIM_EINVAL, "phase index out of range");
    }
    int cur = 0;
    HIPCHK(h, hipGetDevice(&cur));
    if (cur != h->device) return fail(&h->err, TSIM_EINVAL, "the handle's GPU is not the current device");
    int32_t* sp = nullptr;
    HIPCHK(h, noalloc_scratch(&sp));
    HIPCHK(h, hipMemcpyAsync(sp, junction_ids, (size_t)n * 4, hipMemcpyHostToDevice, h->stream));
    HIPCHK(h, hipMemcpyAsync(sp + kNoAllocMaxUpdates, phase_index, (size_t)n * 4, hipMemcpyHostToDevice, h->stream));
    HIPCHK(h, launch_set_phases(h->d_net, h->D, sp, sp + kNoAllocMaxUpdates, n, h->stream));
    // the caller's arrays and this GPU's scratch are free again on return
    HIPCHK(h, hipStreamSynchronize(h->stream));
    return TSIM_OK;
}

int tsim_batch_set_signal_phases(tsim_batch* b, int32_t instance, const int32_t* junction_ids,
                                 const int32_t* phase_index, int32_t n)
{
    return set_phases_impl(b, instance, junction_ids, phase_index, n);
}

static int set_policy_impl(tsim_handle* h, int inst, const int32_t* junction_ids, const int32_t* policy, int32_t n)
{
    if (!h || n < 0 || (n && (!junction_ids || !policy))) return fail(nullptr, TSIM_EINVAL, "bad arguments");
    Build& B = h->B;
    if (inst < 0 || inst >= B.n_inst) return fail(&h->err, TSIM_EINVAL, "instance out of range");
    if (n == 0) return TSIM_OK;
    const int jo = B.junc_off[inst], nj = B.junc_off[inst + 1] - jo;
    if (n > nj) return fail(&h->err, TSIM_EINVAL, "more updates than junctions");
    std::vector<int32_t> ids(n), pol(n);
    bool mp = false;
    for (int c = 0; c < n; ++c) {
        const int j = junction_ids[c];
        if (j < 0 || j >= nj) return fail(&h->err, TSIM_EINVAL, "junction id out of range");
        if (policy[c] < 0 || policy[c] > 3) return fail(&h->err, TSIM_EINVAL, "bad policy");
        const int pb = B.junc_phase_begin[jo + j], np = B.junc_phase_begin[jo + j + 1] - pb;
        if (policy[c] == TSIM_POLICY_MAX_PRESSURE && np > 0 && !(B.phase_dur[pb] > 0))
            return fail(&h->err, TSIM_EINVAL, "max-pressure junction with a non-positive first phase duration");
        mp |= policy[c] == TSIM_POLICY_MAX_PRESSURE;
        ids[c] = jo + j;
        pol[c] = policy[c];
    }
    if (mp) set_mp_any(h, true);
    int32_t* hp = nullptr;
    int32_t* dp = nullptr;
    int rc = stage_slot(h, &hp, &dp);
    if (rc) return rc;
    std::memcpy(hp, ids.data(), (size_t)n * 4);
    std::memcpy(hp + B.NJ, pol.data(), (size_t)n * 4);
    HIPCHK(h, hipMemcpyAsync(dp, hp, (size_t)2 * B.NJ * 4, hipMemcpyHostToDevice, h->stream));
    HIPCHK(h, launch_set_policy(h->d_net, h->D, dp, dp + B.NJ, n, h->stream));
    HIPCHK(h, hipEventRecord(h->pin_ev[h->pin_slot ^ 1], h->stream));
    return TSIM_OK;
}

int tsim_set_signal_policy(tsim_handle* h, const int32_t* junction_ids, const int32_t* policy, int32_t n)
{
    return set_policy_impl(h, 0, junction_ids, policy, n);
}

int tsim_batch_set_signal_policy(tsim_batch* b, int32_t instance, const int32_t* junction_ids, const int32_t* policy,
                                 int32_t n)
{
    return set_policy_impl(b, instance, junction_ids, policy, n);
}

static int lane_speed_impl(tsim_handle* h, int k, const int32_t* lane_ids, const float* max_speed, int32_t n)
{
    if (!h || n < 0 || (n && (!lane_ids || !max_speed)) || k >= h->B.n_inst || (k < 0 && h->B.n_inst != 1))
        return fail(nullptr, TSIM_EINVAL, "bad arguments");
    Build& B = h->B;
    const Ranges g = ranges_of(B, k);
    const int nl = g.nrl + g.njl;
    if (n > nl) return fail(&h->err, TSIM_EINVAL, "more updates than lanes");
    if (n == 0) return TSIM_OK;
    // the largest desired-speed factor of the instance bounds one step of travel
    float fmax = 0.0f;
    for (int i = g.v0; i < g.v1; ++i) fmax = std::max(fmax, B.vf[i]);
    const double reach = 0.5 * h->params.a_max * h->params.dt * h->params.dt;
    std::vector<int32_t> ids(n);
    std::vector<float> val(n);
    for (int c = 0; c < n; ++c) {
        const int l = lane_ids[c];
        if (l < 0 || l >= nl) return fail(&h->err, TSIM_EINVAL, "lane id out of range");
        const float v = max_speed[c];
        if (!(v > 0.0f) || !std::isfinite(v)) return fail(&h->err, TSIM_EINVAL, "speed limit must be positive");
        const int m = B.int_of_ext[union_lane(B, g, l)];
        if (!(B.lane_len[m] > (double)fmax * v * h->params.dt + reach))
            return fail(&h->err, TSIM_EINVAL, "lane " + std::to_string(l) + " shorter than one step of travel at that limit");
        ids[c] = m;
        val[c] = v;
    }
    for (int c = 0; c < n; ++c) B.lane_lim[ids[c]] = val[c];
    HIPCHK(h, hipMemcpyAsync(h->d_io_lane, ids.data(), (size_t)n * 4, hipMemcpyHostToDevice, h->stream));
    HIPCHK(h, hipMemcpyAsync(h->d_io_lane + B.NL, val.data(), (size_t)n * 4, hipMemcpyHostToDevice, h->stream));
    HIPCHK(h, launch_set_lane_speed(h->D, h->d_io_lane, (const float*)(h->d_io_lane + B.NL), n, h->stream));
    HIPCHK(h, hipStreamSynchronize(h->stream));
    return TSIM_OK;
}

int tsim_set_lane_max_speed(tsim_handle* h, const int32_t* lane_ids, const float* max_speed, int32_t n)
{
    return lane_speed_impl(h, -1, lane_ids, max_speed, n);
}

int tsim_batch_set_lane_max_speed(tsim_batch* b, int32_t instance, const int32_t* lane_ids, const float* max_speed,
                                  int32_t n)
{
    if (!b || instance < 0) return fail(nullptr, TSIM_EINVAL, "bad batch or instance");
    return lane_speed_impl(b, instance, lane_ids, max_speed, n);
}

static int restriction_impl(tsim_handle* h, int k, const int32_t* lane_ids, const int32_t* flags, int32_t n)
{
    if (!h || n < 0 || (n && (!lane_ids || !flags)) || k >= h->B.n_inst || (k < 0 && h->B.n_inst != 1))
        return fail(nullptr, TSIM_EINVAL, "bad arguments");
    Build& B = h->B;
    DevNet& D = h->D;
    const Ranges g = ranges_of(B, k);
    const int nl = g.nrl + g.njl;
    if (n == 0) return TSIM_OK;
    std::vector<int> ids(n);
    for (int c = 0; c < n; ++c) {
        const int l = lane_ids[c];
        if (l < 0 || l >= nl) return fail(&h->err, TSIM_EINVAL, "lane id out of range");
        ids[c] = B.int_of_ext[union_lane(B, g, l)];
    }
    if ((int)B.restricted.size() < B.NL) B.restricted.resize(B.NL, 0);
    // lanes whose device record changes: the given ones, and the junction
    // lanes feeding a given road lane (they close and open with it)
    std::vector<int> lanes;
    for (int c = 0; c < n; ++c) {
        const int m = ids[c];
        B.restricted[m] = flags[c] != 0 ? 1 : 0;
        lanes.push_back(m);
        if (B.jl_out[m] < 0)
            for (int e = B.feed_begin[m]; e < B.feed_begin[m + 1]; ++e) lanes.push_back(B.feed_jl[e]);
    }
    std::sort(lanes.begin(), lanes.end());
    lanes.erase(std::unique(lanes.begin(), lanes.end()), lanes.end());
    // staged copies live until the stream is synchronised below
    std::vector<LaneInfo> recs;
    std::vector<int32_t> pairs;
    std::vector<long long> pair_at;
    for (int m : lanes) {
        recs.push_back(lane_info_of(B, m));
        if (B.jl_out[m] >= 0) {
            // the junction lane's entry in its in lane's out-connection table
            const int in = B.tile_lane_begin[B.lane_tile[m]] + B.jl_in_local[m];
            for (int e = B.out_begin[in]; e < B.out_begin[in + 1]; ++e)
                if (B.out_jl[e] == m) {
                    pairs.push_back(jl_road_eff(B, m));
                    pairs.push_back(m);
                    pair_at.push_back(e);
                }
        }
    }
    for (size_t i = 0; i < lanes.size(); ++i)
        HIPCHK(h, hipMemcpyAsync((void*)(D.lane_info + lanes[i]), &recs[i], sizeof(LaneInfo), hipMemcpyHostToDevice,
                                 h->stream));
    for (size_t i = 0; i < pair_at.size(); ++i)
        HIPCHK(h, hipMemcpyAsync((void*)(D.out_pair + pair_at[i]), &pairs[2 * i], 8, hipMemcpyHostToDevice, h->stream));
    // departure lanes of the queues of the roads these lanes belong to
    std::vector<int> roads;
    for (int m : lanes) roads.push_back(B.lane_tile[m]);
    std::sort(roads.begin(), roads.end());
    roads.erase(std::unique(roads.begin(), roads.end()), roads.end());
    std::vector<uint32_t> masks;
    std::vector<int> mask_at;
    for (int r : roads)
        for (int q = B.q_begin[r]; q < B.q_begin[r + 1]; ++q) {
            const int v = B.q_veh[q];
            const uint32_t mk = depart_mask(B, r, B.rlen[v] > 1 ? B.route[B.rstart[v] + 1] : -1);
            if (mk != B.q_mask[q]) {
                B.q_mask[q] = mk;
                masks.push_back(mk);
                mask_at.push_back(q);
            }
        }
    for (size_t i = 0; i < mask_at.size(); ++i)
        HIPCHK(h, hipMemcpyAsync((void*)&D.q_rec[mask_at[i]].mask, &masks[i], 4, hipMemcpyHostToDevice, h->stream));
    HIPCHK(h, hipStreamSynchronize(h->stream));
    return TSIM_OK;
}

int tsim_set_lane_restriction(tsim_handle* h, const int32_t* lane_ids, const int32_t* flags, int32_t n)
{
    return restriction_impl(h, -1, lane_ids, flags, n);
}

int tsim_batch_set_lane_restriction(tsim_batch* b, int32_t instance, const int32_t* lane_ids, const int32_t* flags,
                                    int32_t n)
{
    if (!b || instance < 0) return fail(nullptr, TSIM_EINVAL, "bad batch or instance");
    return restriction_impl(b, instance, lane_ids, flags, n);
}

static int export_state(tsim_handle* h, std::vector<int32_t>& lane, std::vector<float>& x, std::vector<float>& v,
                        std::vector<int32_t>& rpos, std::vector<int32_t>& rank);

// a junction lane leads from some lane of road a to road b
static bool roads_joined(const Build& B, int a, int b)
{
    const int lb = B.tile_lane_begin[a], nrl = B.tile_n_road[a];
    for (int m = lb; m < lb + nrl; ++m)
        for (int e = B.out_begin[m]; e < B.out_begin[m + 1]; ++e)
            if (B.jl_out_road[B.out_jl[e]] == b) return true;
    return false;
}

static int route_impl(tsim_handle* h, int k, int32_t vid_local, const int32_t* roads_local, int32_t len, float end_s)
{
    if (!h || !roads_local || len < 1 || k >= h->B.n_inst || (k < 0 && h->B.n_inst != 1))
        return fail(nullptr, TSIM_EINVAL, "bad arguments");
    Build& B = h->B;
    DevNet& D = h->D;
    const Ranges g = ranges_of(B, k);
    if (vid_local < 0 || vid_local >= g.v1 - g.v0) return fail(&h->err, TSIM_EINVAL, "vehicle id out of range");
    const int i = g.v0 + vid_local;
    std::vector<int32_t> roads(len);
    for (int c = 0; c < len; ++c) {
        const int r = roads_local[c];
        if (r < 0 || r >= g.r1 - g.r0) return fail(&h->err, TSIM_EINVAL, "road id out of range");
        roads[c] = g.r0 + r;
        if (c > 0 && !roads_joined(B, roads[c - 1], roads[c]))
            return fail(&h->err, TSIM_EINVAL, "consecutive roads of the route are not joined by a junction lane");
    }
    if (!(end_s < 0.0f) && !(end_s > 0.0f && end_s <= B.lane_len[B.tile_lane_begin[roads[len - 1]]]))
        return fail(&h->err, TSIM_EINVAL, "end position beyond the route's last road");
    if ((long long)B.route.size() + len > h->cap.E)
        return fail(&h->err, TSIM_ENOMEM, "no room left for changed routes");
    // where the vehicle is: status, and for an active vehicle its lane and
    // place in the lane order at this step boundary
    std::vector<int32_t> lane, rpos, rank;
    std::vector<float> x, v;
    int32_t st = 0;
    HIPCHK(h, hipMemcpyAsync(&st, D.status + i, 4, hipMemcpyDeviceToHost, h->stream));
    HIPCHK(h, hipStreamSynchronize(h->stream));
    if (st == TSIM_FINISHED) return fail(&h->err, TSIM_EINVAL, "the vehicle has finished its trip");
    const int32_t nst = (int32_t)B.route.size();
    const float new_end = end_s < 0.0f ? -1.0f : end_s;
    const int32_t rem = len - 1;
    // the record's next-road word (on a one-road route, the trip's end)
    const int32_t nr = len > 1 ? roads[1] : end_word(new_end, B.lane_len[B.tile_lane_begin[roads[len - 1]]]);
    if (st == TSIM_WAITING) {
        const int origin = B.route[B.rstart[i]];
        if (roads[0] != origin) return fail(&h->err, TSIM_EINVAL, "a waiting vehicle's route must start at its origin road");
        // its departure queue entry: place, lanes toward the new next road
        int q = -1;
        for (int e = B.q_begin[origin]; e < B.q_begin[origin + 1]; ++e)
            if (B.q_veh[e] == i) q = e;
        if (q < 0) return fail(&h->err, TSIM_ESTATE, "vehicle missing from its departure queue");
        const uint32_t mask = depart_mask(B, origin, len > 1 ? roads[1] : -1);
        B.q_mask[q] = mask;
        QRec qr;
        qr.tau = B.tau[i];
        qr.mask = mask;
        qr.vid = i;
        qr.len = B.vlen[i];
        qr.f = B.vf[i];
        qr.rp = nst;
        qr.rem = rem;
        qr.nr = nr;
        HIPCHK(h, hipMemcpyAsync((void*)(D.q_rec + q), &qr, sizeof(QRec), hipMemcpyHostToDevice, h->stream));
    } else {
        int rc = export_state(h, lane, x, v, rpos, rank);
        if (rc) return rc;
        const int m = B.int_of_ext[lane[i]];
        const int cur = B.lane_tile[m];
        if (roads[0] != cur) return fail(&h->err, TSIM_EINVAL, "the route must start with the vehicle's current road");
        if (B.jl_out[m] >= 0 && (len < 2 || roads[1] != B.jl_out_road[m]))
            return fail(&h->err, TSIM_EINVAL, "a vehicle on a junction lane must keep the road that lane leads to");
        // its record: a lane slot of the current buffer, or the lane's inbox
        long long gnow = 0;
        int32_t cnt = 0;
        HIPCHK(h, hipMemcpyAsync(&gnow, D.gstep, 8, hipMemcpyDeviceToHost, h->stream));
        HIPCHK(h, hipStreamSynchronize(h->stream));
        const int inst = B.tile_inst[cur];
        long long t0 = 0, end = 0;
        HIPCHK(h, hipMemcpyAsync(&t0, D.inst_t0 + inst, 8, hipMemcpyDeviceToHost, h->stream));
        HIPCHK(h, hipMemcpyAsync(&end, D.inst_end + inst, 8, hipMemcpyDeviceToHost, h->stream));
        HIPCHK(h, hipStreamSynchronize(h->stream));
        const long long loc = gnow - t0;
        const bool odd = ((t0 + (loc < end ? loc : end)) & 1) != 0;
        const LaneSum* sum = odd ? D.sum1 : D.sum0;
        VehRec* slab = odd ? D.slab1 : D.slab0;
        HIPCHK(h, hipMemcpyAsync(&cnt, &sum[m].cnt, 4, hipMemcpyDeviceToHost, h->stream));
        HIPCHK(h, hipStreamSynchronize(h->stream));
        VehRec* rec = rank[i] < cnt ? slab + B.lane_base[m] + rank[i] : D.inbox + m;
        const int32_t tail[3] = {nst, rem, nr};   // rp, rem, nr: the record's last three words
        HIPCHK(h, hipMemcpyAsync(&rec->rp, tail, sizeof(tail), hipMemcpyHostToDevice, h->stream));
    }
    B.route.insert(B.route.end(), roads.begin(), roads.end());
    B.rstart[i] = nst;
    B.rlen[i] = len;
    B.vend[i] = new_end;
    HIPCHK(h, up_range(h, (int32_t*)D.route, B.route, nst, nst + len));
    HIPCHK(h, up_range(h, (float*)D.vend, B.vend, i, i + 1));
    HIPCHK(h, hipMemcpyAsync((void*)(D.route_begin + i), &B.rstart[i], 4, hipMemcpyHostToDevice, h->stream));
    HIPCHK(h, hipStreamSynchronize(h->stream));
    return TSIM_OK;
}

int tsim_set_vehicle_route(tsim_handle* h, int32_t vehicle_id, const int32_t* roads, int32_t n_roads, float end_s)
{
    return route_impl(h, -1, vehicle_id, roads, n_roads, end_s);
}

int tsim_batch_set_vehicle_route(tsim_batch* b, int32_t instance, int32_t vehicle_id, const int32_t* roads,
                                 int32_t n_roads, float end_s)
{
    if (!b || instance < 0) return fail(nullptr, TSIM_EINVAL, "bad batch or instance");
    return route_impl(b, instance, vehicle_id, roads, n_roads, end_s);
}

// ---------------------------------------------------------------------------
// Shortest routes on the device (Section 4 "Congestion Pricing"; Appendix F
// road prices; Appendix E routes of shortest time)

// movement graph of a network given as host arrays (one limit per road)
static int route_graph_of_network(const tsim_network* net, RouteGraph& G, std::string* err)
{
    if (!net || net->n_roads < 1 || net->n_jlanes < 0 || !net->road_lane_begin || !net->road_length ||
        !net->road_limit || (net->n_jlanes > 0 && (!net->jl_in_lane || !net->jl_out_lane || !net->jl_length ||
                                                   !net->jl_limit))) {
        *err = "bad network arrays";
        return TSIM_EINVAL;
    }
    const int R = net->n_roads;
    if (net->road_lane_begin[0] != 0) {
        *err = "road_lane_begin must start at 0";
        return TSIM_EINVAL;
    }
    for (int r = 0; r < R; ++r)
        if (net->road_lane_begin[r + 1] <= net->road_lane_begin[r]) {
            *err = "every road needs at least one lane";
            return TSIM_EINVAL;
        }
    const int NRL = net->road_lane_begin[R];
    std::vector<int32_t> road_of(NRL);
    for (int r = 0; r < R; ++r)
        for (int l = net->road_lane_begin[r]; l < net->road_lane_begin[r + 1]; ++l) road_of[l] = r;
    G = RouteGraph{};
    G.R = R;
    G.road_lane_begin.resize(R + 1);
    std::iota(G.road_lane_begin.begin(), G.road_lane_begin.end(), 0);
    G.road_len.assign(net->road_length, net->road_length + R);
    G.lane_lim.assign(net->road_limit, net->road_limit + R);
    std::vector<std::array<int32_t, 3>> mv;   // (from road, to road, junction lane)
    mv.reserve(net->n_jlanes);
    for (int q = 0; q < net->n_jlanes; ++q) {
        const int a = net->jl_in_lane[q], b = net->jl_out_lane[q];
        if (a < 0 || a >= NRL || b < 0 || b >= NRL) {
            *err = "junction lane joins a lane id out of range";
            return TSIM_EINVAL;
        }
        mv.push_back({road_of[a], road_of[b], q});
    }
    std::sort(mv.begin(), mv.end());
    G.e_begin.assign(R + 1, 0);
    size_t c = 0;
    for (int r = 0; r < R; ++r) {
        G.e_begin[r] = (int32_t)G.e_to.size();
        while (c < mv.size() && mv[c][0] == r) {
            const int b = mv[c][1];
            G.e_to.push_back(b);
            G.e_jl_begin.push_back((int32_t)G.jl_len.size());
            for (; c < mv.size() && mv[c][0] == r && mv[c][1] == b; ++c) {
                G.jl_len.push_back(net->jl_length[mv[c][2]]);
                G.jl_lim.push_back(net->jl_limit[mv[c][2]]);
            }
        }
    }
    G.e_begin[R] = (int32_t)G.e_to.size();
    G.e_jl_begin.push_back((int32_t)G.jl_len.size());
    return TSIM_OK;
}

// movement graph of one instance of a handle as it stands: lane limits in
// force, closed junction lanes left out; local road ids
static void route_graph_of_build(const Build& B, const Ranges& g, RouteGraph& G)
{
    G = RouteGraph{};
    G.R = g.r1 - g.r0;
    G.e_begin.assign(G.R + 1, 0);
    std::vector<std::pair<int32_t, int32_t>> mv;   // (to road, junction lane)
    for (int r = 0; r < G.R; ++r) {
        const int rr = g.r0 + r, lb = B.tile_lane_begin[rr], nrl = B.tile_n_road[rr], le = B.tile_lane_begin[rr + 1];
        G.road_lane_begin.push_back((int32_t)G.lane_lim.size());
        for (int m = lb; m < lb + nrl; ++m) G.lane_lim.push_back(B.lane_lim[m]);
        G.road_len.push_back(B.lane_len[lb]);
        mv.clear();
        for (int m = lb + nrl; m < le; ++m)
            if (jl_open(B, m)) mv.push_back({B.jl_out_road[m] - g.r0, m});
        std::sort(mv.begin(), mv.end());
        G.e_begin[r] = (int32_t)G.e_to.size();
        for (size_t c = 0; c < mv.size();) {
            const int b = mv[c].first;
            G.e_to.push_back(b);
            G.e_jl_begin.push_back((int32_t)G.jl_len.size());
            for (; c < mv.size() && mv[c].first == b; ++c) {
                G.jl_len.push_back(B.lane_len[mv[c].second]);
                G.jl_lim.push_back(B.lane_lim[mv[c].second]);
            }
        }
    }
    G.road_lane_begin.push_back((int32_t)G.lane_lim.size());
    G.e_begin[G.R] = (int32_t)G.e_to.size();
    G.e_jl_begin.push_back((int32_t)G.jl_len.size());
}

int tsim_route_footprint(const tsim_network* net, int32_t n_pairs, size_t* min_bytes, size_t* hint_bytes)
{
    if (n_pairs < 0) return fail(nullptr, TSIM_EINVAL, "bad pair count");
    RouteGraph G;
    std::string err;
    const int rc = route_graph_of_network(net, G, &err);
    if (rc) return fail(nullptr, rc, err);
    if (min_bytes) *min_bytes = route_workspace_min(G, n_pairs);
    if (hint_bytes) *hint_bytes = route_workspace_hint(G, n_pairs);
    return TSIM_OK;
}

int tsim_shortest_routes(const tsim_network* net, const float* road_price, const float* road_time,
                         const int32_t* origin, const int32_t* dest, int32_t n, void* hip_stream, void* workspace,
                         size_t workspace_bytes, int32_t* route_begin, int32_t* route_roads, int64_t max_roads,
                         int32_t* n_unreachable)
{
    if (!route_begin || max_roads < 0 || (max_roads > 0 && !route_roads))
        return fail(nullptr, TSIM_EINVAL, "bad output arrays");
    RouteGraph G;
    std::string err;
    int rc = route_graph_of_network(net, G, &err);
    if (rc) return fail(nullptr, rc, err);
    // the routes go straight into the caller's array when they fit
    struct Out : RouteSink {
        int32_t* p;
        int64_t cap;
        int32_t* reserve(int64_t total) override
        {
            return total <= cap && total <= std::numeric_limits<int32_t>::max() ? p : nullptr;
        }
    } out;
    out.p = route_roads;
    out.cap = max_roads;
    std::vector<int64_t> begin;
    int bad = 0;
    rc = route_pairs(G, road_price, road_time, origin, dest, n, (hipStream_t)hip_stream, workspace, workspace_bytes,
                     begin, out, &bad, &err);
    if (!begin.empty() && begin.back() <= std::numeric_limits<int32_t>::max())
        for (size_t p = 0; p < begin.size(); ++p) route_begin[p] = (int32_t)begin[p];
    if (rc == TSIM_ENOMEM && !begin.empty() && begin.back() > max_roads)
        return fail(nullptr, TSIM_ENOMEM, "route_roads holds " + std::to_string(max_roads) +
                                              " roads, the routes need " + std::to_string(begin.back()));
    if (rc) return fail(nullptr, rc, err);
    if (n_unreachable) *n_unreachable = bad;
    return TSIM_OK;
}

static int reroute_footprint_impl(tsim_handle* h, int k, int32_t n, size_t* min_bytes, size_t* hint_bytes)
{
    if (!h || n < 0 || k >= h->B.n_inst || (k < 0 && h->B.n_inst != 1))
        return fail(nullptr, TSIM_EINVAL, "bad arguments");
    RouteGraph G;
    route_graph_of_build(h->B, ranges_of(h->B, k), G);
    if (min_bytes) *min_bytes = route_workspace_min(G, n);
    if (hint_bytes) *hint_bytes = route_workspace_hint(G, n);
    return TSIM_OK;
}

int tsim_reroute_footprint(tsim_handle* h, int32_t n, size_t* min_bytes, size_t* hint_bytes)
{
    return reroute_footprint_impl(h, -1, n, min_bytes, hint_bytes);
}

int tsim_batch_reroute_footprint(tsim_batch* b, int32_t instance, int32_t n, size_t* min_bytes, size_t* hint_bytes)
{
    if (!b || instance < 0) return fail(nullptr, TSIM_EINVAL, "bad batch or instance");
    return reroute_footprint_impl(b, instance, n, min_bytes, hint_bytes);
}

// Every listed vehicle takes the least-cost route from where it is to the
// last road of its route in force (its trip end position kept).  A new route
// is written over the rest of the vehicle's route in force when it fits
// there, else appended to the route pool.
static int reroute_impl(tsim_handle* h, int k, const int32_t* vids_local, int32_t n, const float* price,
                        const float* road_time, void* ws, size_t ws_bytes, int32_t* n_kept)
{
    if (!h || n < 0 || (n > 0 && !vids_local) || k >= h->B.n_inst || (k < 0 && h->B.n_inst != 1))
        return fail(nullptr, TSIM_EINVAL, "bad arguments");
    Build& B = h->B;
    DevNet& D = h->D;
    const Ranges g = ranges_of(B, k);
    const int NV = g.v1 - g.v0;
    std::vector<char> seen(NV, 0);
    for (int c = 0; c < n; ++c) {
        const int v = vids_local[c];
        if (v < 0 || v >= NV) return fail(&h->err, TSIM_EINVAL, "vehicle id out of range");
        if (seen[v]) return fail(&h->err, TSIM_EINVAL, "a vehicle is listed twice");
        seen[v] = 1;
    }
    if (n_kept) *n_kept = 0;
    if (n == 0) return TSIM_OK;
    std::vector<int32_t> st(NV);
    HIPCHK(h, hipMemcpyAsync(st.data(), D.status + g.v0, (size_t)NV * 4, hipMemcpyDeviceToHost, h->stream));
    HIPCHK(h, hipStreamSynchronize(h->stream));
    std::vector<int32_t> lane, rpos, rank;
    std::vector<float> x, v;
    bool any_active = false;
    for (int c = 0; c < n; ++c) any_active |= st[vids_local[c]] == TSIM_ACTIVE;
    if (any_active) {
        const int rc = export_state(h, lane, x, v, rpos, rank);
        if (rc) return rc;
    }
    // start road, the road a vehicle on a junction lane keeps, destination
    struct Job {
        int i, prefix, rp0;
        bool waiting;
    };
    std::vector<Job> jobs;
    std::vector<int32_t> po, pd;
    int kept = 0;
    for (int c = 0; c < n; ++c) {
        const int vl = vids_local[c], i = g.v0 + vl;
        if (st[vl] == TSIM_FINISHED) {
            ++kept;
            continue;
        }
        const int dest = B.route[B.rstart[i] + B.rlen[i] - 1];
        Job J{i, -1, B.rstart[i], st[vl] == TSIM_WAITING};
        int start = B.route[B.rstart[i]];
        if (!J.waiting && lane[i] < 0) {
            ++kept;   // not found on any lane (cannot happen at a step boundary)
            continue;
        }
        if (!J.waiting) {
            const int m = B.int_of_ext[lane[i]];
            const int cur = B.lane_tile[m];
            J.rp0 = B.rstart[i] + rpos[i];
            if (B.jl_out[m] >= 0) {
                J.prefix = cur;
                start = B.jl_out_road[m];
            } else {
                start = cur;
            }
        }
        jobs.push_back(J);
        po.push_back(start - g.r0);
        pd.push_back(dest - g.r0);
    }
    RouteGraph G;
    route_graph_of_build(B, g, G);
    std::vector<int64_t> begin;
    VectorSink sink;
    std::string err;
    int bad = 0;
    int rc = route_pairs(G, price, road_time, po.data(), pd.data(), (int)jobs.size(), h->stream, ws, ws_bytes, begin,
                         sink, &bad, &err);
    if (rc) return fail(&h->err, rc, err);
    const std::vector<int32_t>& roads = sink.roads;
    // install: per-vehicle route position, roads after it, next-road word
    // and (waiting) departure lanes, applied to the records on the device
    const int N = B.N;
    std::vector<int32_t> n_rp(N, -1), n_rem(N, 0), n_nr(N, 0);
    std::vector<uint32_t> n_mask(N, 0);
    std::vector<int32_t> qidx;
    long long lo = std::numeric_limits<long long>::max(), hi = -1;
    std::vector<int32_t> full;
    for (size_t c = 0; c < jobs.size(); ++c) {
        const Job& J = jobs[c];
        const int i = J.i;
        if (begin[c + 1] == begin[c]) {
            ++kept;
            continue;
        }
        full.clear();
        if (J.prefix >= 0) full.push_back(J.prefix);
        for (int64_t e = begin[c]; e < begin[c + 1]; ++e) full.push_back(roads[e] + g.r0);
        const int len = (int)full.size();
        long long pos;
        if ((long long)J.rp0 + len <= (long long)B.rstart[i] + B.rlen[i]) {
            pos = J.rp0;
        } else if ((long long)B.route.size() + len <= h->cap.E) {
            pos = (long long)B.route.size();
            B.route.resize(B.route.size() + len);
        } else {
            ++kept;   // the route pool is full: the vehicle keeps its route
            continue;
        }
        std::copy(full.begin(), full.end(), B.route.begin() + pos);
        lo = std::min(lo, pos);
        hi = std::max(hi, pos + len);
        B.rstart[i] = (int32_t)pos;
        B.rlen[i] = len;
        n_rp[i] = (int32_t)pos;
        n_rem[i] = len - 1;
        n_nr[i] = len > 1 ? full[1] : end_word(B.vend[i], B.lane_len[B.tile_lane_begin[full[len - 1]]]);
        if (J.waiting) {
            if (qidx.empty()) {
                qidx.assign(NV, -1);
                for (int e = B.q_begin[g.r0]; e < B.q_begin[g.r1]; ++e) qidx[B.q_veh[e] - g.v0] = e;
            }
            const uint32_t mask = depart_mask(B, full[0], len > 1 ? full[1] : -1);
            B.q_mask[qidx[i - g.v0]] = mask;
            n_mask[i] = mask;
        }
    }
    if (hi > lo) HIPCHK(h, up_range(h, (int32_t*)D.route, B.route, lo, hi));
    HIPCHK(h, up_range(h, (int32_t*)D.route_begin, B.rstart, g.v0, g.v1));
    HIPCHK(h, hipMemcpyAsync(h->d_io_i0, n_rp.data(), (size_t)N * 4, hipMemcpyHostToDevice, h->stream));
    HIPCHK(h, hipMemcpyAsync(h->d_io_i1, n_rem.data(), (size_t)N * 4, hipMemcpyHostToDevice, h->stream));
    HIPCHK(h, hipMemcpyAsync(h->d_io_i2, n_nr.data(), (size_t)N * 4, hipMemcpyHostToDevice, h->stream));
    HIPCHK(h, hipMemcpyAsync(h->d_io_f0, n_mask.data(), (size_t)N * 4, hipMemcpyHostToDevice, h->stream));
    HIPCHK(h, launch_apply_routes(D, h->d_io_i0, h->d_io_i1, h->d_io_i2, (const uint32_t*)h->d_io_f0,
                                  B.q_begin[B.R], h->stream));
    HIPCHK(h, hipStreamSynchronize(h->stream));
    if (n_kept) *n_kept = kept;
    return TSIM_OK;
}

int tsim_reroute_shortest(tsim_handle* h, const int32_t* vehicle_ids, int32_t n, const float* road_price,
                          const float* road_time, void* workspace, size_t workspace_bytes, int32_t* n_kept)
{
    return reroute_impl(h, -1, vehicle_ids, n, road_price, road_time, workspace, workspace_bytes, n_kept);
}

int tsim_batch_reroute_shortest(tsim_batch* b, int32_t instance, const int32_t* vehicle_ids, int32_t n,
                                const float* road_price, const float* road_time, void* workspace,
                                size_t workspace_bytes, int32_t* n_kept)
{
    if (!b || instance < 0) return fail(nullptr, TSIM_EINVAL, "bad batch or instance");
    return reroute_impl(b, instance, vehicle_ids, n, road_price, road_time, workspace, workspace_bytes, n_kept);
}

int tsim_batch_set_horizon(tsim_batch* b, int32_t instance, int64_t n_steps)
{
    if (!b || instance < 0 || instance >= b->B.n_inst || n_steps < 0)
        return fail(nullptr, TSIM_EINVAL, "bad batch, instance or step count");
    HIPCHK(b, launch_set_end(b->D, instance, (long long)n_steps, b->stream));
    return TSIM_OK;
}

int tsim_batch_set_all_phases(tsim_batch* b, const int32_t* phase_index, int32_t n_total)
{
    if (!b || !phase_index || n_total != b->B.NJ) return fail(nullptr, TSIM_EINVAL, "bad arguments");
    Build& B = b->B;
    for (int j = 0; j < B.NJ; ++j) {
        const int np = B.junc_phase_begin[j + 1] - B.junc_phase_begin[j];
        if (phase_index[j] >= np) return fail(&b->err, TSIM_EINVAL, "phase index out of range");
    }
    int32_t* hp = nullptr;
    int32_t* dp = nullptr;
    int rc = stage_slot(b, &hp, &dp);
    if (rc) return rc;
    std::memcpy(hp, phase_index, (size_t)B.NJ * 4);
    HIPCHK(b, hipMemcpyAsync(dp, hp, (size_t)B.NJ * 4, hipMemcpyHostToDevice, b->stream));
    HIPCHK(b, launch_set_all_phases(b->d_net, b->D, dp, b->stream));
    HIPCHK(b, hipEventRecord(b->pin_ev[b->pin_slot ^ 1], b->stream));
    return TSIM_OK;
}

static int metrics_impl(tsim_handle* h, int inst, tsim_metrics* out)
{
    if (!h || !out) return fail(nullptr, TSIM_EINVAL, "bad arguments");
    if (inst < 0 || inst >= h->B.n_inst) return fail(&h->err, TSIM_EINVAL, "instance out of range");
    HIPCHK(h, launch_fold(h->D, h->stream));
    DevMetrics M;
    HIPCHK(h, hipMemcpyAsync(&M, h->D.met + inst, sizeof(M), hipMemcpyDeviceToHost, h->stream));
    HIPCHK(h, hipStreamSynchronize(h->stream));
    const long long n_veh = h->B.veh_off[inst + 1] - h->B.veh_off[inst];
    std::memset(out, 0, sizeof(*out));
    out->step = M.step;
    out->n_waiting = n_veh - M.departed;
    out->n_active = M.departed - M.finished;
    out->n_finished = M.finished;
    out->sum_travel_time = (double)M.sum_tt_fx / kTimeFx;
    out->att = M.finished > 0 ? out->sum_travel_time / (double)M.finished : 0.0;
    out->mean_speed_last = M.mean_speed_last;
    out->mean_speed_avg = M.speed_steps > 0 ? M.speed_acc / (double)M.speed_steps : 0.0;
    out->vehicle_steps = M.vehicle_steps;
    out->lane_changes = M.lane_changes;
    out->transfers = M.transfers;
    out->clamps = M.clamps;
    out->feeder_blocks = M.feeder_blocks;
    out->departures = M.dep_events;
    out->speed_steps = M.speed_steps;
    out->errors = M.errors;
    out->lane_steps = M.lane_steps;
    out->road_entries = M.road_entries;
    out->stalled_steps = M.stall_steps;
    out->max_stalled_steps = M.max_stall;
    return M.errors ? TSIM_ESTATE : TSIM_OK;
}

int tsim_get_metrics(tsim_handle* h, tsim_metrics* out) { return metrics_impl(h, 0, out); }

int tsim_batch_get_metrics(tsim_batch* b, int32_t instance, tsim_metrics* out)
{
    return metrics_impl(b, instance, out);
}

static int road_speed_impl(tsim_handle* h, int k, float* out, int32_t n_roads)
{
    if (!h || !out || k >= h->B.n_inst || (k < 0 && h->B.n_inst != 1)) return fail(nullptr, TSIM_EINVAL, "bad arguments");
    const Ranges g = ranges_of(h->B, k);
    if (n_roads != g.r1 - g.r0) return fail(&h->err, TSIM_EINVAL, "n_roads differs from the instance's roads");
    HIPCHK(h, hipMemcpyAsync(out, h->D.road_speed + g.r0, (size_t)n_roads * 4, hipMemcpyDeviceToHost, h->stream));
    HIPCHK(h, hipStreamSynchronize(h->stream));
    return TSIM_OK;
}

static int lane_wait_impl(tsim_handle* h, int k, int32_t* out, int32_t n_lanes)
{
    if (!h || !out || k >= h->B.n_inst || (k < 0 && h->B.n_inst != 1)) return fail(nullptr, TSIM_EINVAL, "bad arguments");
    const Ranges g = ranges_of(h->B, k);
    if (n_lanes != g.nrl + g.njl) return fail(&h->err, TSIM_EINVAL, "n_lanes differs from the instance's lanes");
    std::vector<int32_t> tmp(g.m1 - g.m0);
    HIPCHK(h, hipMemcpyAsync(tmp.data(), h->D.lane_wait + g.m0, tmp.size() * 4, hipMemcpyDeviceToHost, h->stream));
    HIPCHK(h, hipStreamSynchronize(h->stream));
    for (int m = g.m0; m < g.m1; ++m) out[local_lane(h->B, g, h->B.ext_of_int[m])] = tmp[m - g.m0];
    return TSIM_OK;
}

int tsim_get_road_mean_speed(tsim_handle* h, float* out, int32_t n_roads) { return road_speed_impl(h, -1, out, n_roads); }

int tsim_get_lane_waiting_counts(tsim_handle* h, int32_t* out, int32_t n_lanes)
{
    return lane_wait_impl(h, -1, out, n_lanes);
}

int tsim_batch_get_road_mean_speed(tsim_batch* b, int32_t instance, float* out, int32_t n_roads)
{
    if (!b || instance < 0) return fail(nullptr, TSIM_EINVAL, "bad batch or instance");
    return road_speed_impl(b, instance, out, n_roads);
}

int tsim_batch_get_lane_waiting_counts(tsim_batch* b, int32_t instance, int32_t* out, int32_t n_lanes)
{
    if (!b || instance < 0) return fail(nullptr, TSIM_EINVAL, "bad batch or instance");
    return lane_wait_impl(b, instance, out, n_lanes);
}

static int export_state(tsim_handle* h, std::vector<int32_t>& lane, std::vector<float>& x, std::vector<float>& v,
                        std::vector<int32_t>& rpos, std::vector<int32_t>& rank)
{
    const int N = h->B.N;
    if (N == 0) return TSIM_OK;
    HIPCHK(h, hipMemsetAsync(h->d_io_i0, 0xFF, (size_t)N * 4, h->stream));
    HIPCHK(h, hipMemsetAsync(h->d_io_f0, 0, (size_t)N * 4, h->stream));
    HIPCHK(h, hipMemsetAsync(h->d_io_f1, 0, (size_t)N * 4, h->stream));
    HIPCHK(h, hipMemsetAsync(h->d_io_i1, 0, (size_t)N * 4, h->stream));
    HIPCHK(h, hipMemsetAsync(h->d_io_i2, 0, (size_t)N * 4, h->stream));
    HIPCHK(h, launch_export(h->d_net, h->D, h->d_lane_ext, h->d_io_i0, h->d_io_f0, h->d_io_f1, h->d_io_i1, h->d_io_i2,
                            h->stream));
    lane.resize(N);
    x.resize(N);
    v.resize(N);
    rpos.resize(N);
    rank.resize(N);
    HIPCHK(h, hipMemcpyAsync(lane.data(), h->d_io_i0, (size_t)N * 4, hipMemcpyDeviceToHost, h->stream));
    HIPCHK(h, hipMemcpyAsync(x.data(), h->d_io_f0, (size_t)N * 4, hipMemcpyDeviceToHost, h->stream));
    HIPCHK(h, hipMemcpyAsync(v.data(), h->d_io_f1, (size_t)N * 4, hipMemcpyDeviceToHost, h->stream));
    HIPCHK(h, hipMemcpyAsync(rpos.data(), h->d_io_i1, (size_t)N * 4, hipMemcpyDeviceToHost, h->stream));
    HIPCHK(h, hipMemcpyAsync(rank.data(), h->d_io_i2, (size_t)N * 4, hipMemcpyDeviceToHost, h->stream));
    HIPCHK(h, hipStreamSynchronize(h->stream));
    return TSIM_OK;
}

static int lane_order_impl(tsim_handle* h, int k, int32_t* offsets, int32_t* vehicle_ids, int32_t n_lanes,
                           int32_t max_ids)
{
    if (!h || !offsets || !vehicle_ids || k >= h->B.n_inst || (k < 0 && h->B.n_inst != 1))
        return fail(nullptr, TSIM_EINVAL, "bad arguments");
    const Ranges g = ranges_of(h->B, k);
    if (n_lanes != g.nrl + g.njl) return fail(&h->err, TSIM_EINVAL, "n_lanes differs from the instance's lanes");
    std::vector<int32_t> lane, rpos, rank;
    std::vector<float> x, v;
    int rc = export_state(h, lane, x, v, rpos, rank);
    if (rc) return rc;
    std::vector<int32_t> cnt(n_lanes + 1, 0);
    for (int i = g.v0; i < g.v1; ++i)
        if (lane[i] >= 0) cnt[local_lane(h->B, g, lane[i]) + 1]++;
    for (int m = 0; m < n_lanes; ++m) cnt[m + 1] += cnt[m];
    if (cnt[n_lanes] > max_ids) return fail(&h->err, TSIM_EINVAL, "vehicle_ids too small");
    for (int m = 0; m <= n_lanes; ++m) offsets[m] = cnt[m];
    for (int i = g.v0; i < g.v1; ++i)
        if (lane[i] >= 0) {
            const int l = local_lane(h->B, g, lane[i]);
            const int pos = cnt[l] + rank[i];
            if (pos >= cnt[l + 1]) return fail(&h->err, TSIM_ESTATE, "inconsistent lane order");
            vehicle_ids[pos] = i - g.v0;
        }
    return TSIM_OK;
}

int tsim_get_lane_order(tsim_handle* h, int32_t* offsets, int32_t* vehicle_ids, int32_t n_lanes, int32_t max_ids)
{
    return lane_order_impl(h, -1, offsets, vehicle_ids, n_lanes, max_ids);
}

int tsim_batch_get_lane_order(tsim_batch* b, int32_t instance, int32_t* offsets, int32_t* vehicle_ids, int32_t n_lanes,
                              int32_t max_ids)
{
    if (!b || instance < 0) return fail(nullptr, TSIM_EINVAL, "bad batch or instance");
    return lane_order_impl(b, instance, offsets, vehicle_ids, n_lanes, max_ids);
}

static int get_state_impl(tsim_handle* h, int inst, tsim_state_host* out)
{
    if (!h || !out || !out->status || !out->lane || !out->route_pos || !out->x || !out->v || !out->finish_step ||
        !out->junc_policy || !out->junc_phase)
        return fail(nullptr, TSIM_EINVAL, "bad arguments");
    Build& B = h->B;
    if (inst < 0 || inst >= B.n_inst) return fail(&h->err, TSIM_EINVAL, "instance out of range");
    const int N = B.N;
    std::vector<int32_t> lane, rpos, rank;
    std::vector<float> x, v;
    int rc = export_state(h, lane, x, v, rpos, rank);
    if (rc) return rc;
    std::vector<int32_t> status(N), finish(N), pol(B.NJ), man(B.NJ);
    HIPCHK(h, launch_fold(h->D, h->stream));
    DevMetrics M;
    HIPCHK(h, hipMemcpyAsync(status.data(), h->D.status, (size_t)N * 4, hipMemcpyDeviceToHost, h->stream));
    HIPCHK(h, hipMemcpyAsync(finish.data(), h->D.finish_step, (size_t)N * 4, hipMemcpyDeviceToHost, h->stream));
    HIPCHK(h, hipMemcpyAsync(pol.data(), h->D.junc_policy, (size_t)B.NJ * 4, hipMemcpyDeviceToHost, h->stream));
    HIPCHK(h, hipMemcpyAsync(man.data(), h->D.junc_manual, (size_t)B.NJ * 4, hipMemcpyDeviceToHost, h->stream));
    HIPCHK(h, hipMemcpyAsync(&M, h->D.met + inst, sizeof(M), hipMemcpyDeviceToHost, h->stream));
    HIPCHK(h, hipStreamSynchronize(h->stream));
    out->step = M.step;
    const Ranges g = ranges_of(B, inst);
    const int vo = g.v0, nv = g.v1 - g.v0;
    for (int k = 0; k < nv; ++k) {
        const int i = vo + k;
        const bool act = status[i] == TSIM_ACTIVE;
        int l = -1;
        if (act) l = local_lane(B, g, lane[i]);
        out->status[k] = status[i];
        out->finish_step[k] = finish[i];
        out->lane[k] = l;
        out->x[k] = act ? x[i] : 0.0f;
        out->v[k] = act ? v[i] : 0.0f;
        out->route_pos[k] = act ? rpos[i] : (status[i] == TSIM_WAITING ? 0 : B.rlen[i] - 1);
    }
    const int jo = B.junc_off[inst], nj = B.junc_off[inst + 1] - jo;
    for (int j = 0; j < nj; ++j) {
        out->junc_policy[j] = pol[jo + j];
        out->junc_phase[j] = man[jo + j];
    }
    return TSIM_OK;
}

int tsim_get_state(tsim_handle* h, tsim_state_host* out) { return get_state_impl(h, 0, out); }

int tsim_batch_get_state(tsim_batch* b, int32_t instance, tsim_state_host* out)
{
    return get_state_impl(b, instance, out);
}

static int set_state_impl(tsim_handle* h, int k, const tsim_state_host* in)
{
    if (!h || !in || !in->status || !in->lane || !in->route_pos || !in->x || !in->v || !in->finish_step ||
        !in->junc_policy || !in->junc_phase || in->step < 0)
        return fail(nullptr, TSIM_EINVAL, "bad arguments");
    if (k >= h->B.n_inst) return fail(&h->err, TSIM_EINVAL, "instance out of range");
    const Ranges g = ranges_of(h->B, k);
    for (int jl = 0; jl < g.j1 - g.j0; ++jl) {
        const int j = g.j0 + jl;
        const int pol = in->junc_policy[jl];
        if (pol < 0 || pol > 3) return fail(&h->err, TSIM_EINVAL, "bad policy");
        const int pb = h->B.junc_phase_begin[j], np = h->B.junc_phase_begin[j + 1] - pb;
        if ((pol == TSIM_POLICY_MANUAL || pol == TSIM_POLICY_MAX_PRESSURE) && np > 0 &&
            (in->junc_phase[jl] < 0 || in->junc_phase[jl] >= np))
            return fail(&h->err, TSIM_EINVAL, "manual or held phase out of range");
        if (pol == TSIM_POLICY_MAX_PRESSURE && np > 0 && !(h->B.phase_dur[pb] > 0))
            return fail(&h->err, TSIM_EINVAL, "max-pressure junction with a non-positive first phase duration");
    }
    return upload_state(h, k, in->step, in->status, in->lane, in->route_pos, in->x, in->v, in->finish_step,
                        in->junc_policy, in->junc_phase);
}

int tsim_set_state(tsim_handle* h, const tsim_state_host* in)
{
    if (h && h->B.n_inst != 1) return fail(&h->err, TSIM_EINVAL, "tsim_set_state on a batch: use tsim_batch_set_state");
    return set_state_impl(h, -1, in);
}

int tsim_batch_set_state(tsim_batch* b, int32_t instance, const tsim_state_host* in)
{
    if (!b || instance < 0) return fail(nullptr, TSIM_EINVAL, "bad batch or instance");
    return set_state_impl(b, instance, in);
}

int tsim_destroy(tsim_handle* h)
{
    if (!h) return fail(nullptr, TSIM_EINVAL, "null handle");
    (void)hipStreamSynchronize(h->stream);
    for (int k = 0; k < 2; ++k)
        for (auto& e : h->ev[k]) (void)hipEventDestroy(e);
    if (h->graph) (void)hipGraphExecDestroy(h->graph);
    if (h->cap_stream) (void)hipStreamDestroy(h->cap_stream);
    for (int i = 0; i < 3; ++i) {
        if (h->ps.aux[i]) (void)hipStreamDestroy(h->ps.aux[i]);
        if (h->ps.join[i]) (void)hipEventDestroy(h->ps.join[i]);
    }
    if (h->ps.fork) (void)hipEventDestroy(h->ps.fork);
    for (int k = 0; k < 2; ++k) {
        if (h->pin_ev[k]) (void)hipEventDestroy(h->pin_ev[k]);
        if (h->h_pin[k]) (void)hipHostFree(h->h_pin[k]);
    }
    delete h;
    return TSIM_OK;
}

int tsim_batch_step(tsim_batch* b, int32_t n_steps) { return tsim_step(b, n_steps); }

int tsim_batch_set_graph_steps(tsim_batch* b, int32_t chunk) { return tsim_set_graph_steps(b, chunk); }

int tsim_batch_destroy(tsim_batch* b) { return tsim_destroy(b); }

// ---------------------------------------------------------------------------
// instances joining and leaving a running batch
// ---------------------------------------------------------------------------
}  // extern "C"

struct tsim_instance {
    Build B;
    tsim_params params{};
};

namespace {

// appends the tables of a single-instance build M (instance key from seed)
// to the batch's host tables; returns the span of the new entries, or sets
// the error and returns false when the reserved capacity is exceeded
bool append_build(tsim_handle* h, const Build& M, uint64_t seed, Span& sp)
{
    Build& B = h->B;
    const Caps& c = h->cap;
    const int R0 = B.R, NJ0 = B.NJ, NL0 = B.NL, N0 = B.N, k = B.n_inst;
    const int NRL0 = B.rl_off.back(), NJL0 = B.jl_off.back();
    const long long S0 = (long long)B.slots, P0 = (long long)B.phase_dur.size(), E0 = (long long)B.route.size();
    const int Q0 = (int)B.out_jl.size(), QV0 = (int)B.q_veh.size();
    if (k + 1 > c.n_inst || R0 + M.R > c.R || NJ0 + M.NJ > c.NJ || NL0 + M.NL > c.NL || NRL0 + M.NRL > c.NRL ||
        NJL0 + M.NJL > c.NJL || N0 + M.N > c.N || S0 + (long long)M.slots > c.S ||
        P0 + (long long)M.phase_dur.size() > c.P || E0 + (long long)M.route.size() > c.E) {
        h->err = "the instance does not fit the batch's remaining capacity";
        return false;
    }
    auto uext = [&](int e) { return e < M.NRL ? NRL0 + e : B.NRL + NJL0 + (e - M.NRL); };
    for (int r = 0; r < M.R; ++r) {
        B.tile_lane_begin.push_back(M.tile_lane_begin[r + 1] + NL0);
        B.tile_n_road.push_back(M.tile_n_road[r]);
        B.q_begin.push_back(M.q_begin[r + 1] + QV0);
        B.tile_inst.push_back(k);
    }
    for (int m = 0; m < M.NL; ++m) {
        const bool jl = M.jl_out[m] >= 0;
        B.lane_len.push_back(M.lane_len[m]);
        B.lane_lim.push_back(M.lane_lim[m]);
        B.lane_base.push_back((uint32_t)(M.lane_base[m] + S0));
        B.lane_cap.push_back(M.lane_cap[m]);
        B.lane_tile.push_back(M.lane_tile[m] + R0);
        B.lane_local.push_back(M.lane_local[m]);
        B.jl_out.push_back(jl ? M.jl_out[m] + NL0 : -1);
        B.jl_junc.push_back(jl ? M.jl_junc[m] + NJ0 : 0);
        B.jl_green_mask.push_back(M.jl_green_mask[m]);
        B.jl_ext.push_back(jl ? M.jl_ext[m] + NJL0 : -1);
        B.jl_in_local.push_back(M.jl_in_local[m]);
        B.jl_out_road.push_back(jl ? M.jl_out_road[m] + R0 : -1);
        B.out_begin.push_back(M.out_begin[m + 1] + Q0);
        B.feed_begin.push_back(M.feed_begin[m + 1] + Q0);
        const int e = uext(M.ext_of_int[m]);
        B.ext_of_int[NL0 + m] = e;
        B.int_of_ext[e] = NL0 + m;
    }
    if (!M.restricted.empty()) {
        B.restricted.resize(NL0 + M.NL, 0);
        std::copy(M.restricted.begin(), M.restricted.end(), B.restricted.begin() + NL0);
    }
    for (int q : M.out_jl) B.out_jl.push_back(q + NL0);
    for (int q : M.feed_jl) B.feed_jl.push_back(q + NL0);
    for (int j = 0; j < M.NJ; ++j) {
        B.junc_phase_begin.push_back(M.junc_phase_begin[j + 1] + (int)P0);
        B.junc_policy.push_back(M.junc_policy[j]);
        B.junc_cycle.push_back(M.junc_cycle[j]);
        B.mp_begin.push_back(M.mp_begin[j + 1] + Q0);
        B.junc_inst.push_back(k);
    }
    for (size_t q = 0; q < M.mp_mov.size(); q += 4) {
        B.mp_mov.push_back(M.mp_mov[q] + NL0);
        B.mp_mov.push_back(M.mp_mov[q + 1] + NL0);
        B.mp_mov.push_back(M.mp_mov[q + 2]);
        B.mp_mov.push_back(0);
    }
    for (float d : M.phase_dur) B.phase_dur.push_back(d);
    for (int i = 0; i < M.N; ++i) {
        B.tau.push_back(M.tau[i]);
        B.vf.push_back(M.vf[i]);
        B.vlen.push_back(M.vlen[i]);
        B.vend.push_back(M.vend[i]);
        B.vstart.push_back(M.vstart[i]);
        B.route_begin.push_back(M.route_begin[i + 1] + (int)E0);
        B.rstart.push_back(M.rstart[i] + (int)E0);
        B.rlen.push_back(M.rlen[i]);
    }
    for (int r : M.route) B.route.push_back(r + R0);
    for (size_t q = 0; q < M.q_veh.size(); ++q) {
        B.q_veh.push_back(M.q_veh[q] + N0);
        B.q_mask.push_back(M.q_mask[q]);
    }
    B.slots += M.slots;
    B.R += M.R;
    B.NJ += M.NJ;
    B.NL += M.NL;
    B.N += M.N;
    B.NJL += M.NJL;
    B.n_inst += 1;
    B.inst_vbase.push_back(N0);
    B.inst_key.push_back((uint32_t)seed);
    B.inst_key.push_back((uint32_t)(seed >> 32));
    B.inst_t0.push_back(0);
    B.road_off.push_back(B.R);
    B.junc_off.push_back(B.NJ);
    B.rl_off.push_back(NRL0 + M.NRL);
    B.jl_off.push_back(NJL0 + M.NJL);
    B.veh_off.push_back(B.N);
    sp = Span{R0, B.R, NL0, B.NL, NJ0, B.NJ, N0, B.N, Q0, (int)B.out_jl.size(), (int)P0, (int)B.phase_dur.size(), k,
              k + 1, E0, (long long)B.route.size()};
    return true;
}

// removes the last instance's entries from the host tables
void pop_build(tsim_handle* h)
{
    Build& B = h->B;
    const int k = B.n_inst - 1;
    const int r0 = B.road_off[k], j0 = B.junc_off[k], v0 = B.veh_off[k];
    const int m0 = B.tile_lane_begin[r0];
    const int q0 = B.out_begin[m0], qv0 = B.q_begin[r0];
    const int p0 = B.junc_phase_begin[j0];
    // the route pool keeps every route in force of the remaining instances
    // (routes changed after an instance joined are appended after it)
    int e0 = B.route_begin[v0];
    for (int i = 0; i < v0; ++i) e0 = std::max(e0, B.rstart[i] + B.rlen[i]);
    const uint64_t s0 = m0 < (int)B.lane_base.size() ? B.lane_base[m0] : B.slots;
    for (int m = m0; m < B.NL; ++m) B.int_of_ext[B.ext_of_int[m]] = -1;
    B.tile_lane_begin.resize(r0 + 1);
    B.tile_n_road.resize(r0);
    B.q_begin.resize(r0 + 1);
    B.tile_inst.resize(r0);
    for (auto* v : {&B.lane_cap, &B.lane_tile, &B.lane_local, &B.jl_out, &B.jl_junc, &B.jl_ext, &B.jl_in_local,
                    &B.jl_out_road})
        v->resize(m0);
    B.lane_len.resize(m0);
    B.lane_lim.resize(m0);
    if ((int)B.restricted.size() > m0) B.restricted.resize(m0);
    B.lane_base.resize(m0);
    B.jl_green_mask.resize(m0);
    B.out_begin.resize(m0 + 1);
    B.feed_begin.resize(m0 + 1);
    B.out_jl.resize(q0);
    B.feed_jl.resize(q0);
    B.junc_phase_begin.resize(j0 + 1);
    B.junc_policy.resize(j0);
    B.junc_cycle.resize(j0);
    B.mp_begin.resize(j0 + 1);
    B.mp_mov.resize(4 * (size_t)q0);
    B.junc_inst.resize(j0);
    B.phase_dur.resize(p0);
    B.tau.resize(v0);
    B.vf.resize(v0);
    B.vlen.resize(v0);
    B.vend.resize(v0);
    B.vstart.resize(v0);
    B.route_begin.resize(v0 + 1);
    B.route.resize(e0);
    B.rstart.resize(v0);
    B.rlen.resize(v0);
    B.q_veh.resize(qv0);
    B.q_mask.resize(qv0);
    B.slots = s0;
    B.R = r0;
    B.NJ = j0;
    B.NL = m0;
    B.N = v0;
    B.NJL = B.jl_off[k];
    B.n_inst = k;
    B.inst_vbase.resize(k);
    B.inst_key.resize(2 * (size_t)k);
    B.inst_t0.resize(k);
    for (auto* v : {&B.road_off, &B.junc_off, &B.rl_off, &B.jl_off, &B.veh_off}) v->resize(k + 1);
}

// after the batch's instances changed: sizes and grids, the device view, and
// no captured graph of the old launches
int batch_changed(tsim_handle* h)
{
    refresh_view(h);
    if (h->graph) {
        (void)hipGraphExecDestroy(h->graph);
        h->graph = nullptr;
    }
    HIPCHK(h, hipMemcpyAsync(h->d_net, &h->D, sizeof(DevNet), hipMemcpyHostToDevice, h->stream));
    return TSIM_OK;
}

bool same_model(const tsim_params& a, const tsim_params& b)
{
    return a.dt == b.dt && a.T == b.T && a.a_max == b.a_max && a.b_comf == b.b_comf && a.s0 == b.s0 &&
           a.delta == b.delta && a.politeness == b.politeness && a.a_th == b.a_th && a.b_safe == b.b_safe &&
           a.p_max == b.p_max && a.p_min == b.p_min && a.a_emerg == b.a_emerg;
}

// appends a built instance and uploads its tables; the state follows
int add_impl(tsim_handle* b, const Build& M, const tsim_params& prm, int32_t* instance)
{
    if (!same_model(prm, b->params))
        return fail(&b->err, TSIM_EINVAL, "batch instances must share every parameter but the seed");
    // the step still pending is folded under the view it ran with (one
    // instance folds workgroup partials, several fold per-instance sums)
    HIPCHK(b, launch_fold(b->D, b->stream));
    HIPCHK(b, hipStreamSynchronize(b->stream));
    Span sp;
    if (!append_build(b, M, prm.seed, sp)) return fail(&b->err, TSIM_ENOMEM, b->err);
    b->removed.push_back(0);
    int rc = upload_tables(b, sp);
    if (rc == TSIM_OK) rc = batch_changed(b);
    if (rc) return rc;
    *instance = b->B.n_inst - 1;
    return TSIM_OK;
}

void fill_capacity(const Caps& c, tsim_batch_capacity* out)
{
    out->instances = (int32_t)c.n_inst;
    out->junctions = (int32_t)c.NJ;
    out->roads = (int32_t)c.R;
    out->road_lanes = (int32_t)c.NRL;
    out->jlanes = (int32_t)c.NJL;
    out->phases = (int32_t)c.P;
    out->vehicles = (int32_t)c.N;
    out->route_entries = c.E;
    out->slots = c.S;
}

int caps_from(const tsim_batch_capacity* cap, Caps& c)
{
    if (!cap || cap->instances < 0 || cap->junctions < 0 || cap->roads < 0 || cap->road_lanes < 0 || cap->jlanes < 0 ||
        cap->phases < 0 || cap->vehicles < 0 || cap->route_entries < 0 || cap->slots < 0 || cap->slots >= (1ll << 31))
        return TSIM_EINVAL;
    c.n_inst = cap->instances;
    c.NJ = cap->junctions;
    c.R = cap->roads;
    c.NRL = cap->road_lanes;
    c.NJL = cap->jlanes;
    c.NL = (long long)cap->road_lanes + cap->jlanes;
    c.P = cap->phases;
    c.N = cap->vehicles;
    c.E = cap->route_entries;
    c.S = cap->slots;
    c.G = g_bound((int)c.R);
    return TSIM_OK;
}

}  // namespace

extern "C" {

int tsim_instance_build(const tsim_network* net, const tsim_trips* trips, const tsim_params* params,
                        tsim_instance** out)
{
    if (!out) return fail(nullptr, TSIM_EINVAL, "null out");
    *out = nullptr;
    tsim_instance* in = new (std::nothrow) tsim_instance();
    if (!in) return fail(nullptr, TSIM_ENOMEM, "host allocation failed");
    const int rc = build_tables(net, trips, params, in->B, nullptr);
    if (rc) {
        delete in;
        return rc;
    }
    single_instance(in->B, params);
    in->params = *params;
    *out = in;
    return TSIM_OK;
}

int tsim_instance_free(tsim_instance* in)
{
    delete in;
    return TSIM_OK;
}

int tsim_instance_capacity(const tsim_instance* in, tsim_batch_capacity* out)
{
    if (!in || !out) return fail(nullptr, TSIM_EINVAL, "bad arguments");
    Caps c = caps_of(in->B);
    fill_capacity(c, out);
    return TSIM_OK;
}

int tsim_batch_reserve_footprint(const tsim_batch_capacity* cap, size_t* bytes_out)
{
    if (!bytes_out) return fail(nullptr, TSIM_EINVAL, "null bytes_out");
    tsim_handle tmp;
    if (caps_from(cap, tmp.cap)) return fail(nullptr, TSIM_EINVAL, "bad capacity");
    *bytes_out = arena_size(&tmp) + 256;
    return TSIM_OK;
}

int tsim_batch_reserve(const tsim_batch_capacity* cap, const tsim_params* params, void* hip_stream,
                       void* device_arena, size_t arena_bytes, tsim_batch** out)
{
    if (!out || !params || !device_arena) return fail(nullptr, TSIM_EINVAL, "bad arguments");
    *out = nullptr;
    if (!(params->dt > 0) || !(params->a_max > 0) || !(params->b_comf > 0) || !(params->T >= 0) || !(params->s0 >= 0))
        return fail(nullptr, TSIM_EINVAL, "bad parameters");
    tsim_handle* h = new (std::nothrow) tsim_handle();
    if (!h) return fail(nullptr, TSIM_ENOMEM, "host allocation failed");
    if (caps_from(cap, h->cap)) {
        delete h;
        return fail(nullptr, TSIM_EINVAL, "bad capacity");
    }
    // an empty union: external road lanes of later instances from 0, their
    // junction lanes after the reserved road lanes
    Build& B = h->B;
    B.NRL = (int)h->cap.NRL;
    B.n_inst = 0;
    B.tile_lane_begin.assign(1, 0);
    B.out_begin.assign(1, 0);
    B.feed_begin.assign(1, 0);
    B.junc_phase_begin.assign(1, 0);
    B.mp_begin.assign(1, 0);
    B.route_begin.assign(1, 0);
    B.q_begin.assign(1, 0);
    B.int_of_ext.assign(h->cap.NRL + h->cap.NJL, -1);
    B.ext_of_int.assign(h->cap.NL, -1);
    for (auto* v : {&B.road_off, &B.junc_off, &B.rl_off, &B.jl_off, &B.veh_off}) v->assign(1, 0);
    count_tiles(B);
    return create_impl(h, params, hip_stream, device_arena, arena_bytes, out);
}

int tsim_batch_add(tsim_batch* b, const tsim_instance* in, int32_t* instance)
{
    if (!b || !in || !instance) return fail(nullptr, TSIM_EINVAL, "bad arguments");
    int rc = add_impl(b, in->B, in->params, instance);
    if (rc) return rc;
    // a fresh instance: every vehicle waiting at local step 0
    const Build& M = in->B;
    std::vector<int32_t> st(M.N, TSIM_WAITING), lane(M.N, -1), rpos(M.N, 0), fs(M.N, -1);
    std::vector<float> xz(M.N, 0.f), vz(M.N, 0.f);
    std::vector<int32_t> zero_nj(M.NJ, 0);
    return upload_state(b, *instance, 0, st.data(), lane.data(), rpos.data(), xz.data(), vz.data(), fs.data(),
                        M.junc_policy.data(), zero_nj.data());
}

int tsim_batch_add_member(tsim_batch* b, tsim_handle* member, int32_t* instance)
{
    if (!b || !member || !instance || member == b || member->B.n_inst != 1)
        return fail(nullptr, TSIM_EINVAL, "bad arguments (the member must be a single-instance handle)");
    const Build& M = member->B;
    std::vector<int32_t> status(M.N), lane(M.N), rpos(M.N), fs(M.N), pol(M.NJ), ph(M.NJ);
    std::vector<float> x(M.N), v(M.N);
    tsim_state_host st{0, status.data(), lane.data(), rpos.data(), x.data(), v.data(), fs.data(), pol.data(), ph.data()};
    int rc = tsim_get_state(member, &st);
    if (rc) return rc;
    rc = add_impl(b, M, member->params, instance);
    if (rc) return rc;
    return upload_state(b, *instance, st.step, status.data(), lane.data(), rpos.data(), x.data(), v.data(), fs.data(),
                        pol.data(), ph.data());
}

int tsim_batch_remove(tsim_batch* b, int32_t instance)
{
    if (!b || instance < 0 || instance >= b->B.n_inst || b->removed[instance])
        return fail(nullptr, TSIM_EINVAL, "bad batch or instance");
    // frozen from its current local step on (no further change of any kind)
    tsim_metrics m;
    int rc = metrics_impl(b, instance, &m);
    if (rc && rc != TSIM_ESTATE) return rc;
    HIPCHK(b, launch_set_end(b->D, instance, (long long)m.step, b->stream));
    HIPCHK(b, hipStreamSynchronize(b->stream));
    b->removed[instance] = 1;
    // its AOIs go with it (the caller's buffer is no longer referenced)
    if ((size_t)instance < b->aois.size()) b->aois[instance] = tsim_handle::AoiSet{};
    // trailing removed instances give their space back
    bool popped = false;
    while (b->B.n_inst > 0 && b->removed.back()) {
        pop_build(b);
        b->removed.pop_back();
        popped = true;
    }
    if (b->aois.size() > (size_t)b->B.n_inst) b->aois.resize((size_t)b->B.n_inst);
    return popped ? batch_changed(b) : TSIM_OK;
}

int tsim_batch_capacity_left(tsim_batch* b, tsim_batch_capacity* out)
{
    if (!b || !out) return fail(nullptr, TSIM_EINVAL, "bad arguments");
    const Build& B = b->B;
    Caps c = b->cap;
    c.n_inst -= B.n_inst;
    c.R -= B.R;
    c.NJ -= B.NJ;
    c.NL -= B.NL;
    c.NRL -= B.rl_off.back();
    c.NJL -= B.jl_off.back();
    c.N -= B.N;
    c.S -= (long long)B.slots;
    c.P -= (long long)B.phase_dur.size();
    c.E -= (long long)B.route.size();
    fill_capacity(c, out);
    return TSIM_OK;
}

int tsim_batch_num_instances(tsim_batch* b, int32_t* n)
{
    if (!b || !n) return fail(nullptr, TSIM_EINVAL, "bad arguments");
    *n = b->B.n_inst;
    return TSIM_OK;
}

const char* tsim_last_error(const tsim_handle* h)
{
    if (h && !h->err.empty()) return h->err.c_str();
    return g_error.c_str();
}

}  // extern "C"
