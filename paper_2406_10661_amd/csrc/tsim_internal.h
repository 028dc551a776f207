// Internal device layout of the gfx950 stepper (not part of the C ABI).
//
// Vehicles live in lane slabs: every lane owns a fixed-capacity run of
// 32-byte records, front vehicle first.  Two slab buffers alternate by step
// parity: step t reads buffer t&1 (the snapshot of Section 3.1's two-phase
// process) and writes buffer (t+1)&1, so no vehicle ever reads a value written
// in the same step.  A lane's capacity follows from the no-overlap invariant:
// floor(length / shortest vehicle) + 2.
//
// Work is organised by road tiles: tile r holds the road lanes of road r
// followed by the junction lanes that leave it, so every lane change and every
// road-to-junction transfer stays inside one tile; only junction-to-road
// transfers cross tiles, through a one-record inbox per road lane that the
// next prepare kernel appends at the lane rear.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace tsim {

constexpr int kMaxTileLanes = 64;    // road lanes + junction lanes of one road
constexpr int kMaxRoadLanes = 32;
constexpr int kMaxPhases = 32;
constexpr int kWave = 64;
constexpr int kChangerCap = 64;      // lane changers per tile kept in LDS (wide tiles)
constexpr int kMergeCap = 64;        // merging vehicles per tile kept in LDS (wide tiles)
constexpr int kWideLanes = 32;       // lanes of a tile of the wide list
constexpr int kWideCap = 128;        // vehicles of a tile of the wide list (staged in LDS)
constexpr int kHugeCap = 512;        // vehicles of a huge tile staged in LDS (more: global scratch)
constexpr int kNoGate = 0x7FFFFFFF;  // no feeder holds the lane
constexpr int kNoFeeder = (int)0x80000000;  // no nonempty feeder
constexpr int kNoAllocMaxUpdates = 1 << 18; // junction updates per tsim_set_signal_phases_noalloc call

// Update schedules: how road tiles map onto wavefronts.  A tile of at most
// `width` lanes that holds at most `cap` vehicles goes to a group of `width`
// lanes of a wavefront (64 / width tiles per wavefront); other tiles run one
// per wavefront in the wide pass.
enum Schedule {
    kSchedWide = 0,
    kSched16x32 = 1,
    kSched16x64 = 2,
    kSched32x64 = 3,
    kSched8x16 = 4,
    kSched16x32P = 5,   // as 16x32, with the wide pass software-pipelined like the grouped one
    kSched8and16 = 6,   // as 16x32P, with tiles of <= 8 lanes and <= 16 vehicles in groups of 8
    kSchedFused = 7,    // the lists of 8and16, all passes in one launch
    kNumSched = 8
};
constexpr int kCntStride = 32;           // work-list counters one 128-byte line apart
constexpr int kNumLists = 6;             // small, wide, huge, tiny, medium, large
constexpr int kFoldWGs = 16;             // prepare workgroups that sum slices of the previous step's partials
constexpr int kMedCap = 64;              // medium tiles (fused schedule): at most kWideLanes lanes and 64 vehicles
constexpr int kLargeCap = 176;           // large tiles (fused schedule): above the wide list, at most 176 vehicles
                                         // (two images fit the fused launch's LDS; larger tiles go to the huge list)
constexpr int kLargeLanes = 48;          // and at most 48 lanes
constexpr float kSpeedFx = 1048576.0f;   // fixed-point scale of speed sums (2^20)
constexpr double kTimeFx = 65536.0;      // fixed-point scale of travel times (2^16)
constexpr int kWaitSpeedFlag = 0;

struct __align__(16) VehRec {
    float x;      // front-bumper coordinate along the lane
    float v;      // speed
    int32_t vid;  // vehicle id
    float len;    // vehicle length
    float f;      // desired-speed factor (v0 = f * lane limit)
    int32_t rp;   // index into the route array of the current road
    int32_t rem;  // roads of the route after the current one
    int32_t nr;   // next road of the route; on the last road (rem == 0) the trip end position's word (end_word)
};

// one departure queue entry with everything the prepare kernel needs to
// place the vehicle (one 32-byte load instead of a chain through the trip
// tables)
struct __align__(16) QRec {
    float tau;       // departure time
    uint32_t mask;   // origin-road lanes (bits) that lead to the next road
    int32_t vid;
    float len;
    float f;         // desired-speed factor
    int32_t rp;      // route position of the origin road
    int32_t rem;     // roads after the origin road
    int32_t nr;      // next road; on a one-road route the trip end position's word (end_word)
};

// per-lane summary of one step's state, read by other tiles (lookahead,
// merge priority, departure safety) so that one 32-byte load serves them
struct __align__(32) LaneSum {
    int32_t cnt;        // vehicles in the lane
    float rear;         // rearmost vehicle's rear bumper (x - length)
    float rear_v;       // its speed
    float front_reach;  // front vehicle's x + v dt + a_max dt^2/2 - lane length
    // feeder gates of a road lane (built with 64-bit atomicMax by the tiles
    // that write its feeders' front vehicles), each tagged in its high word
    // with the step that reads it plus one, so an entry left from an earlier
    // step is simply stale and nothing is ever cleared:
    //   gate: smallest external index of a nonempty feeder whose front
    //         vehicle can cross the lane end within the step (kNoGate if none)
    //   fmax: largest front reach of a nonempty feeder (kNoFeeder if none)
    uint64_t gate;
    uint64_t fmax;
};

// tagged gate words (see LaneSum); `step` is the global step that reads them
__host__ __device__ inline uint32_t gate_tag(long long step) { return (uint32_t)(step + 1); }
__host__ __device__ inline uint64_t gate_key(long long step, int ext)
{
    return ((uint64_t)gate_tag(step) << 32) | (uint64_t)(0xFFFFFFFFu - (uint32_t)ext);
}
__host__ __device__ inline int gate_of(uint64_t w, long long step)
{
    return (uint32_t)(w >> 32) == gate_tag(step) ? (int)(0xFFFFFFFFu - (uint32_t)w) : kNoGate;
}
__host__ __device__ inline uint64_t fmax_key(long long step, int ordered_reach)
{
    return ((uint64_t)gate_tag(step) << 32) | (uint64_t)((uint32_t)ordered_reach ^ 0x80000000u);
}
__host__ __device__ inline int fmax_of(uint64_t w, long long step)
{
    return (uint32_t)(w >> 32) == gate_tag(step) ? (int)((uint32_t)w ^ 0x80000000u) : kNoFeeder;
}

// static per-lane tables, one 48-byte record per lane so that a tile's lanes
// load as one contiguous run
struct __align__(16) LaneInfo {
    uint32_t base;        // first slab slot
    int32_t cap;          // slab capacity
    float len;
    float lim;
    int32_t jl_out;       // junction lanes: out lane (internal), else -1
    int32_t jl_out_road;  // its road; -2 while the junction lane is closed (it, or its out lane, restricted)
    int32_t jl_junc;      // junction
    uint32_t green_mask;  // phases in which it is green
    int32_t jl_ext;       // external junction-lane index (feeder priority)
    int32_t jl_in_local;  // local index of its in lane within the tile
    int32_t flags;        // road lanes: bit 0 set while the lane is restricted (no lane change into it)
    int32_t pad1;
};

// A vehicle record's next-road word: on the last road of the trip (no next
// road) it holds the trip's end position instead, as float bits: end_s when
// it lies before the road's end, else the road's end
__host__ __device__ inline int32_t end_word(float end_s, float road_len)
{
    const float e = (end_s >= 0.0f && end_s < road_len) ? end_s : road_len;
    int32_t w;
    __builtin_memcpy(&w, &e, 4);
    return w;
}
__host__ __device__ inline float word_end(int32_t w)
{
    float e;
    __builtin_memcpy(&e, &w, 4);
    return e;
}

// order-preserving map of floats to ints (for atomicMax on floats)
__host__ __device__ inline int f2o(float f)
{
    int i;
    __builtin_memcpy(&i, &f, 4);
    return i >= 0 ? i : i ^ 0x7FFFFFFF;
}
__host__ __device__ inline float o2f(int i)
{
    const int b = i >= 0 ? i : i ^ 0x7FFFFFFF;
    float f;
    __builtin_memcpy(&f, &b, 4);
    return f;
}

struct KParams {
    float dt, T, a_max, s0, delta, p, a_th, b_safe, p_max, p_min, a_emerg;
    float inv_2sqrt_ab;  // 1 / (2 sqrt(a_max b_comf))
    float reach;         // a_max dt^2 / 2
    double dt_d;
    uint32_t key0, key1; // Philox key
    int delta_is_4;
};

// one vehicle's state at a recorded step boundary (trajectory output)
struct TrajRec {
    int64_t step;   // the step about to run (the state is the end of step - 1)
    int32_t vid;
    int32_t lane;   // external lane id
    float x, v;
};
static_assert(sizeof(TrajRec) == 24, "trajectory records are 24 bytes");

// cumulative metrics; a step's sums are folded in by the next step's prepare
// kernel, or before the host reads them
struct DevMetrics {
    long long step;
    long long departed;
    long long finished;
    long long sum_tt_fx;
    long long vehicle_steps;
    long long lane_changes;
    long long transfers;
    long long clamps;
    long long feeder_blocks;
    long long errors;
    long long speed_steps;
    long long dep_events;    // departures since create / set_state
    long long lane_steps;    // sum over steps of lanes holding vehicles at the step start
    long long road_entries;  // junction-to-road crossings (each reads one route word)
    long long stall_steps;   // gridlock detector: current run of steps in which nothing moved
    long long max_stall;     // its longest run
    long long stall_dep;     // departures counted at the last fold
    double speed_acc;
    double mean_speed_last;
};

// per-workgroup partial sums of one step
struct WGPartial {
    long long sumv_fx, cnt, active, changes, transfers, clamps, feeder_blocks, finished, sum_tt_fx, errors,
        lanes_busy, road_entries;
};
constexpr int kPartWords = 12;
static_assert(sizeof(WGPartial) == 8 * kPartWords && kPartWords % 2 == 0,
              "the fold reads partials as 16-byte words");

struct DevNet {
    int32_t R, NJ, NL, N, G;     // roads, junctions, lanes, vehicles, update grid size
    // instances (a batch is the disjoint union of several networks)
    int32_t n_inst;
    const int32_t* tile_inst;        // [R] instance of each road tile
    const int32_t* junc_inst;        // [NJ]
    const int32_t* inst_vbase;       // [n_inst] first vehicle id of each instance
    const uint32_t* inst_key;        // [2 n_inst] Philox key of each instance
    const long long* inst_t0;        // [n_inst] global step at which the instance starts
    long long* inst_end;             // [n_inst] local step from which the instance is frozen
    WGPartial* inst_acc;             // [n_inst] sums of the current step (batches)
    long long* gstep;                // global step counter
    // tiles
    const int32_t* tile_lane_begin;  // [R+1]
    const int32_t* tile_n_road;      // [R]
    // lanes (internal ids)
    const LaneInfo* lane_info;       // [NL]
    const float* lane_len;
    const float* lane_lim;
    const uint32_t* lane_base;
    const int32_t* lane_cap;
    const int32_t* lane_tile;        // tile (road) owning the lane
    const int32_t* lane_local;       // index within its tile
    const int32_t* jl_out;           // out lane (internal) of a junction lane, -1 for road lanes
    const int32_t* jl_out_local;     // local index of that out lane within its own tile
    const int32_t* jl_junc;          // junction of a junction lane
    const uint32_t* jl_green_mask;   // phases (bit index) in which it is green
    const int32_t* jl_ext;           // external junction-lane index (feeder priority)
    const int32_t* jl_in_local;      // local index of its in lane within the tile
    const int32_t* jl_out_road;      // road of its out lane
    const int32_t* out_begin;        // [NL+1] junction lanes leaving a road lane
    const int32_t* out_jl;
    const int2* out_pair;            // per out_jl entry: (road of its out lane, junction lane)
    const int32_t* feed_begin;       // [NL+1] junction lanes entering a road lane, by external id
    const int32_t* feed_jl;
    // junctions
    const int32_t* junc_phase_begin; // [NJ+1]
    const int32_t* mp_begin;         // [NJ+1] movements (junction lanes) of each junction
    const int4* mp_mov;              // (in road lane, out road lane, green phase mask, 0), internal lane ids
    const float* phase_dur;
    const double* junc_cycle;
    int32_t* junc_policy;
    int32_t* junc_manual;            // MANUAL phase, or the phase a MAX_PRESSURE junction holds
    int32_t* junc_cur;               // phase index of the current step, -1 = all green
    // vehicles
    const float* tau;
    const int32_t* route_begin;
    const int32_t* route;
    const float* vf;
    const float* vlen;
    const float* vend;               // [N] trip end position on the last road, < 0: its end
    const float* vstart;             // [N] trip start position on the origin road, 0: its start
    int32_t* status;
    int32_t* finish_step;
    const int32_t* q_begin;          // [R+1] departure queue of each origin road
    const QRec* q_rec;               // [N] departure queue entries
    int32_t* q_head;
    // slabs
    VehRec* slab0;
    VehRec* slab1;
    LaneSum* sum0;                   // lane summaries read at even steps
    LaneSum* sum1;                   // lane summaries read at odd steps
    int32_t* tile_n0;                // vehicles of each tile, read at even steps
    int32_t* tile_n1;
    VehRec* inbox;                   // [NL]
    int32_t* inbox_flag;             // [NL]
    // per-slot scratch of the update kernel (indexed like the read slab)
    uint32_t* sh_gmask;
    int32_t* sh_jq;                  // packed junction lanes of the route
    float* sh_aown;
    int32_t* sh_merge;               // local index of the merge target lane, -1 none
    float* sh_lrear;                 // own leader's rear (lane coordinate), +inf none
    float* sh_lv;
    float* sh_nx;
    float* sh_nv;
    int32_t* sh_kind;                // 0 stay, 1 change, 2 enter junction lane, 3 leave tile, 4 finished
    int32_t* sh_nlane;               // local index of the new lane
    int32_t* sh_pref;                // stayer prefix count within the tile enumeration
    // work lists of the step's update, filled by the prepare kernel: tiles
    // with vehicles that fit a group of the schedule, wide tiles, huge tiles
    int32_t* list_small;             // [R]
    int32_t* list_big;               // [R] tiles of at most kWideLanes lanes and kWideCap vehicles
    int32_t* list_huge;              // [R] the rest
    int32_t* list_tiny;              // [R] tiles for the narrowest groups (two-width schedules)
    int32_t* list_med;               // [R] tiles of at most kWideLanes lanes and kMedCap vehicles (fused schedule)
    int32_t* list_large;             // [R] tiles above the wide list with at most kLargeLanes lanes and kLargeCap vehicles (fused schedule)
    int32_t* list_cnt;               // [2][kNumLists kCntStride] by step parity (one 128-byte line each)
    // schedule (host side; passed to the kernels as arguments)
    int32_t sched, GA, GB, GC, GT, GM, GL;   // GT, GM, GL: workgroups of the tiny, medium and large passes
    int32_t mp_any;                  // host side: some junction may use MAX_PRESSURE (k_signals is launched)
    // metrics
    float* road_speed;               // [R] mean speed of the last step, -1 empty
    int32_t* lane_wait;              // [NL] (internal ids)
    WGPartial* part;                 // [G] (G >= GA + GB for every schedule)
    // step protocol: the prepare kernel of step t publishes t in *ustep (read
    // by that step's update kernels, whose workgroups then advance *gstep to
    // t + 1) and sums the partials of step t - 1 in slices (part2) when that
    // step's parity p has fold_flag[2 p] set (fold_flag[2 p + 1]: the number
    // of partials); fold_flag[4] marks slice sums that the update still has
    // to combine into the metrics
    long long* ustep;
    int32_t* fold_flag;              // [6]
    WGPartial* part2;                // [kFoldWGs]
    DevMetrics* met;                 // [n_inst]
    KParams P;
};

// Side streams on which the update passes of a step run concurrently: the
// passes touch disjoint tiles (the feeder gates they raise in other tiles are
// atomic min/max), so they need no order among themselves, only after the
// prepare kernel and before the next step.  n = 0 keeps every pass on the
// step's stream.
struct PassStreams {
    int n = 0;
    hipStream_t aux[3] = {nullptr, nullptr, nullptr};
    hipEvent_t fork = nullptr;
    hipEvent_t join[3] = {nullptr, nullptr, nullptr};
};

}  // namespace tsim
