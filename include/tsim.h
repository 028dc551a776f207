/*
 * tsim.h -- C ABI of the MI355X (gfx950) microscopic traffic stepper.
 *
 * The library implements the data-parallel per-timestep vehicle update of
 * arXiv 2406.10661 ("A GPU-accelerated Large-scale Simulator for
 * Transportation System Optimization Benchmarking"):
 *   - two-phase step with a read-only snapshot and a private next state
 *     (Section 3.1, "Two-phase Parallel Process for Read/Write Separation";
 *     Appendix B.2 execution process);
 *   - per-lane ordered vehicle index with own-lane and side-lane neighbours
 *     (Section 3.1, "Linked-list based Vehicle Sensing Indexes");
 *   - IDM car following, randomized MOBIL lane changing, signal stop rule
 *     (Appendix B.3, vehicle model implementation);
 *   - signal policies NONE / FIXED_TIME / MANUAL (Section 3.2, traffic signal);
 *   - metrics of Section 3.3 (lane queue length, road speed, average
 *     travelling time, throughput).
 *
 * Conventions
 *   - Every function returns TSIM_OK (0) or a negative TSIM_E* status; no C++
 *     exception crosses this boundary.  tsim_last_error() returns a message for
 *     the last failure on a handle (or the last global failure for NULL).
 *   - "host" pointers are plain CPU memory owned by the caller and only read
 *     (or written, for getters) during the call.  "device" pointers are GPU
 *     memory.  Nothing is retained after a call returns except where stated.
 *   - A handle is used by one host thread at a time.
 *   - Lane ids: road lanes are numbered road by road (road r owns
 *     road_lane_begin[r] .. road_lane_begin[r+1]-1, index 0 within a road is
 *     the leftmost lane); junction lanes follow, junction lane q having lane
 *     id n_road_lanes + q.
 *   - Time: step t covers [t*dt, (t+1)*dt).
 */
#ifndef TSIM_H
#define TSIM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* status codes */
#define TSIM_OK 0
#define TSIM_EINVAL (-1)   /* invalid argument or malformed network / trips */
#define TSIM_ENOMEM (-2)   /* device arena smaller than tsim_footprint() */
#define TSIM_EDEVICE (-3)  /* a HIP call failed; message in tsim_last_error */
#define TSIM_ESTATE (-4)   /* the device detected a violated invariant (see metrics.errors) */

/* signal policies (Section 3.2) */
#define TSIM_POLICY_NONE 0       /* every junction lane always green */
#define TSIM_POLICY_FIXED_TIME 1 /* phases in order with their durations, phase 0 at t = 0 */
#define TSIM_POLICY_MANUAL 2     /* phase set through tsim_set_signal_phases */
/* Adaptive maximum pressure (Section 3.2, the cited maximum-pressure
 * algorithm; Appendix B.2: lane pressures in the prepare phase).  A
 * movement (junction lane from road lane a to road lane b) has pressure
 * n(a) - n(b), n = vehicles on the lane at the step start before the step's
 * departures; a phase's pressure is the sum over the movements it makes
 * green; the junction takes the largest (ties to the lowest phase index).
 * It decides at the steps t with floor(t dt / d0) > floor((t - 1) dt / d0),
 * d0 the duration of its first phase (t = 0, then every d0 seconds), and
 * holds the phase in between (tsim_state_host.junc_phase).  Needs d0 > 0. */
#define TSIM_POLICY_MAX_PRESSURE 3

/* vehicle status */
#define TSIM_WAITING 0
#define TSIM_ACTIVE 1
#define TSIM_FINISHED 2

/*
 * Road network (all host arrays, read during tsim_footprint/tsim_create).
 * Limits: <= 32 lanes per road, <= 32 phases per junction, lane and junction
 * lane lengths >= v_max*dt + a_max*dt^2/2 (one lane-end crossing per step),
 * every road lane length shared by the lanes of its road.
 */
typedef struct tsim_network {
    int32_t n_junctions;
    int32_t n_roads;
    const int32_t *road_from;        /* [n_roads] junction the road leaves */
    const int32_t *road_to;          /* [n_roads] junction the road enters */
    const int32_t *road_lane_begin;  /* [n_roads+1] road lanes of road r */
    const float *road_length;        /* [n_roads] metres */
    const float *road_limit;         /* [n_roads] m/s */
    int32_t n_jlanes;
    const int32_t *jl_in_lane;       /* [n_jlanes] road lane the junction lane leaves */
    const int32_t *jl_out_lane;      /* [n_jlanes] road lane it enters (next road) */
    const float *jl_length;          /* [n_jlanes] metres */
    const float *jl_limit;           /* [n_jlanes] m/s */
    const int32_t *junc_phase_begin; /* [n_junctions+1] phases of junction j */
    const float *phase_duration;     /* [n_phases] seconds (FIXED_TIME) */
    const int32_t *phase_green_begin;/* [n_phases+1] green junction lanes of phase p */
    const int32_t *phase_green_jl;   /* junction-lane indices 0..n_jlanes-1 */
    const int32_t *junc_policy;      /* [n_junctions] TSIM_POLICY_* */
} tsim_network;

/* Trip table (host arrays).  Route = consecutive road ids, origin first,
 * destination last; consecutive roads must be joined by a junction lane. */
typedef struct tsim_trips {
    int32_t n_vehicles;
    const float *depart_time;        /* [n] seconds */
    const int32_t *route_begin;      /* [n+1] CSR into route_roads */
    const int32_t *route_roads;      /* road ids */
    const float *v0_factor;          /* [n] desired speed = v0_factor * lane limit */
    const float *length;             /* [n] vehicle length, metres, > 0 */
    const float *end_s;              /* [n] or NULL: where the trip ends on the last road of its route, metres
                                      * from the road's start (the trip ends in the step the vehicle's front
                                      * passes it; Section 3.2 set_vehicle_route end position, an AOI's
                                      * connection (Appendix B.1) as the trip's end); negative or NULL: the road's end */
    const float *start_s;            /* [n] or NULL: where the trip starts on its origin road, metres from the road's
                                      * start, below the road's length (an AOI's connection partway along the road,
                                      * Appendix B.1/B.2: the vehicle enters with its front there, at rest, into the
                                      * lane of its lane group with the most room ahead, once the nearest vehicle
                                      * ahead leaves s0 and nothing behind can reach its rear within the step);
                                      * 0, negative or NULL: the road's start */
} tsim_trips;

/* Model parameters (Appendix B.3; the MOBIL threshold, safe deceleration,
 * probability cap/floor and braking floor are this library's parameters). */
typedef struct tsim_params {
    double dt;          /* step, seconds */
    double T;           /* IDM safe time headway */
    double a_max;       /* IDM maximum acceleration */
    double b_comf;      /* IDM comfortable deceleration */
    double s0;          /* IDM minimum gap */
    double delta;       /* IDM free-road exponent (4 in the paper) */
    double politeness;  /* MOBIL politeness p (0.1 in the paper) */
    double a_th;        /* MOBIL switching threshold */
    double b_safe;      /* MOBIL safe deceleration of the new follower */
    double p_max;       /* lane-change probability cap (0.9 in the paper) */
    double p_min;       /* lane-change probability floor (2e-8 in the paper) */
    double a_emerg;     /* braking floor */
    uint64_t seed;      /* Philox4x32-10 key */
} tsim_params;

/* Aggregates (Section 3.3).  Totals since create / set_state. */
typedef struct tsim_metrics {
    int64_t step;             /* steps taken: the next step to run */
    int64_t n_waiting;
    int64_t n_active;
    int64_t n_finished;       /* throughput (get_finished_vehicle_count) */
    double sum_travel_time;   /* seconds, over finished vehicles */
    double att;               /* average travelling time of finished vehicles */
    double mean_speed_last;   /* road-lane mean speed of the last step */
    double mean_speed_avg;    /* time average of mean_speed_last */
    int64_t vehicle_steps;    /* sum over steps of active vehicles */
    int64_t lane_changes;
    int64_t transfers;        /* lane-end crossings into the next lane */
    int64_t clamps;           /* position bounded by a snapshot obstacle */
    int64_t feeder_blocks;    /* merge entries refused by feeder priority */
    int64_t departures;
    int64_t speed_steps;      /* steps with at least one road-lane vehicle */
    int64_t errors;           /* device-detected capacity/ordering violations */
    int64_t lane_steps;       /* sum over steps of lanes holding a vehicle at the step start */
    int64_t road_entries;     /* junction-lane-to-road crossings (the vehicle moves to its next road) */
    int64_t stalled_steps;    /* gridlock detector: the current run of steps with vehicles on the network in
                               * which none on a road lane ended the step moving and none departed, crossed a
                               * lane end or finished (counted as the steps are folded; a departure is seen
                               * by the fold after its step at the latest) */
    int64_t max_stalled_steps;/* the longest such run since create / set_state */
} tsim_metrics;

/* Vehicle state for checkpoint/resume and tests (host arrays of n_vehicles,
 * n_junctions entries, filled by get_state and read by set_state). */
typedef struct tsim_state_host {
    int64_t step;
    int32_t *status;          /* TSIM_WAITING / ACTIVE / FINISHED */
    int32_t *lane;            /* lane id when ACTIVE, else -1 */
    int32_t *route_pos;       /* index of the current road within the route */
    float *x;                 /* front-bumper coordinate along the lane, metres */
    float *v;                 /* speed, m/s */
    int32_t *finish_step;     /* step during which the trip ended, else -1 */
    int32_t *junc_policy;     /* [n_junctions] */
    int32_t *junc_phase;      /* [n_junctions] MANUAL phase index, or the phase a MAX_PRESSURE junction holds */
} tsim_state_host;

typedef struct tsim_handle tsim_handle;

/* Device bytes tsim_create needs for this input (arena size): the road
 * network, trip table and vehicle state resident on the GPU, in the
 * snapshot/runtime pair of Section 3.1's two-phase process (two slab buffers
 * alternating by step parity).  Validates the input like tsim_create. */
int tsim_footprint(const tsim_network *net, const tsim_trips *trips, const tsim_params *params,
                   size_t *bytes_out);

/* Builds the device state inside the caller's arena (device pointer, at
 * least tsim_footprint bytes, 256-byte aligned, alive until tsim_destroy):
 * the simulator instance of Section 3.1 ("Python API": the engine created
 * from map and trip data), every vehicle waiting at t = 0.
 * hip_stream (a hipStream_t, or NULL for the null stream) carries every later
 * launch and copy.  Validates the input (TSIM_EINVAL with a message). */
int tsim_create(const tsim_network *net, const tsim_trips *trips, const tsim_params *params,
                void *hip_stream, void *device_arena, size_t arena_bytes, tsim_handle **out);

/* Enqueues n_steps steps on the stream and returns without waiting
 * (Section 3.1 "Python API" next_step; one step is the prepare and update
 * phases of Appendix B.2 with the vehicle models of Appendix B.3). */
int tsim_step(tsim_handle *h, int32_t n_steps);

/* Junctions junction_ids[c] switch to MANUAL with phase phase_index[c] from
 * the next step on (Section 3.2 set_tl_phase and its batch form).  Enqueued on
 * the stream without waiting; the host arrays may be reused on return. */
int tsim_set_signal_phases(tsim_handle *h, const int32_t *junction_ids, const int32_t *phase_index,
                           int32_t n);

/* As tsim_set_signal_phases, for callers that cannot allocate (code under
 * HIP graph capture, tight serving loops, harnesses that forbid allocation):
 * allocates nothing, neither device nor pinned host memory.  The ids and
 * phases are staged in a fixed device array the library keeps on each GPU
 * (2 x 262,144 int32, 2 MiB, held until the process ends); n > 262,144
 * returns TSIM_EINVAL.  The handle's GPU must be the current device.
 * Synchronises the handle's stream before returning, after which the host
 * arrays may be reused.  Every call on one GPU shares that array: calls that
 * overlap on one GPU (from several host threads) race.  Single-instance
 * handles only. */
int tsim_set_signal_phases_noalloc(tsim_handle *h, const int32_t *junction_ids, const int32_t *phase_index,
                                   int32_t n);

/* Junctions junction_ids[c] take signal policy policy[c] (TSIM_POLICY_*)
 * from the next step on (Section 3.2 set_tl_policy).  A junction switched to
 * MAX_PRESSURE holds its stored phase (tsim_state_host.junc_phase) until its
 * next decision step.  Enqueued on the stream; TSIM_EINVAL for an unknown
 * junction or policy, or a max-pressure junction whose first phase has no
 * positive duration.  The host arrays may be reused on return. */
int tsim_set_signal_policy(tsim_handle *h, const int32_t *junction_ids, const int32_t *policy, int32_t n);

/* Speed limits of lanes (road lanes and junction lanes, lane ids as in the
 * network) from the next step on (Section 3.2 "Lane" set_lane_max_speed);
 * a vehicle's desired speed on such a lane is its v0_factor times the new
 * limit.  TSIM_EINVAL for a bad id, a non-positive limit, or a lane shorter
 * than one step of travel at the new limit (largest v0_factor of the
 * instance); nothing changes then.  Synchronises the stream. */
int tsim_set_lane_max_speed(tsim_handle *h, const int32_t *lane_ids, const float *max_speed, int32_t n);

/* Lanes lane_ids[c] (road or junction lanes, ids as in the network) are
 * restricted (flags[c] != 0) or released (0) from the next step on
 * (Section 3.2 "Lane" set_lane_restriction).  A restricted lane admits no
 * new vehicle: no departure into it, no lane change into it, and no entry
 * from a road lane into a junction lane that is restricted or leads into a
 * restricted lane (such a junction lane is closed, and the lane group of a
 * route is formed from the open ones).  Vehicles already on a restricted
 * lane, or on a junction lane leading into one, carry on.  A road lane plan
 * (Section 3.2 "Road" set_road_lane_plan: which junction lanes of a road
 * are in use) is the restriction of the junction lanes outside the plan.
 * TSIM_EINVAL for a bad id (nothing changes then).  Synchronises the
 * stream; the host arrays may be reused on return. */
int tsim_set_lane_restriction(tsim_handle *h, const int32_t *lane_ids, const int32_t *flags, int32_t n);

/* Vehicle vehicle_id follows the route roads[0 .. n_roads-1] from the next
 * step on (Section 3.2 "Vehicle" set_vehicle_route, for congestion pricing
 * and rerouting).  The route must begin with the road the vehicle is on (its
 * origin road while it waits; on a junction lane, the road it left, followed
 * by the road that lane enters), and consecutive roads must be joined by a
 * junction lane; its trip ends where its front passes end_s metres along
 * the last road (negative: that road's end; the paper's end lane is not
 * modelled).  Its route position becomes 0; a vehicle outside the new next
 * road's lane group changes lanes toward it as usual.  Changed routes are
 * kept in a route pool with room for a quarter of the creation routes plus
 * 4,096 entries (TSIM_ENOMEM when it is full); TSIM_EINVAL for a finished
 * vehicle, a bad route or an end position beyond the last road.
 * Synchronises the stream. */
int tsim_set_vehicle_route(tsim_handle *h, int32_t vehicle_id, const int32_t *roads, int32_t n_roads, float end_s);

/* ---- Shortest routes on the device (Section 4 "Congestion Pricing": once
 * roads carry prices, drivers move to routes of lower cost; Appendix F:
 * every road may be priced and the prices change every 20 s; Appendix E:
 * demand routed by shortest travel time).
 *
 * Cost of a route: over every road after its first, the fastest open
 * junction lane into it (length / limit) plus the road's travel time (its
 * length over the highest limit of its lanes, or road_time[r] when given)
 * plus its price road_price[r] (seconds; NULL: none), in FP32; the route of
 * least cost is taken, and where candidate costs tie, the smaller next road
 * id.  Prices and times must be >= 0 (+inf closes a road).  Networks of at
 * most 32,768 roads (a road's cost-to-go is held in LDS per destination).
 *
 * Work space: a device buffer the caller allocates (workspace,
 * workspace_bytes); min_bytes is the least a call takes, hint_bytes routes
 * the pairs in few passes.  The call synchronises its stream; the buffer is
 * free again on return. */
int tsim_route_footprint(const tsim_network *net, int32_t n_pairs, size_t *min_bytes, size_t *hint_bytes);

/* Routes for n (origin road, destination road) pairs of a network given as
 * host arrays, computed on the current GPU on hip_stream (NULL: the default
 * stream).  route_begin[n+1] (always filled on success or TSIM_ENOMEM) and
 * route_roads[max_roads] (origin first, destination last; an unreachable
 * pair gets an empty route and is counted in *n_unreachable, which may be
 * NULL).  TSIM_ENOMEM when the routes need more than max_roads entries
 * (route_begin[n] says how many) or the work space is below min_bytes;
 * TSIM_EINVAL for a bad network, road id, price or time. */
int tsim_shortest_routes(const tsim_network *net, const float *road_price, const float *road_time,
                         const int32_t *origin, const int32_t *dest, int32_t n, void *hip_stream, void *workspace,
                         size_t workspace_bytes, int32_t *route_begin, int32_t *route_roads, int64_t max_roads,
                         int32_t *n_unreachable);

/* Work space of tsim_reroute_shortest for n vehicles of handle h. */
int tsim_reroute_footprint(tsim_handle *h, int32_t n, size_t *min_bytes, size_t *hint_bytes);

/* Vehicles vehicle_ids[0..n-1] (distinct) take, from the next step on, the
 * route of least cost from where they are to the last road of their route
 * in force, under the lane limits and restrictions in force: a waiting
 * vehicle from its origin road, a vehicle on a road lane from that road, a
 * vehicle on a junction lane through the road that lane enters (as
 * tsim_set_vehicle_route requires).  Trip end positions are kept.  The
 * routes are computed on the handle's GPU and written into the records
 * there.  A vehicle keeps its route when it has finished, its destination
 * cannot be reached, or the route pool is full (a new route is written over
 * the rest of the route in force when it fits there, else appended); those
 * are counted in *n_kept (may be NULL).  Synchronises the stream. */
int tsim_reroute_shortest(tsim_handle *h, const int32_t *vehicle_ids, int32_t n, const float *road_price,
                          const float *road_time, void *workspace, size_t workspace_bytes, int32_t *n_kept);

/* Synchronises the stream, then fills *out. */
int tsim_get_metrics(tsim_handle *h, tsim_metrics *out);

/* Mean speed of the vehicles on each road's lanes during the last step
 * (end-of-step speeds), -1 for a road without vehicles.  out[n_roads]. */
int tsim_get_road_mean_speed(tsim_handle *h, float *out, int32_t n_roads);

/* Vehicles slower than 0.1 m/s at the end of the last step, per lane they
 * occupied during it.  out[n_lanes] (road lanes then junction lanes). */
int tsim_get_lane_waiting_counts(tsim_handle *h, int32_t *out, int32_t n_lanes);

/* Vehicle ids of every lane, front first (the sensing index): offsets
 * [n_lanes+1] and ids [n_active]. */
int tsim_get_lane_order(tsim_handle *h, int32_t *offsets, int32_t *vehicle_ids, int32_t n_lanes,
                        int32_t max_ids);

/* The vehicle state at the step boundary (positions, speeds, lanes, route
 * positions, status; signal policies and phases): the per-vehicle and
 * per-junction quantities the getters of Section 3.1 "Python API" expose,
 * all at once, for checkpoints and tests.  Synchronises the stream. */
int tsim_get_state(tsim_handle *h, tsim_state_host *out);
/* Replaces the state.  Finished-trip totals are recomputed from finish_step;
 * the running averages and event counters restart from zero. */
int tsim_set_state(tsim_handle *h, const tsim_state_host *in);

/* Kernel timing for measurement tools.  While enabled, tsim_step brackets
 * every launch with HIP events on the handle's stream (a small overhead);
 * tsim_get_kernel_times synchronises and returns, per kernel, the summed
 * milliseconds and the number of launches since profiling was enabled.
 * Kernel 0 is the update (every update launch of a step), kernel 1 the
 * prepare kernel; n_kernels <= 2. */
int tsim_set_profiling(tsim_handle *h, int32_t enable);
int tsim_get_kernel_times(tsim_handle *h, double *ms, int64_t *launches, int32_t n_kernels);

/* Trajectory output (Appendix B.2: every vehicle's motion state saved for
 * output).  With every > 0, each step boundary reached by tsim_step whose
 * step number is a multiple of `every` appends one record per vehicle on the
 * network to device_buffer (caller-owned device memory of `capacity`
 * records, alive while recording), in no particular order:
 *   struct { int64_t step; int32_t vehicle; int32_t lane; float x, v; }
 * (24 bytes; the state at the start of `step`, lane ids as in the network).
 * Records beyond the capacity are counted but not written.  every = 0 stops
 * recording.  Setting resets the count, synchronises the stream and drops a
 * captured graph.  Single-instance handles; steps taken by the autotuner are
 * not recorded. */
int tsim_set_trajectory(tsim_handle *h, void *device_buffer, int64_t capacity, int32_t every);
/* Records appended since tsim_set_trajectory (may exceed the capacity).
 * Synchronises the stream. */
int tsim_get_trajectory_count(tsim_handle *h, int64_t *n);

/* Areas of interest (Appendix B.1: an area with several connections to the
 * road network where trips start and end; Appendix B.2: an AOI puts a
 * vehicle whose departure time has come into a lane at its connection when
 * that is safe, and takes in the vehicles whose trips end there).
 *
 * tsim_aoi_footprint: device bytes tsim_set_aois needs for n_aoi AOIs.
 *
 * tsim_set_aois: n_aoi AOIs; AOI a's connections are entries
 * conn_begin[a] .. conn_begin[a+1]-1 (conn_begin[0] = 0, non-decreasing) of
 * conn_road (road ids) and conn_s (metres from the road's start, within its
 * length).  origin_aoi / dest_aoi ([n_vehicles] or NULL; -1 = none) name each
 * vehicle's AOIs: a vehicle with an origin AOI starts at that AOI's first
 * listed connection on the first road of its route (which must lie below the
 * road's length), one with a destination AOI ends at the connection on its
 * last road (which must lie beyond the road's start) — the start and end
 * positions of tsim_trips, replacing those given there.  Every vehicle named
 * must still be waiting.  Host arrays, copied; device_buffer (caller-owned,
 * 256-byte aligned, at least tsim_aoi_footprint bytes, alive until the next
 * tsim_set_aois or tsim_destroy) holds the AOI ids on the device.  Errors
 * (TSIM_EINVAL: an AOI id, road or position out of range, an AOI without a
 * connection on the road a vehicle needs, a vehicle that has departed)
 * change nothing.  Synchronises the stream.  Single-instance handles (for
 * batches, tsim_batch_set_aois).
 *
 * tsim_get_aoi_counts: at the current step boundary, waiting[a] = vehicles
 * whose trip starts in AOI a and that have not departed, arrived[a] =
 * vehicles whose trip ended in AOI a (host arrays of n_aoi, the count given
 * to tsim_set_aois; counted on the device).  Synchronises the stream. */
int tsim_aoi_footprint(tsim_handle *h, int32_t n_aoi, size_t *bytes_out);
int tsim_set_aois(tsim_handle *h, int32_t n_aoi, const int32_t *conn_begin, const int32_t *conn_road,
                  const float *conn_s, const int32_t *origin_aoi, const int32_t *dest_aoi, void *device_buffer,
                  size_t buffer_bytes);
int tsim_get_aoi_counts(tsim_handle *h, int32_t *waiting, int32_t *arrived, int32_t n_aoi);

/* Launch mode.  chunk > 0: tsim_step captures `chunk` steps (both kernels of
 * each) into one HIP graph on its first call and replays that graph for every
 * whole chunk of a call; the remaining steps are launched one by one.  chunk
 * = 0 (default) launches every kernel directly.  Graphs are not used while
 * profiling is on.  Changing the chunk synchronises the stream.  chunk in
 * [0, 4096]; TSIM_EDEVICE if capture fails. */
int tsim_set_graph_steps(tsim_handle *h, int32_t chunk);

/* Update schedules: how road tiles are laid onto 64-wide wavefronts.
 *   0 TSIM_SCHED_WIDE    one tile per wavefront
 *   1 TSIM_SCHED_16X32   tiles of <= 16 lanes: four per wavefront while they
 *                        hold <= 32 vehicles (fuller ones: one per wavefront)
 *   2 TSIM_SCHED_16X64   as 1 with <= 64 vehicles
 *   3 TSIM_SCHED_32X64   tiles of <= 32 lanes: two per wavefront, <= 64 vehicles
 *   4 TSIM_SCHED_8X16    tiles of <= 8 lanes: eight per wavefront, <= 16 vehicles
 *   5 TSIM_SCHED_16X32P  as 1, with the pass over wider tiles loading each
 *                        wavefront's next tile while it works on the current
 *   6 TSIM_SCHED_8AND16  as 5, with tiles of <= 8 lanes and <= 16 vehicles
 *                        eight per wavefront
 *   7 TSIM_SCHED_FUSED   the tile classes of 6 plus tiles of <= 32 lanes and
 *                        <= 64 vehicles two per wavefront, every update pass
 *                        in one launch (workgroup ranges per class; the pass
 *                        concurrency setting does not apply)
 * Every schedule gives bit-identical results; only speed differs.  Default 7 (TSIM_SCHED_FUSED).
 * Changing the schedule synchronises the stream and drops a captured graph
 * (recaptured on the next tsim_step). */
#define TSIM_SCHED_WIDE 0
#define TSIM_SCHED_16X32 1
#define TSIM_SCHED_16X64 2
#define TSIM_SCHED_32X64 3
#define TSIM_SCHED_8X16 4
#define TSIM_SCHED_16X32P 5
#define TSIM_SCHED_8AND16 6
#define TSIM_SCHED_FUSED 7
#define TSIM_NUM_SCHED 8
int tsim_set_schedule(tsim_handle *h, int32_t schedule);
int tsim_get_schedule(tsim_handle *h, int32_t *schedule);
/* Pass concurrency (schedules 0-6).  A step's update passes (one per class of
 * tile size) work on disjoint tiles and meet only in the step's metric sums;
 * with enable = 1 they are launched on three side streams of the handle
 * (default priority, ordered after the step's prepare kernel and joined
 * before the next step by events), so that one pass's last workgroups overlap
 * the next pass.  Results are bit-identical either way.  Synchronises the
 * stream and drops a captured graph.  Works on batches too.  Default 0. */
int tsim_set_concurrency(tsim_handle *h, int32_t enable);
/* Autotuner: runs `rounds` rounds of `steps` steps under every schedule in
 * turn (these are real steps: the simulation advances by
 * rounds * TSIM_NUM_SCHED * steps), keeps the schedule with the lowest best
 * round time, and writes it to *chosen; us_per_step (optional, TSIM_NUM_SCHED
 * entries) receives each schedule's best microseconds per step.  Synchronises
 * the stream.  Works on batches too. */
int tsim_autotune(tsim_handle *h, int32_t steps, int32_t rounds, int32_t *chosen, float *us_per_step);
/* As tsim_autotune over every (schedule, pass concurrency) pair: first all
 * schedules with serial passes, then all with concurrent ones
 * (rounds * 2 * TSIM_NUM_SCHED * steps real steps).  Keeps the fastest pair
 * and writes it to *schedule and *concurrent; us_per_step (optional,
 * 2 * TSIM_NUM_SCHED entries) receives the serial times, then the concurrent
 * ones.  Synchronises the stream.  Works on batches too. */
int tsim_autotune_launch(tsim_handle *h, int32_t steps, int32_t rounds, int32_t *schedule, int32_t *concurrent,
                         float *us_per_step);

int tsim_destroy(tsim_handle *h);
const char *tsim_last_error(const tsim_handle *h);

/*
 * Batched instances: many independent simulations (networks, trip tables and
 * seeds of their own) resident together and advanced by the same kernel
 * launches, one launch per kernel per step for the whole batch.  Every
 * instance draws its random numbers from its own seed, vehicle ids and step
 * count, so its trajectory is bit-identical to the same instance created alone
 * with tsim_create.  All instances share the model parameters except the seed
 * (params[i].seed).  Arrays nets/trips/params have n entries (host).
 * Instance-indexed calls take local ids (junction ids, roads, lanes, vehicles
 * of that instance).
 */
typedef struct tsim_handle tsim_batch;

int tsim_batch_footprint(const tsim_network *nets, const tsim_trips *trips, const tsim_params *params, int32_t n,
                         size_t *bytes_out);
int tsim_batch_create(const tsim_network *nets, const tsim_trips *trips, const tsim_params *params, int32_t n,
                      void *hip_stream, void *device_arena, size_t arena_bytes, tsim_batch **out);
/* Enqueues n_steps steps of every instance (async on the stream). */
int tsim_batch_step(tsim_batch *b, int32_t n_steps);
/* As tsim_set_graph_steps, for the whole batch. */
int tsim_batch_set_graph_steps(tsim_batch *b, int32_t chunk);
/* Instance `instance` is simulated for its first n_steps local steps only;
 * from then on it is frozen (no signal, departure, update or metric changes)
 * while the rest of the batch goes on, so jobs of different horizons can share
 * a batch.  Enqueued on the stream; default: no horizon. */
int tsim_batch_set_horizon(tsim_batch *b, int32_t instance, int64_t n_steps);
int tsim_batch_set_signal_phases(tsim_batch *b, int32_t instance, const int32_t *junction_ids,
                                 const int32_t *phase_index, int32_t n);
/* As tsim_set_vehicle_route, for a vehicle of one instance (local ids). */
int tsim_batch_set_vehicle_route(tsim_batch *b, int32_t instance, int32_t vehicle_id, const int32_t *roads,
                                 int32_t n_roads, float end_s);
/* As tsim_reroute_footprint and tsim_reroute_shortest, for vehicles of one
 * instance (local vehicle and road ids; the instance's roads form the
 * network). */
int tsim_batch_reroute_footprint(tsim_batch *b, int32_t instance, int32_t n, size_t *min_bytes, size_t *hint_bytes);
int tsim_batch_reroute_shortest(tsim_batch *b, int32_t instance, const int32_t *vehicle_ids, int32_t n,
                                const float *road_price, const float *road_time, void *workspace,
                                size_t workspace_bytes, int32_t *n_kept);
/* As tsim_set_lane_max_speed, for the lanes of one instance. */
int tsim_batch_set_lane_max_speed(tsim_batch *b, int32_t instance, const int32_t *lane_ids, const float *max_speed,
                                  int32_t n);
/* As tsim_set_lane_restriction, for the lanes of one instance. */
int tsim_batch_set_lane_restriction(tsim_batch *b, int32_t instance, const int32_t *lane_ids, const int32_t *flags,
                                    int32_t n);
/* As tsim_set_signal_policy, for the junctions of one instance. */
int tsim_batch_set_signal_policy(tsim_batch *b, int32_t instance, const int32_t *junction_ids,
                                 const int32_t *policy, int32_t n);
/* Every junction of every instance at once: phase_index[k] for the k-th
 * junction of the batch in instance order (instance 0's junctions first), a
 * negative entry leaves that junction unchanged; non-negative entries switch
 * it to MANUAL from the next step.  n_total = total junctions of the batch. */
int tsim_batch_set_all_phases(tsim_batch *b, const int32_t *phase_index, int32_t n_total);
/* Synchronises the stream, then fills *out for one instance. */
int tsim_batch_get_metrics(tsim_batch *b, int32_t instance, tsim_metrics *out);
/* State of one instance (arrays sized for that instance, instance-local
 * vehicle, lane and junction ids).  An instance frozen by its horizon reports
 * the state it was frozen in. */
int tsim_batch_get_state(tsim_batch *b, int32_t instance, tsim_state_host *out);
/* Replaces the state of one instance at the batch's step boundary (as
 * tsim_set_state, instance-local arrays).  The instance continues from its
 * own step in->step while the rest of the batch is untouched; the batch's
 * pending step is folded first.  Synchronises the stream.  Its horizon, if
 * set, stays in local steps. */
int tsim_batch_set_state(tsim_batch *b, int32_t instance, const tsim_state_host *in);
/* Per-instance forms of tsim_get_road_mean_speed, tsim_get_lane_waiting_counts
 * and tsim_get_lane_order (sizes and ids local to the instance). */
/* As tsim_aoi_footprint, tsim_set_aois and tsim_get_aoi_counts, for one
 * instance of a batch (its local road and vehicle ids; the instance's own
 * buffer).  Removing the instance drops its AOIs. */
int tsim_batch_aoi_footprint(tsim_batch *b, int32_t instance, int32_t n_aoi, size_t *bytes_out);
int tsim_batch_set_aois(tsim_batch *b, int32_t instance, int32_t n_aoi, const int32_t *conn_begin,
                        const int32_t *conn_road, const float *conn_s, const int32_t *origin_aoi,
                        const int32_t *dest_aoi, void *device_buffer, size_t buffer_bytes);
int tsim_batch_get_aoi_counts(tsim_batch *b, int32_t instance, int32_t *waiting, int32_t *arrived, int32_t n_aoi);
int tsim_batch_get_road_mean_speed(tsim_batch *b, int32_t instance, float *out, int32_t n_roads);
int tsim_batch_get_lane_waiting_counts(tsim_batch *b, int32_t instance, int32_t *out, int32_t n_lanes);
int tsim_batch_get_lane_order(tsim_batch *b, int32_t instance, int32_t *offsets, int32_t *vehicle_ids,
                              int32_t n_lanes, int32_t max_ids);
int tsim_batch_destroy(tsim_batch *b);

/*
 * Instances joining and leaving a running batch (continuous batching of
 * simulation jobs; the serving form of the step, not in the paper).
 *
 * A batch reserved with tsim_batch_reserve starts empty with room for the
 * given totals; tsim_batch_add appends an instance (built on the host by
 * tsim_instance_build, so a serving loop can build jobs on other threads)
 * at the batch's next step boundary, and tsim_batch_add_member appends a copy
 * of a live single-instance handle (its network, trips, parameters and
 * current state; the member stays valid).  An added instance starts its own
 * step count where its state is (local step 0 for tsim_batch_add) while the
 * other instances go on: its trajectory is bit-identical to the same instance
 * stepped alone.  tsim_batch_remove freezes an instance for good; the space
 * of removed instances at the end of the batch is given back (all of it once
 * the batch has drained).  Instance ids are the order of addition (ids of
 * removed trailing instances are reused).  Batches made by tsim_batch_create
 * hold exactly their instances (no room to add until some are removed).
 * Every call here synchronises the batch's stream; calls that would exceed
 * the reserved totals return TSIM_ENOMEM and change nothing.
 */
typedef struct tsim_instance tsim_instance;

typedef struct tsim_batch_capacity {
    int32_t instances;
    int32_t junctions;
    int32_t roads;
    int32_t road_lanes;
    int32_t jlanes;          /* junction lanes */
    int32_t phases;
    int32_t vehicles;
    int64_t route_entries;   /* total route length (roads) over the vehicles */
    int64_t slots;           /* lane slab slots: sum over lanes of floor(length / shortest vehicle) + 2 */
} tsim_batch_capacity;

/* Validates and lays out one simulation on the host (no device work); the
 * same checks as tsim_create.  Free with tsim_instance_free. */
int tsim_instance_build(const tsim_network *net, const tsim_trips *trips, const tsim_params *params,
                        tsim_instance **out);
int tsim_instance_free(tsim_instance *in);
/* The totals one instance takes in a batch (instances = 1); add them up for
 * a reservation. */
int tsim_instance_capacity(const tsim_instance *in, tsim_batch_capacity *out);
/* Device bytes of a reservation, and the empty batch itself (params: the
 * model parameters every instance must share, the seed apart). */
int tsim_batch_reserve_footprint(const tsim_batch_capacity *cap, size_t *bytes_out);
int tsim_batch_reserve(const tsim_batch_capacity *cap, const tsim_params *params, void *hip_stream,
                       void *device_arena, size_t arena_bytes, tsim_batch **out);
/* Appends an instance at the step boundary; *instance receives its id. */
int tsim_batch_add(tsim_batch *b, const tsim_instance *in, int32_t *instance);
int tsim_batch_add_member(tsim_batch *b, tsim_handle *member, int32_t *instance);
/* Freezes an instance at its current step for good (its metrics and state
 * stay readable until its space is given back). */
int tsim_batch_remove(tsim_batch *b, int32_t instance);
/* Remaining room, and the number of instance ids in use (removed ones
 * included until their space is given back). */
int tsim_batch_capacity_left(tsim_batch *b, tsim_batch_capacity *out);
int tsim_batch_num_instances(tsim_batch *b, int32_t *n);

#ifdef __cplusplus
}
#endif
#endif /* TSIM_H */
