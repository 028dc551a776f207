// Device kernels of the gfx950 microscopic traffic stepper.
//
// One simulation step (Section 3.1 two-phase process, Appendix B.2):
//   k_prepare         one thread per junction: phase of the step (Section 3.2
//                     FIXED_TIME / MANUAL / NONE); one thread per road: append
//                     the junction-to-road entrant held in each road lane's
//                     inbox, release due departures into the origin road's
//                     lanes when safe, clear the feeder gates the step builds,
//                     and put the road's tile on the step's work list of its
//                     size class (or finish it if it has just become empty);
//                     workgroup 0 folds the previous step's metric sums and
//                     publishes the step.
//   k_update_fused    (default) every size class in one launch, workgroup
//                     ranges: huge tiles (a workgroup per tile, up to
//                     kFusedHugeCap vehicles in LDS, more on global scratch), wide
//                     tiles (one per wavefront), medium, small and tiny tiles
//                     (64 / W per wavefront, a group of W lanes per tile,
//                     staged in LDS).  k_update_grouped / k_update_wide / k_update_block
//                     run one class each for the other schedules.
// Per tile: pass 1 own leader (or two-lane lookahead), lane group, stop
// obstacle, own IDM acceleration, merge target; pass 2 randomized MOBIL
// (Appendix B.3), Philox draw, ballistic integration with snapshot bounds,
// lane-end transfer; pass 3 new per-lane order (stayers keep theirs, changers
// and entrants merge by position) written to the other slab buffer with the
// lane summaries and feeder gates other tiles read next step.
// Reads of the step come only from slab buffer t&1 and its lane summaries;
// writes go to buffer (t+1)&1, the inboxes and per-vehicle status, so the update
// is free of read/write races without any lock.
#include "tsim_internal.h"

#include <mutex>

namespace tsim {

#define TS_INF __builtin_huge_valf()

// Every update workgroup is a single wavefront: LDS written by one lane is
// visible to the others once the wave has passed this point in program order
// (LDS requests of a wave complete in order), so no workgroup barrier and no
// wait for outstanding global stores is needed between passes.
__device__ __forceinline__ void wave_sync()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// a tile worked on by GW threads: one wavefront (or a part of one) needs only
// the wavefront fence, a whole workgroup needs its barrier
template <int GW>
__device__ __forceinline__ void tile_sync()
{
    if constexpr (GW > 64) __syncthreads();
    else wave_sync();
}

// A leader at rear bumper a + b in the follower's lane coordinate.  The IDM
// gap is formed as (a - x) + b: for a leader on the follower's own lane a is
// its front and b minus its length, so a - x is exact for nearby vehicles and
// the gap is rounded at its own magnitude, not at that of the positions; for
// a leader on a later lane a is the distance to that lane's start and b its
// rear there.
struct Lead {
    float a, b;
    float v;
    bool ex;
};
__device__ __forceinline__ float lead_rear(const Lead& L) { return L.a + L.b; }
__device__ __forceinline__ float lead_gap(const Lead& L, float x) { return (L.a - x) + L.b; }

// a record's next road, -1 on the last road of its trip (whose next-road
// word holds the trip's end position, end_word)
__device__ __forceinline__ int next_road(const VehRec& r) { return r.rem > 0 ? r.nr : -1; }

__device__ __forceinline__ bool ahead(float xa, int va, float xb, int vb)
{
    return xa > xb || (xa == xb && va < vb);
}

// Philox4x32-10 (Salmon et al., SC'11): word 0 of the block for the counter
// (c0, c1, 0, 0) under the 64-bit key (k0, k1).
__device__ __forceinline__ uint32_t philox_word0(uint32_t k0, uint32_t k1, uint32_t c0, uint32_t c1)
{
    uint32_t c2 = 0u, c3 = 0u;
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        if (r) {
            k0 += 0x9E3779B9u;
            k1 += 0xBB67AE85u;
        }
        const uint32_t lo0 = 0xD2511F53u * c0, hi0 = __umulhi(0xD2511F53u, c0);
        const uint32_t lo1 = 0xCD9E8D57u * c2, hi1 = __umulhi(0xCD9E8D57u, c2);
        const uint32_t n0 = hi1 ^ c1 ^ k0;
        const uint32_t n2 = hi0 ^ c3 ^ k1;
        c0 = n0;
        c1 = lo1;
        c2 = n2;
        c3 = lo0;
    }
    return c0;
}

// IDM (Appendix B.3) floored at -a_emerg; a non-positive gap brakes at the floor.
// divisions by the hardware reciprocal (about 1 ulp): the kernels are
// compared with the FP64 oracle at 1e-5 relative
__device__ __forceinline__ float idm_free_term(float v, float v0, const KParams& P)
{
    const float r = v * __builtin_amdgcn_rcpf(v0);
    const float q = P.delta_is_4 ? (r * r) * (r * r) : powf(r, P.delta);
    return 1.0f - q;
}

__device__ __forceinline__ float idm_follow(float v, float v0, float s, float dv, const KParams& P)
{
    if (!(s > 0.0f)) return -P.a_emerg;
    const float fr = idm_free_term(v, v0, P);
    const float ss = P.s0 + fmaxf(0.0f, v * P.T + v * dv * P.inv_2sqrt_ab);
    const float q = ss * __builtin_amdgcn_rcpf(s);
    return fmaxf(P.a_max * (fr - q * q), -P.a_emerg);
}

__device__ __forceinline__ float idm_freeroad(float v, float v0, const KParams& P)
{
    return fmaxf(P.a_max * idm_free_term(v, v0, P), -P.a_emerg);
}

__device__ __forceinline__ float accel(float v, float v0, float x, Lead ld, bool stop, float len, const KParams& P)
{
    float a = ld.ex ? idm_follow(v, v0, lead_gap(ld, x), v - ld.v, P) : idm_freeroad(v, v0, P);
    if (stop) a = fminf(a, idm_follow(v, v0, len - x, v, P));
    return a;
}

__device__ __forceinline__ bool jl_green(const DevNet& D, int g)
{
    const int cur = D.junc_cur[D.jl_junc[g]];
    return cur < 0 || ((D.jl_green_mask[g] >> cur) & 1u);
}

// junction lane leaving road lane m toward road nr (global tables), or -1
__device__ __forceinline__ int out_toward_range(const DevNet& D, int b, int e, int nr)
{
    for (; e > b && nr >= 0; ++b) {
        const int2 pr = D.out_pair[b];
        if (pr.x == nr) return pr.y;
    }
    return -1;
}

__device__ __forceinline__ int out_toward(const DevNet& D, int m, int nr)
{
    return out_toward_range(D, D.out_begin[m], D.out_begin[m + 1], nr);
}

__device__ __forceinline__ float front_reach(float x, float v, float len, const KParams& P)
{
    return x + v * P.dt + P.reach - len;
}

// writes the per-step part of a lane summary (count, rear, front reach),
// leaving the feeder gates and the static connection range alone
__device__ __forceinline__ void put_dyn(LaneSum& d, const LaneSum& s)
{
    d.cnt = s.cnt;
    d.rear = s.rear;
    d.rear_v = s.rear_v;
    d.front_reach = s.front_reach;
}

// appends val to list for every lane of the wave with pred set, one atomic per
// wavefront (call from converged code)
__device__ __forceinline__ void append_wave(int32_t* list, int32_t* cnt, bool pred, int val)
{
    const unsigned long long m = __ballot(pred);
    if (!m) return;
    const int lane = __lane_id();
    const int leader = __ffsll((long long)m) - 1;
    int base = 0;
    if (lane == leader) base = atomicAdd(cnt, __popcll(m));
    base = __shfl(base, leader);
    if (pred) list[base + __popcll(m & ((1ull << lane) - 1ull))] = val;
}

// ---------------------------------------------------------------------------
// prepare
// ---------------------------------------------------------------------------
// what one prepare thread hands to its workgroup
struct PrepOut {
    int r = -1;          // road
    int list = -1;       // work list of its tile (0 small, 1 wide, 2 huge), -1 none
    int inst = 0;
    int departed = 0;
    int errors = 0;
};

__device__ __forceinline__ void prepare_one(const DevNet& D, long long tg, int i, int small_lanes, int small_cap,
                                            int tiny_lanes, int tiny_cap, PrepOut& out)
{
    const int p = (int)(tg & 1);
    VehRec* slab = p ? D.slab1 : D.slab0;
    LaneSum* sum = p ? D.sum1 : D.sum0;
    int32_t* tile_n = p ? D.tile_n1 : D.tile_n0;
    int32_t* tile_n_w = p ? D.tile_n0 : D.tile_n1;
    LaneSum* wsum = p ? D.sum0 : D.sum1;
    const KParams& P = D.P;

    // threads [0, NJ): junction signals; threads [NJ, NJ + R): roads
    if (i < D.NJ) {
        if (!(tg - D.inst_t0[D.junc_inst[i]] < D.inst_end[D.junc_inst[i]])) return;
        const long long t = tg - D.inst_t0[D.junc_inst[i]];
        const int b = D.junc_phase_begin[i], e = D.junc_phase_begin[i + 1];
        int cur = -1;
        const int pol = D.junc_policy[i];
        if (pol != 0 && e > b) {
            if (pol == 2 || pol == 3) {
                // MANUAL, or the phase a MAX_PRESSURE junction holds (decided
                // by k_signals before this kernel)
                cur = D.junc_manual[i];
            } else {
                const double cyc = D.junc_cycle[i];
                const double tt = fmod((double)t * P.dt_d, cyc);
                double acc = 0.0;
                cur = e - b - 1;
                for (int q = b; q < e; ++q) {
                    acc += (double)D.phase_dur[q];
                    if (tt < acc) {
                        cur = q - b;
                        break;
                    }
                }
            }
        }
        D.junc_cur[i] = cur;
        return;
    }
    if (i >= D.NJ + D.R) return;
    const int r = i - D.NJ;
    // the road's words, its lanes' inbox flags and the first queued departure
    // time are all read before the first store, so that their loads overlap
    const int inst = D.tile_inst[r];
    const int lb = D.tile_lane_begin[r];
    const int nl = D.tile_lane_begin[r + 1] - lb;
    const int nrl = D.tile_n_road[r];
    int head = D.q_head[r];
    const int qe = D.q_begin[r + 1];
    const int n_prev = tile_n[r];
    const int n_w = tile_n_w[r];
    const long long t = tg - D.inst_t0[inst];
    const long long t_end = D.inst_end[inst];
    QRec qr0{};
    if (head < qe) qr0 = D.q_rec[head];
    // inbox flags count the entrants written this step: one is taken, more
    // (two tiles writing one inbox, which the feeder gates rule out) is an
    // error, counted here so that the writers need not wait for an atomic
    uint32_t inb = 0u;
    int extra = 0;
#pragma unroll 4
    for (int li = 0; li < nrl; ++li) {
        const int f = D.inbox_flag[lb + li];
        inb |= (f != 0 ? 1u : 0u) << li;
        extra += f > 1 ? f - 1 : 0;
    }
    // an instance past its horizon is frozen: none of its tiles is listed
    if (t >= t_end) return;
    long long errors = extra;
    int appended = 0;
    for (int li = 0; li < nrl; ++li) {
        const int m = lb + li;
        if ((inb >> li) & 1u) {
            LaneSum s = sum[m];
            VehRec z = D.inbox[m];
            // the entrant's next road (its writer leaves it to this kernel,
            // so that the update does not wait on the route load)
            z.nr = z.rem > 0 ? D.route[z.rp + 1] : end_word(D.vend[z.vid], D.lane_len[m]);
            if (s.cnt < D.lane_cap[m]) {
                slab[D.lane_base[m] + s.cnt] = z;
                if (s.cnt == 0) s.front_reach = front_reach(z.x, z.v, D.lane_len[m], P);
                s.cnt += 1;
                s.rear = z.x - z.len;
                s.rear_v = z.v;
                put_dyn(sum[m], s);
                appended++;
            } else {
                errors++;
            }
            D.inbox_flag[m] = 0;
        }
    }
    // departures (FIFO per origin road, one per lane per step, safe entry).
    // Each entry's loads are issued together (its vehicle's status, the next
    // queue entry, every lane's summary and tables) and the choice is made
    // by selects, so that an entry costs one round of memory latency.
    const double now = (double)t * P.dt_d;
    unsigned used = 0u;
    int departed = 0;
    QRec qr = qr0;
    while (head < qe) {
        // departure times ascend along the queue: the first future one ends
        // the scan (entries already departed are skipped once they are due)
        if (!((double)qr.tau <= now)) break;
        const int v = qr.vid;
        const int st_v = D.status[v];
        const float pstart = D.vstart[v];
        QRec qn{};
        if (head + 1 < qe) qn = D.q_rec[head + 1];
        const float Lv = qr.len;
        int best = -1;
        float best_room = -TS_INF;
        int b_cnt = 0, b_cap = 0;
        uint32_t b_base = 0u;
        float b_len = 0.0f, b_fr = 0.0f;
        const uint32_t lanes_ok = qr.mask & ~used;
#pragma unroll 4
        for (int li = 0; li < nrl; ++li) {
            const int m = lb + li;
            const LaneSum s = sum[m];
            const int cap = D.lane_cap[m];
            const uint32_t base = D.lane_base[m];
            const float len = D.lane_len[m];
            // no nonempty feeder may reach past the entrant's rear (x = 0)
            const int fm = fmax_of(s.fmax, tg);
            const bool ok = ((lanes_ok >> li) & 1u) && !(fm != kNoFeeder && !(-Lv - o2f(fm) >= 0.0f));
            const float room = s.cnt > 0 ? s.rear : TS_INF;
            const bool better = ok && room > best_room;
            best_room = better ? room : best_room;
            best = better ? li : best;
            b_cnt = better ? s.cnt : b_cnt;
            b_fr = better ? s.front_reach : b_fr;
            b_cap = better ? cap : b_cap;
            b_base = better ? base : b_base;
            b_len = better ? len : b_len;
        }
        if (st_v != 0) {
            head++;
            qr = qn;
            continue;
        }
        // a start partway along the road (an AOI's connection): the entry
        // point's place in each lane's order by binary search over the
        // lane's records (front first); room ahead to the nearest vehicle
        // ahead; the nearest vehicle behind, or on a lane without one its
        // feeders, must not reach the entrant's rear within the step
        int b_k = b_cnt;
        float b_rear = 0.0f, b_rear_v = 0.0f;
        if (pstart > 0.0f) {
            best = -1;
            best_room = -TS_INF;
            for (int li = 0; li < nrl; ++li) {
                if (!((lanes_ok >> li) & 1u)) continue;
                const int m = lb + li;
                const LaneSum s = sum[m];
                const uint32_t base = D.lane_base[m];
                const VehRec* rl = slab + base;
                int lo = 0, hi = s.cnt;
                while (lo < hi) {
                    const int mid = (lo + hi) >> 1;
                    const float zx = rl[mid].x;
                    if (zx > pstart || (zx == pstart && rl[mid].vid < v)) lo = mid + 1;
                    else hi = mid;
                }
                const float room = lo > 0 ? (rl[lo - 1].x - rl[lo - 1].len) - pstart : TS_INF;
                bool safe;
                if (lo < s.cnt) {
                    const VehRec f = rl[lo];
                    safe = f.x + f.v * P.dt + P.reach <= pstart - Lv;
                } else {
                    const int fm = fmax_of(s.fmax, tg);
                    safe = !(fm != kNoFeeder && !((pstart - Lv) - o2f(fm) >= 0.0f));
                }
                if (safe && room > best_room) {
                    best_room = room;
                    best = li;
                    b_k = lo;
                    b_cnt = s.cnt;
                    b_cap = D.lane_cap[m];
                    b_base = base;
                    b_len = D.lane_len[m];
                    b_fr = s.front_reach;
                    b_rear = s.rear;
                    b_rear_v = s.rear_v;
                }
            }
        }
        if (best < 0 || !(best_room >= P.s0)) break;
        const int m = lb + best;
        if (b_cnt >= b_cap) {
            errors++;
            break;
        }
        VehRec nrec;
        nrec.x = pstart > 0.0f ? pstart : 0.0f;
        nrec.v = 0.0f;
        nrec.vid = v;
        nrec.len = Lv;
        nrec.f = qr.f;
        nrec.rp = qr.rp;
        nrec.rem = qr.rem;
        nrec.nr = qr.nr;
        LaneSum s;
        s.cnt = b_cnt + 1;
        if (pstart > 0.0f) {
            VehRec* rl = slab + b_base;
            for (int q = b_cnt; q > b_k; --q) rl[q] = rl[q - 1];
            rl[b_k] = nrec;
            s.rear = b_k == b_cnt ? pstart - Lv : b_rear;
            s.rear_v = b_k == b_cnt ? 0.0f : b_rear_v;
            s.front_reach = b_k == 0 ? front_reach(pstart, 0.0f, b_len, P) : b_fr;
        } else {
            slab[b_base + b_cnt] = nrec;
            s.rear = 0.0f - Lv;
            s.rear_v = 0.0f;
            s.front_reach = b_cnt == 0 ? front_reach(0.0f, 0.0f, b_len, P) : b_fr;
        }
        put_dyn(sum[m], s);
        D.status[v] = 1;
        used |= 1u << best;
        departed++;
        head++;
        qr = qn;
    }
    D.q_head[r] = head;
    const int n = n_prev + appended + departed;
    if (appended + departed) tile_n[r] = n;
    // the update kernels' work lists: tiles with vehicles, by size; a tile
    // emptied since the last step gets its empty summaries here
    out.r = r;
    out.inst = inst;
    out.departed = departed;
    out.errors = (int)errors;
    if (n > 0) {
        if (nl <= tiny_lanes && n <= tiny_cap) out.list = 3;
        else if (nl <= small_lanes && n <= small_cap) out.list = 0;
        else if (D.sched == kSchedFused && nl <= kWideLanes && n <= kMedCap) out.list = 4;
        else if (nl <= kWideLanes && n <= kWideCap) out.list = 1;
        else if (D.sched == kSchedFused && nl <= kLargeLanes && n <= kLargeCap) out.list = 5;
        else out.list = 2;
    }
    if (n == 0 && n_w != 0) {
        LaneSum e;
        e.cnt = 0;
        e.rear = TS_INF;
        e.rear_v = 0.0f;
        e.front_reach = -TS_INF;
        for (int li = 0; li < nl; ++li) {
            put_dyn(wsum[lb + li], e);
            D.lane_wait[lb + li] = 0;
        }
        D.road_speed[r] = -1.0f;
        tile_n_w[r] = 0;
    }
}

constexpr int kPrepThreads = 512;

// Work lists and departure counts are combined per workgroup before they
// touch the shared counters: one atomic per list (and per metric) per
// workgroup instead of one per road or wavefront.
template <int NT>
__device__ void fold_step(const DevNet& D, int total_wg);
template <int NT>
__device__ void sum_partials(const DevNet& D, int lo, int hi, long long* a);

__global__ __launch_bounds__(kPrepThreads) void k_prepare(const DevNet D, int small_lanes, int small_cap,
                                                          int tiny_lanes, int tiny_cap, int total_wg)
{
    constexpr int NW = kPrepThreads / kWave;
    constexpr int NL = kNumLists;
    __shared__ int wcnt[NL][NW];
    __shared__ int base[NL];
    __shared__ long long bsum[2][NW];
    const long long tg = *D.gstep;
    // workgroups [0, kFoldWGs) fold the previous step (below); junctions
    // and roads are spread over the others, so that the fold is not added
    // to a workgroup's share of them
    const int i = ((int)blockIdx.x - kFoldWGs) * (int)blockDim.x + (int)threadIdx.x;
    PrepOut o;
    if (blockIdx.x >= kFoldWGs) prepare_one(D, tg, i, small_lanes, small_cap, tiny_lanes, tiny_cap, o);
    const int wv = (int)threadIdx.x / kWave, lane = (int)threadIdx.x % kWave;
    unsigned long long m[NL];
#pragma unroll
    for (int L = 0; L < NL; ++L) {
        m[L] = __ballot(o.list == L);
        if (lane == 0) wcnt[L][wv] = __popcll(m[L]);
    }
    const bool one = D.n_inst == 1;
    long long dep = one ? o.departed : 0, err = one ? o.errors : 0;
    for (int off = 32; off > 0; off >>= 1) {
        dep += __shfl_down(dep, off);
        err += __shfl_down(err, off);
    }
    if (lane == 0) {
        bsum[0][wv] = dep;
        bsum[1][wv] = err;
    }
    __syncthreads();
    if (threadIdx.x < NL) {
        const int L = threadIdx.x;
        int tot = 0;
        for (int w = 0; w < NW; ++w) tot += wcnt[L][w];
        base[L] = tot ? atomicAdd(&D.list_cnt[((int)(tg & 1) * kNumLists + L) * kCntStride], tot) : 0;
    } else if (threadIdx.x == NL && one) {
        long long d = 0, e = 0;
        for (int w = 0; w < NW; ++w) {
            d += bsum[0][w];
            e += bsum[1][w];
        }
        if (d) {
            atomicAdd((unsigned long long*)&D.met[0].departed, (unsigned long long)d);
            atomicAdd((unsigned long long*)&D.met[0].dep_events, (unsigned long long)d);
        }
        if (e) atomicAdd((unsigned long long*)&D.met[0].errors, (unsigned long long)e);
    }
    __syncthreads();
    if (o.list >= 0) {
        const int L = o.list;
        int off = base[L];
        for (int w = 0; w < wv; ++w) off += wcnt[L][w];
        off += __popcll(m[L] & ((1ull << lane) - 1ull));
        int32_t* list = L == 0   ? D.list_small
                        : L == 1 ? D.list_big
                        : L == 2 ? D.list_huge
                        : L == 3 ? D.list_tiny
                        : L == 4 ? D.list_med
                                 : D.list_large;
        list[off] = o.r;
    }
    if (!one && o.r >= 0) {
        // batches: per-instance counts
        if (o.departed) {
            atomicAdd((unsigned long long*)&D.met[o.inst].departed, (unsigned long long)o.departed);
            atomicAdd((unsigned long long*)&D.met[o.inst].dep_events, (unsigned long long)o.departed);
        }
        if (o.errors) atomicAdd((unsigned long long*)&D.met[o.inst].errors, (unsigned long long)o.errors);
    }
    // step protocol.  The update's partials of the step before this one
    // (pending flag and count kept by that step's parity) are summed in
    // kFoldWGs slices here, one per fold workgroup, and the slices are
    // combined into the metrics by the first workgroup of this step's update
    // (fold_finish; batches fold their per-instance sums in workgroup 0 at
    // once).  Workgroup 0 then publishes this step for the update kernels
    // (with its number of partials, under this step's parity) and clears the
    // other parity's work-list counters for the next step.
    if (blockIdx.x < kFoldWGs) {
        const int pp = (int)((tg - 1) & 1);
        const int pending = D.fold_flag[2 * pp];
        if (pending && D.n_inst == 1) {
            const int total = D.fold_flag[2 * pp + 1];
            const int b = (int)blockIdx.x;
            long long a[kPartWords];
            sum_partials<kPrepThreads>(D, (int)((long long)total * b / kFoldWGs),
                                       (int)((long long)total * (b + 1) / kFoldWGs), a);
            if (threadIdx.x == 0) {
                long long* q = (long long*)&D.part2[b];
                for (int k = 0; k < kPartWords; ++k) q[k] = a[k];
            }
        }
        if (blockIdx.x == 0) {
            if (pending && D.n_inst > 1) fold_step<kPrepThreads>(D, 0);
            __syncthreads();
            if (threadIdx.x == 0) {
                D.fold_flag[4] = pending && D.n_inst == 1 ? 1 : 0;
                D.fold_flag[2 * (int)(tg & 1)] = 1;
                D.fold_flag[2 * (int)(tg & 1) + 1] = total_wg;
                *D.ustep = tg;
            }
            if (threadIdx.x < kNumLists)
                D.list_cnt[((int)((tg + 1) & 1) * kNumLists + (int)threadIdx.x) * kCntStride] = 0;
        }
    }
}

// ---------------------------------------------------------------------------
// update
// ---------------------------------------------------------------------------
struct DirEval {
    float u;   // utility, -inf when infeasible
    float ta;  // prospective acceleration in the target lane
    Lead lead; // target-lane leader
};

// LDS image of one road tile: lane tables, per-tile lists and counters, and
// (when staged) the tile's records and per-vehicle scratch, indexed by the
// tile enumeration j (lanes in order, front first)
template <int LANES, int CAP, int CHG>
struct TileLds {
    static constexpr int kLanes = LANES, kCap = CAP, kChg = CHG;
    int lane[LANES];
    int cnt[LANES];
    int start[LANES + 1];
    uint32_t base[LANES];
    int cap[LANES];
    float len[LANES];
    float lim[LANES];
    int jl_out[LANES];
    int jl_out_road[LANES];
    int jl_in_local[LANES];
    int jl_ext[LANES];
    int green[LANES];
    int fmx[LANES];        // road lanes: feeder max front reach (ordered int)
    LaneSum osum[LANES];   // junction lanes: summary of the out lane (with its gate and connections)
    int nstay[LANES];
    int nin[LANES];
    int nenter[LANES];
    int mcnt[LANES];       // vehicles whose merge target is this lane
    int moff[LANES];       // their bucket in mrg: start, then (once filled) end
    int wait[LANES];       // queue at the lane end: first snapshot rank whose end-of-step speed is >= 0.1
    int nlanes, nroad, n;
    int nchg, nmerge;
    int ncand;             // MOBIL candidates of the tile (listed as bytes in chg_vid until the changers use it)
    uint32_t rmask;        // restricted road lanes (bit = local lane): no lane change into them
    float chg_x[CHG];
    int chg_vid[CHG];
    int chg_lane[CHG];
    int4 mrg[CHG];         // vehicles merging: target lane, rear and speed (float bits), id
    unsigned long long sumv;
    unsigned long long sum_tt;
    int cntv;
    int changes, transfers, clamps, fblocks, finished, errors, entries;
    VehRec rec[CAP];
    float aown[CAP];
    float lrear[CAP];
    float lv[CAP];
    float nx[CAP];
    float nv[CAP];
    uint32_t gmask[CAP];
    int jq[CAP];           // packed junction lanes of the route (jq_pack)
    int pref[CAP];
    signed char merge[CAP];
    signed char kind[CAP];
    signed char nlane[CAP];
    signed char vl[CAP];   // lane of vehicle j
};

template <class TS>
__device__ __forceinline__ int lane_of(const TS& S, int j)
{
    int li = 0;
    while (j >= S.start[li + 1]) li++;
    return li;
}

template <class TS>
struct LdsView {
    TS& S;
    __device__ int lane(int j) const { return S.vl[j]; }
    __device__ VehRec rec(int j) const { return S.rec[j]; }
    __device__ float aown(int j) const { return S.aown[j]; }
    __device__ float lrear(int j) const { return S.lrear[j]; }
    __device__ float lv(int j) const { return S.lv[j]; }
    __device__ float nx(int j) const { return S.nx[j]; }
    __device__ float nv(int j) const { return S.nv[j]; }
    __device__ uint32_t gmask(int j) const { return S.gmask[j]; }
    __device__ int merge(int j) const { return (S.merge[j] & 63) - 1; }
    __device__ bool stopf(int j) const { return (S.merge[j] >> 6) & 1; }
    __device__ int kind(int j) const { return S.kind[j]; }
    __device__ int nlane(int j) const { return S.nlane[j]; }
    __device__ int pref(int j) const { return S.pref[j]; }
    __device__ int jq(int j) const { return S.jq[j]; }
    __device__ void set1(int j, uint32_t g, float a, int mt, float lr, float lvv, bool stop, int jq)
    {
        S.gmask[j] = g;
        S.jq[j] = jq;
        S.aown[j] = a;
        S.merge[j] = (signed char)((mt + 1) | (stop ? 64 : 0));
        S.lrear[j] = lr;
        S.lv[j] = lvv;
    }
    __device__ void set2(int j, float x, float v, int kind, int nl)
    {
        S.nx[j] = x;
        S.nv[j] = v;
        S.kind[j] = (signed char)kind;
        S.nlane[j] = (signed char)nl;
    }
    __device__ void set_pref(int j, int v) { S.pref[j] = v; }
    // MOBIL result of pass 2, held in the slots pass 2 fills last: decision
    // and leader flag (kind), acceleration or draw (nx), leader rear (nv)
    // and speed (pref)
    __device__ void set_mobil(int j, int dec, float ta, float rear, float lv, bool ex)
    {
        S.kind[j] = (signed char)(dec | (ex ? 4 : 0));
        S.nx[j] = ta;
        S.nv[j] = rear;
        S.pref[j] = __float_as_int(lv);
    }
    __device__ int mobil_dec(int j) const { return S.kind[j] & 3; }
    __device__ bool mobil_ex(int j) const { return (S.kind[j] & 4) != 0; }
    __device__ float mobil_ta(int j) const { return S.nx[j]; }
    __device__ float mobil_rear(int j) const { return S.nv[j]; }
    __device__ float mobil_lv(int j) const { return __int_as_float(S.pref[j]); }
};

// the same storage in global per-slot scratch, for tiles above the LDS cap
template <class TS>
struct GlobalView {
    TS& S;
    const DevNet& D;
    const VehRec* rd;
    __device__ int lane(int j) const { return lane_of(S, j); }
    __device__ uint32_t slot(int j) const
    {
        const int li = lane_of(S, j);
        return S.base[li] + (uint32_t)(j - S.start[li]);
    }
    __device__ VehRec rec(int j) const { return rd[slot(j)]; }
    __device__ float aown(int j) const { return D.sh_aown[slot(j)]; }
    __device__ float lrear(int j) const { return D.sh_lrear[slot(j)]; }
    __device__ float lv(int j) const { return D.sh_lv[slot(j)]; }
    __device__ float nx(int j) const { return D.sh_nx[slot(j)]; }
    __device__ float nv(int j) const { return D.sh_nv[slot(j)]; }
    __device__ uint32_t gmask(int j) const { return D.sh_gmask[slot(j)]; }
    __device__ int merge(int j) const { return (D.sh_merge[slot(j)] & 63) - 1; }
    __device__ bool stopf(int j) const { return (D.sh_merge[slot(j)] >> 6) & 1; }
    __device__ int kind(int j) const { return D.sh_kind[slot(j)]; }
    __device__ int nlane(int j) const { return D.sh_nlane[slot(j)]; }
    __device__ int pref(int j) const { return D.sh_pref[slot(j)]; }
    __device__ int jq(int j) const { return D.sh_jq[slot(j)]; }
    __device__ void set1(int j, uint32_t g, float a, int mt, float lr, float lvv, bool stop, int jq)
    {
        const uint32_t s = slot(j);
        D.sh_gmask[s] = g;
        D.sh_jq[s] = jq;
        D.sh_aown[s] = a;
        D.sh_merge[s] = (mt + 1) | (stop ? 64 : 0);
        D.sh_lrear[s] = lr;
        D.sh_lv[s] = lvv;
    }
    __device__ void set2(int j, float x, float v, int kind, int nl)
    {
        const uint32_t s = slot(j);
        D.sh_nx[s] = x;
        D.sh_nv[s] = v;
        D.sh_kind[s] = kind;
        D.sh_nlane[s] = nl;
    }
    __device__ void set_pref(int j, int v) { D.sh_pref[slot(j)] = v; }
    __device__ void set_mobil(int j, int dec, float ta, float rear, float lv, bool ex)
    {
        const uint32_t s = slot(j);
        D.sh_kind[s] = dec | (ex ? 4 : 0);
        D.sh_nx[s] = ta;
        D.sh_nv[s] = rear;
        D.sh_pref[s] = __float_as_int(lv);
    }
    __device__ int mobil_dec(int j) const { return D.sh_kind[slot(j)] & 3; }
    __device__ bool mobil_ex(int j) const { return (D.sh_kind[slot(j)] & 4) != 0; }
    __device__ float mobil_ta(int j) const { return D.sh_nx[slot(j)]; }
    __device__ float mobil_rear(int j) const { return D.sh_nv[slot(j)]; }
    __device__ float mobil_lv(int j) const { return __int_as_float(D.sh_pref[slot(j)]); }
};

// distance from local lane li (< 32) to the nearest lane of the group (bit
// set), 1 << 20 when the group is empty: the lowest set bit at or above li
// and the highest at or below it
__device__ __forceinline__ int group_dist(uint32_t gmask, int li, int nroad)
{
    (void)nroad;   // gmask has no bits at or above nroad
    const uint32_t up = gmask >> li;
    const uint32_t dn = gmask & (0xFFFFFFFFu >> (31 - li));
    const int du = up ? __builtin_ctz(up) : (1 << 20);
    const int dd = dn ? li - (31 - __builtin_clz(dn)) : (1 << 20);
    return du < dd ? du : dd;
}

// junction lanes (local indices) toward a vehicle's next road from the lane
// left of its own (d = -1), its own (0) and the one right of it (+1), packed
// one byte each (-1 = none)
__device__ __forceinline__ int jq_pack(int qm, int q0, int qp)
{
    return (qm + 1) | ((q0 + 1) << 8) | ((qp + 1) << 16);
}
__device__ __forceinline__ int jq_get(int pk, int d)
{
    return ((pk >> (8 * (d + 1))) & 255) - 1;
}

// stop obstacle at the end of tile lane li for a vehicle whose next road is
// nr, reaching it through junction lane q (-1: the lane does not lead there)
template <class TS>
__device__ __forceinline__ bool stop_at(const TS& S, int li, int nr, int q, bool with_wrong)
{
    if (li >= S.nroad || nr < 0) return false;
    if (q < 0) return with_wrong;
    return !S.green[q];
}

// numbers of vehicles ahead of (xa, va) in tile lane la and of (xb, vb) in
// tile lane lb: two binary searches run interleaved, so that their LDS reads
// overlap; a negative lane leaves its result untouched
template <class TS, class V>
__device__ __forceinline__ void count_ahead2(const TS& S, const V& view, int la, float xa, int va, int& ra, int lb,
                                             float xb, int vb, int& rb)
{
    int loa = 0, hia = la >= 0 ? S.cnt[la] : 0;
    int lob = 0, hib = lb >= 0 ? S.cnt[lb] : 0;
    const int ba = la >= 0 ? S.start[la] : 0, bb = lb >= 0 ? S.start[lb] : 0;
    while (loa < hia || lob < hib) {
        const bool ga = loa < hia, gb = lob < hib;
        const int ma = (loa + hia) >> 1, mb = (lob + hib) >> 1;
        float zxa = 0.0f, zxb = 0.0f;
        int zva = 0, zvb = 0;
        if (ga) {
            const VehRec z = view.rec(ba + ma);
            zxa = z.x;
            zva = z.vid;
        }
        if (gb) {
            const VehRec z = view.rec(bb + mb);
            zxb = z.x;
            zvb = z.vid;
        }
        if (ga) {
            if (ahead(zxa, zva, xa, va)) loa = ma + 1;
            else hia = ma;
        }
        if (gb) {
            if (ahead(zxb, zvb, xb, vb)) lob = mb + 1;
            else hib = mb;
        }
    }
    if (la >= 0) ra = loa;
    if (lb >= 0) rb = lob;
}

// leader substitution for a vehicle at the front of tile lane li (route info
// nr, rp, rem): rearmost vehicle of the next lane, else of the lane after it
// (q: the junction lane toward the vehicle's next road when li is a road lane)
template <class TS, class V>
__device__ Lead lookahead(const DevNet& D, const TS& S, const V& view, const LaneSum* sum, int li, int q, int rp,
                          int rem)
{
    Lead L{TS_INF, 0.0f, 0.0f, false};
    const float off = S.len[li];
    if (li < S.nroad) {
        if (q < 0) return L;
        if (S.cnt[q] > 0) {
            const VehRec z = view.rec(S.start[q] + S.cnt[q] - 1);
            L.ex = true;
            L.a = off;
            L.b = z.x - z.len;
            L.v = z.v;
            return L;
        }
        const LaneSum s2 = S.osum[q];
        if (s2.cnt > 0) {
            L.ex = true;
            L.a = off + S.len[q];
            L.b = s2.rear;
            L.v = s2.rear_v;
        }
        return L;
    }
    const LaneSum s1 = S.osum[li];
    if (s1.cnt > 0) {
        L.ex = true;
        L.a = off;
        L.b = s1.rear;
        L.v = s1.rear_v;
        return L;
    }
    if (rem < 2) return L;
    const int g1 = S.jl_out[li];
    // junction lanes leaving g1: out_pair[out_begin[g1], out_begin[g1 + 1])
    const int g2 = out_toward_range(D, D.out_begin[g1], D.out_begin[g1 + 1], D.route[rp + 2]);
    if (g2 < 0) return L;
    const LaneSum s2 = sum[g2];
    if (s2.cnt > 0) {
        L.ex = true;
        L.a = off + D.lane_len[g1];
        L.b = s2.rear;
        L.v = s2.rear_v;
    }
    return L;
}

// buffers of one step
struct StepBufs {
    long long tg;   // the global step
    const VehRec* rd;
    VehRec* wr;
    const LaneSum* rsum;
    LaneSum* wsum;
    const int32_t* rtn;
    int32_t* wtn;
};

__device__ __forceinline__ StepBufs step_bufs(const DevNet& D, long long tg)
{
    StepBufs B;
    B.tg = tg;
    const int p = (int)(tg & 1);
    B.rd = p ? D.slab1 : D.slab0;
    B.wr = p ? D.slab0 : D.slab1;
    B.rsum = p ? D.sum1 : D.sum0;
    B.wsum = p ? D.sum0 : D.sum1;
    B.rtn = p ? D.tile_n1 : D.tile_n0;
    B.wtn = p ? D.tile_n0 : D.tile_n1;
    return B;
}

// tile header, loaded one round ahead of its use
struct Hdr {
    int r, rt, wt, lb, nl, nroad, inst;
};

__device__ __forceinline__ Hdr load_hdr(const DevNet& D, const StepBufs& B, int r)
{
    Hdr h;
    h.r = r;
    h.rt = h.wt = 0;
    h.lb = h.nl = h.nroad = h.inst = 0;
    if (r < 0) return h;
    h.rt = B.rtn[r];
    h.wt = B.wtn[r];
    h.lb = D.tile_lane_begin[r];
    h.nl = D.tile_lane_begin[r + 1] - h.lb;
    h.nroad = D.tile_n_road[r];
    h.inst = D.tile_inst[r];
    return h;
}

// lane tables of the tile into LDS (thread gt < nl loads lane gt), in two
// rounds: first what the lane scan needs (one dependent load after the
// header), then what junction lanes reach through their out lane and signal,
// issued together with the record staging
struct LaneRegs {
    int g;          // out lane of a junction lane
    int junc;       // its junction
    uint32_t mask;  // its green phases
    int restr;      // a restricted road lane
};

template <class TS>
__device__ __forceinline__ LaneRegs load_lanes_a(const DevNet& D, const StepBufs& B, TS& S, const Hdr& h, int gt)
{
    LaneRegs lr{-1, 0, 0u, 0};
    if (gt >= h.nl) return lr;
    const int m = h.lb + gt;
    const bool jl = gt >= h.nroad;
    const LaneInfo L = D.lane_info[m];
    lr.restr = !jl && (L.flags & 1);
    S.lane[gt] = m;
    const int c0 = B.rsum[m].cnt;
    S.cnt[gt] = c0;
    S.base[gt] = L.base;
    S.cap[gt] = L.cap;
    S.len[gt] = L.len;
    S.lim[gt] = L.lim;
    S.nstay[gt] = 0;
    S.nin[gt] = 0;
    S.nenter[gt] = 0;
    S.mcnt[gt] = 0;
    S.wait[gt] = c0;
    S.jl_out[gt] = L.jl_out;
    S.jl_out_road[gt] = L.jl_out_road;
    S.jl_in_local[gt] = L.jl_in_local;
    S.jl_ext[gt] = L.jl_ext;
    if (jl) {
        lr.g = L.jl_out;
        lr.junc = L.jl_junc;
        lr.mask = L.green_mask;
        S.fmx[gt] = kNoFeeder;
    } else {
        S.fmx[gt] = fmax_of(B.rsum[m].fmax, B.tg);
        S.green[gt] = 1;
    }
    return lr;
}

template <class TS>
__device__ __forceinline__ void load_lanes_b(const DevNet& D, const StepBufs& B, TS& S, const Hdr& h, int gt,
                                             const LaneRegs& lr)
{
    if (gt >= h.nl || gt < h.nroad) return;
    const int cur = D.junc_cur[lr.junc];
    S.green[gt] = (cur < 0 || ((lr.mask >> cur) & 1u)) ? 1 : 0;
    S.osum[gt] = B.rsum[lr.g];
}

template <class TS>
__device__ __forceinline__ void reset_counters(TS& S, const Hdr& h)
{
    S.nlanes = h.nl;
    S.nroad = h.nroad;
    S.nchg = 0;
    S.nmerge = 0;
    S.ncand = 0;
    S.sumv = 0ull;
    S.cntv = 0;
    S.changes = S.transfers = S.clamps = S.fblocks = S.finished = S.errors = S.entries = 0;
    S.sum_tt = 0ull;
}

// MOBIL decision of vehicle j of tile S (Appendix B.3): the feasibility
// checks and utilities of both sides, the randomized choice with the
// vehicle's draw rr, and for a change the prospective acceleration and the
// target-lane leader (a bound of the move).
struct Mobil {
    int dec;     // 0 keep, 1 left, 2 right
    float ta;    // acceleration in the target lane
    Lead lead;   // target-lane leader
};

// MOBIL for one side d (-1 left, +1 right) of vehicle j: utility (-inf when
// the side is infeasible), prospective acceleration, and the target-lane
// leader used as a bound
template <class TS, class V>
__device__ DirEval mobil_side(const DevNet& D, const TS& S, const V& view, const LaneSum* rsum, int j, int d,
                              const KParams& P)
{
    DirEval o;
    o.u = -TS_INF;
    o.ta = 0.0f;
    o.lead.ex = false;
    o.lead.a = TS_INF;
    o.lead.b = 0.0f;
    o.lead.v = 0.0f;
    const int nroad = S.nroad;
    const int li = view.lane(j);
    if (li >= nroad) return o;
    const int k = li + d;
    if (k < 0 || k >= nroad) return o;
    if ((S.rmask >> k) & 1u) return o;   // no change into a restricted lane
    const uint32_t gmask = view.gmask(j);
    const bool in_g = (gmask >> li) & 1u;
    if (in_g) {
        if (!((gmask >> k) & 1u)) return o;
    } else if (!(group_dist(gmask, k, nroad) < group_dist(gmask, li, nroad))) {
        return o;
    }
    const int c = j - S.start[li];
    const VehRec rec = view.rec(j);
    const float len = S.len[li];
    const float lim = S.lim[li];
    const float a_e = view.aown(j);
    const int jqp = view.jq(j);
    const int my_mt = view.merge(j);
    // the vehicle's position among the target lane's vehicles
    int pos = 0, unused = 0;
    count_ahead2(S, view, k, rec.x, rec.vid, pos, -1, 0.0f, 0, unused);
    const int tl = pos > 0 ? S.start[k] + pos - 1 : -1;
    const int tf = pos < S.cnt[k] ? S.start[k] + pos : -1;
    VehRec tlr{}, tfr{};
    if (tl >= 0) tlr = view.rec(tl);
    if (tf >= 0) tfr = view.rec(tf);
    // same gap of k held by a vehicle two lanes right (rightward only)
    if (d > 0 && k + 1 < nroad) {
        int lo2 = 0, hi2 = S.cnt[k + 1];
        count_ahead2(S, view, tl >= 0 ? k + 1 : -1, tlr.x, tlr.vid, lo2, tf >= 0 ? k + 1 : -1, tfr.x, tfr.vid, hi2);
        if (lo2 < hi2) return o;
    }
    Lead tld;
    if (tl >= 0) {
        tld.ex = true;
        tld.a = tlr.x;
        tld.b = -tlr.len;
        tld.v = tlr.v;
    } else {
        tld = lookahead(D, S, view, rsum, k, jq_get(jqp, d), rec.rp, rec.rem);
    }
    const float g3 = tld.ex ? lead_gap(tld, rec.x) : TS_INF;
    if (!(g3 > 0.0f)) return o;
    const bool tf_yields = tf >= 0 && my_mt == k && (rec.x - rec.len > tfr.x);
    if (tf >= 0 && !tf_yields) {
        const float g4 = ((rec.x - tfr.x) - rec.len) - (tfr.v * P.dt + P.reach);
        if (!(g4 >= 0.0f)) return o;
    }
    if (tf < 0) {
        // no follower in the target lane: the lane's feeders must not reach
        // past the changer's rear (largest reach decides)
        const int fm = S.fmx[k];
        if (fm != kNoFeeder) {
            const float g = (rec.x - rec.len) - o2f(fm);
            if (!(g >= 0.0f)) return o;
        }
    }
    // desired speeds in lane k from k's own limit (lanes of a road may have
    // different limits)
    const float lim_k = S.lim[k];
    const float ta_e = accel(rec.v, rec.f * lim_k, rec.x, tld, stop_at(S, k, next_road(rec), jq_get(jqp, d), false),
                             len, P);
    float d_new = 0.0f, d_old = 0.0f;
    if (tf >= 0) {
        const float a_tf = view.aown(tf);
        const Lead me_lead{rec.x, -rec.len, rec.v, true};
        const float ta_tf = accel(tfr.v, tfr.f * lim_k, tfr.x, me_lead, view.stopf(tf), len, P);
        if (!tf_yields && !(ta_tf + P.b_safe >= 0.0f)) return o;
        d_new = ta_tf - a_tf;
    }
    if (c + 1 < S.cnt[li]) {
        // acceleration change of the old follower when this vehicle leaves
        const VehRec ofr = view.rec(j + 1);
        const float a_of = view.aown(j + 1);
        Lead ol;
        if (c > 0) {
            const VehRec z = view.rec(j - 1);
            ol.ex = true;
            ol.a = z.x;
            ol.b = -z.len;
            ol.v = z.v;
        } else {
            ol = lookahead(D, S, view, rsum, li, jq_get(view.jq(j + 1), 0), ofr.rp, ofr.rem);
        }
        const float ta_of = accel(ofr.v, ofr.f * lim, ofr.x, ol, view.stopf(j + 1), len, P);
        d_old = ta_of - a_of;
    }
    const float da = (ta_e - a_e) + P.p * (d_new + d_old);
    float ud = da - P.a_th;
    if (!in_g) ud = fmaxf(ud, 1.0f);
    o.u = ud;
    o.ta = ta_e;
    o.lead = tld;
    return o;
}

// randomized decision from both sides' evaluations and the draw rr (the
// draw only matters when a side is feasible)
__device__ __forceinline__ Mobil mobil_choose(const DirEval& eL, const DirEval& eR, float rr, const KParams& P)
{
    const float uLp = fmaxf(0.0f, eL.u), uRp = fmaxf(0.0f, eR.u);
    const float uT = uLp + uRp;
    const float pLC = uT >= 1.0f ? P.p_max : (uT > 0.0f ? P.p_min + (P.p_max - P.p_min) * uT : P.p_min);
    const bool fL = eL.u > -TS_INF, fR = eR.u > -TS_INF;
    int dec = 0;
    if (fL || fR) {
        if (uT > 0.0f) {
            const float bL = pLC * uLp / uT;
            if (uLp > 0.0f && rr < bL) dec = 1;
            else if (uRp > 0.0f && rr >= bL && rr < pLC) dec = 2;
        } else if (fL && fR) {
            if (rr < 0.5f * P.p_min) dec = 1;
            else if (rr < P.p_min) dec = 2;
        } else {
            if (rr < P.p_min) dec = fL ? 1 : 2;
        }
    }
    Mobil m;
    m.dec = dec;
    m.ta = dec == 1 ? eL.ta : eR.ta;
    m.lead = dec == 1 ? eL.lead : eR.lead;
    return m;
}

template <class TS, class V>
__device__ Mobil mobil_decide(const DevNet& D, const TS& S, const V& view, const LaneSum* rsum, int j, float rr,
                              const KParams& P)
{
    DirEval eL, eR;
#pragma unroll 1
    for (int di = 0; di < 2; ++di) {
        const DirEval e = mobil_side(D, S, view, rsum, j, di ? 1 : -1, P);
        if (di) eR = e;
        else eL = e;
    }
    return mobil_choose(eL, eR, rr, P);
}

// passes 1 and 2 of one tile (see process_tile)
template <int GW, class TS, class V>
__device__ void process_pass12(const DevNet& D, TS& S, V& view, const StepBufs& B, long long t, int inst, int gt,
                               int n)
{
    const uint32_t key0 = D.inst_key[2 * inst], key1 = D.inst_key[2 * inst + 1];
    const int vbase = D.inst_vbase[inst];
    const KParams& P = D.P;
    const int nl = S.nlanes;
    const int nroad = S.nroad;
    const LaneSum* rsum = B.rsum;

    // ---------------- pass 1: own acceleration ----------------
    for (int j = gt; j < n; j += GW) {
        const int li = view.lane(j);
        const int c = j - S.start[li];
        const VehRec rec = view.rec(j);
        const bool is_jl = li >= nroad;
        uint32_t gmask = 0u;
        int qm = -1, q0 = -1, qp = -1;
        if (!is_jl) {
            if (rec.rem == 0) {
                gmask = nroad >= 32 ? 0xFFFFFFFFu : ((1u << nroad) - 1u);
            } else {
                // branch-free so that the unrolled LDS reads issue together
#pragma unroll 4
                for (int q = nroad; q < nl; ++q) {
                    const int in = S.jl_in_local[q];
                    const bool hit = S.jl_out_road[q] == rec.nr;
                    gmask |= hit ? (1u << in) : 0u;
                    qm = (hit && in == li - 1) ? q : qm;
                    q0 = (hit && in == li) ? q : q0;
                    qp = (hit && in == li + 1) ? q : qp;
                }
            }
        }
        const int jqp = jq_pack(qm, q0, qp);
        Lead ld;
        if (c > 0) {
            const VehRec z = view.rec(j - 1);
            ld.ex = true;
            ld.a = z.x;
            ld.b = -z.len;
            ld.v = z.v;
        } else {
            ld = lookahead(D, S, view, rsum, li, q0, rec.rp, rec.rem);
        }
        const bool stop = stop_at(S, li, next_road(rec), q0, true);
        const float a = accel(rec.v, rec.f * S.lim[li], rec.x, ld, stop, S.len[li], P);
        int mt = -1;
        if (!is_jl && rec.rem > 0 && !((gmask >> li) & 1u)) {
            int bl = -1, bd = 1 << 20;
            for (int b = 0; b < nroad; ++b)
                if ((gmask >> b) & 1u) {
                    const int d = b > li ? b - li : li - b;
                    if (d < bd) {
                        bd = d;
                        bl = b;
                    }
                }
            if (bl >= 0) mt = bl < li ? li - 1 : li + 1;
        }
        view.set1(j, gmask, a, mt, ld.ex ? lead_rear(ld) : TS_INF, ld.v, stop, jqp);
        if (mt >= 0) atomicAdd(&S.mcnt[mt], 1);
    }
    tile_sync<GW>();
    // merging vehicles are bucketed by target lane (pass 2 places them), so
    // that a lane keeper scans only the mergers into its own lane: bucket
    // starts are the exclusive prefix of the per-lane counts
    {
        constexpr int SW = GW < kWave ? GW : kWave;   // a tile of several wavefronts: the first one
        if (gt < SW) {
            const int c = gt < nroad ? S.mcnt[gt] : 0;
            int x = c;
#pragma unroll
            for (int off = 1; off < SW; off <<= 1) {
                const int y = __shfl_up(x, off, SW);
                if (gt >= off) x += y;
            }
            if (gt < nroad) S.moff[gt] = x - c;
            if (gt == SW - 1) S.nmerge = x;
        }
    }
    tile_sync<GW>();

    // ---------------- pass 2: decision and motion ----------------
    // A: every vehicle draws its number (Philox, counter (vehicle, step));
    // a change needs r < p_LC <= p_max, so only vehicles with a feasible
    // side and r below p_max (with a margin far above rounding) are MOBIL
    // candidates; the others keep their lane whatever their utilities.
    // B: the candidates of every tile of the wavefront are evaluated
    // together, spread over all its lanes (one pass for up to 64), instead
    // of each tile's group walking its own vehicles.  Tiles spread over
    // several wavefronts evaluate in A.  C: motion, bounds and transfers.
    const float r_cut = P.p_max * 1.001f;
    // candidates are gathered for tiles staged in LDS (the same for every
    // tile of a wavefront: groups only hold tiles of at most kCap vehicles)
    bool compact = false;
    // (candidate indices are listed as bytes in the changer list)
    if constexpr (GW <= kWave) compact = n <= TS::kCap && n <= 4 * TS::kChg && n <= 256;
    for (int j = gt; j < n; j += GW) {
        const int li = view.lane(j);
        const VehRec rec = view.rec(j);
        const bool is_jl = li >= nroad;
        const uint32_t gmask = view.gmask(j);
        const bool in_g = !is_jl && ((gmask >> li) & 1u);
        const int dist_l = (is_jl || in_g) ? 0 : group_dist(gmask, li, nroad);
        const bool okL = !is_jl && li >= 1 &&
                         (in_g ? ((gmask >> (li - 1)) & 1u) != 0u : group_dist(gmask, li - 1, nroad) < dist_l);
        const bool okR = !is_jl && li + 1 < nroad &&
                         (in_g ? ((gmask >> (li + 1)) & 1u) != 0u : group_dist(gmask, li + 1, nroad) < dist_l);
        const int mt = view.merge(j);
        if (mt >= 0) {
            const int q = atomicAdd(&S.moff[mt], 1);
            if (q < TS::kChg) S.mrg[q] = make_int4(mt, __float_as_int(rec.x - rec.len), __float_as_int(rec.v), rec.vid);
        }
        const uint32_t w = philox_word0(key0, key1, (uint32_t)(rec.vid - vbase), (uint32_t)t);
        const float rr = (float)w * 2.3283064365386963e-10f;  // 2^-32
        const bool cand = (okL || okR) && rr < r_cut;
        if (compact) {
            view.set_mobil(j, 0, rr, 0.0f, 0.0f, false);
            if (cand) {
                const int q = atomicAdd(&S.ncand, 1);
                ((unsigned char*)S.chg_vid)[q] = (unsigned char)j;
            }
        } else {
            Mobil m{0, 0.0f, Lead{TS_INF, 0.0f, 0.0f, false}};
            if (cand) m = mobil_decide(D, S, view, rsum, j, rr, P);
            view.set_mobil(j, m.dec, m.ta, lead_rear(m.lead), m.lead.v, m.lead.ex);
        }
    }
    // a tile spread over several wavefronts: the merger buckets (moff, mrg)
    // are complete only once every wavefront has left the loop above (one
    // wavefront needs no fence: its LDS accesses complete in order)
    if constexpr (GW > kWave) tile_sync<GW>();
    if constexpr (GW <= kWave) if (compact) {
        constexpr int NG = kWave / GW;
        wave_sync();
        TS* const S0 = &S - (int)(__lane_id() / GW);   // the wavefront's tiles are consecutive
        int pre[NG];
        int tot = 0;
#pragma unroll
        for (int g = 0; g < NG; ++g) {
            pre[g] = tot;
            tot += S0[g].ncand;
        }
        // two lanes per candidate, one side each (lane 2e left, 2e + 1
        // right); the left lane combines both and decides
        for (int b2 = 0; b2 < 2 * tot; b2 += kWave) {
            const int e2 = b2 + (int)__lane_id();
            const bool act = e2 < 2 * tot;
            const int e = e2 >> 1;
            const int d = (e2 & 1) ? 1 : -1;
            DirEval r;
            r.u = -TS_INF;
            r.ta = 0.0f;
            r.lead = Lead{TS_INF, 0.0f, 0.0f, false};
            int g = 0, j = 0;
            if (act) {
                if constexpr (NG == 1) {
                    j = ((const unsigned char*)S.chg_vid)[e];
                    r = mobil_side(D, S, view, rsum, j, d, P);
                } else {
                    // several tiles per wavefront: always staged in LDS
                    g = NG - 1;
                    while (e < pre[g]) g--;
                    const TS& Sg = S0[g];
                    j = ((const unsigned char*)Sg.chg_vid)[e - pre[g]];
                    r = mobil_side(D, Sg, LdsView<TS>{S0[g]}, rsum, j, d, P);
                }
            }
            DirEval q;
            q.u = __shfl_xor(r.u, 1);
            q.ta = __shfl_xor(r.ta, 1);
            q.lead.a = __shfl_xor(r.lead.a, 1);
            q.lead.b = __shfl_xor(r.lead.b, 1);
            q.lead.v = __shfl_xor(r.lead.v, 1);
            q.lead.ex = __shfl_xor((int)r.lead.ex, 1) != 0;
            if (act && d < 0) {
                if constexpr (NG == 1) {
                    const Mobil m = mobil_choose(r, q, view.mobil_ta(j), P);
                    view.set_mobil(j, m.dec, m.ta, lead_rear(m.lead), m.lead.v, m.lead.ex);
                } else {
                    LdsView<TS> vg{S0[g]};
                    const Mobil m = mobil_choose(r, q, vg.mobil_ta(j), P);
                    vg.set_mobil(j, m.dec, m.ta, lead_rear(m.lead), m.lead.v, m.lead.ex);
                }
            }
        }
        wave_sync();
    }
    long long sv_acc = 0;   // this lane's road-lane speed sum (fixed point) and count
    int cv_acc = 0;
    for (int j = gt; j < n; j += GW) {
        const int li = view.lane(j);
        const int c = j - S.start[li];
        const VehRec rec = view.rec(j);
        const bool is_jl = li >= nroad;
        const float len = S.len[li];
        const float lim = S.lim[li];
        const float v0 = rec.f * lim;
        const float a_e = view.aown(j);
        const int jqp = view.jq(j);
        (void)c;
        const int dec = view.mobil_dec(j);
        const int nli = dec == 1 ? li - 1 : (dec == 2 ? li + 1 : li);
        float a = dec ? view.mobil_ta(j) : a_e;
        // cooperative yielding of lane keepers to vehicles merging into their lane
        bool has_y = false;
        float y_rear = TS_INF, y_v = 0.0f;
        if (!is_jl && !dec && S.mcnt[li] > 0) {
            int y_vid = 0x7FFFFFFF;
            const int nm = S.nmerge;
            if (nm <= TS::kChg) {
                // the mergers into this lane (its bucket): one 16-byte read
                // per merger, selects instead of branches, so that the
                // unrolled reads issue together (the choice does not depend
                // on the scan order)
                const int qe = S.moff[li], qb = qe - S.mcnt[li];
#pragma unroll 4
                for (int q = qb; q < qe; ++q) {
                    const int4 e = S.mrg[q];
                    const float rm = __int_as_float(e.y);
                    const bool take = e.x == li && rm > rec.x &&
                                      (!has_y || rm < y_rear || (rm == y_rear && e.w < y_vid));
                    has_y = has_y || take;
                    y_rear = take ? rm : y_rear;
                    y_v = take ? __int_as_float(e.z) : y_v;
                    y_vid = take ? e.w : y_vid;
                }
            } else {
                for (int dd = -1; dd <= 1; dd += 2) {
                    const int k2 = li + dd;
                    if (k2 < 0 || k2 >= nroad) continue;
                    for (int q = 0; q < S.cnt[k2]; ++q) {
                        const int j2 = S.start[k2] + q;
                        if (view.merge(j2) != li) continue;
                        const VehRec z = view.rec(j2);
                        const float rm = z.x - z.len;
                        if (!(rm > rec.x)) continue;
                        if (!has_y || rm < y_rear || (rm == y_rear && z.vid < y_vid)) {
                            has_y = true;
                            y_rear = rm;
                            y_v = z.v;
                            y_vid = z.vid;
                        }
                    }
                }
            }
            if (has_y) a = fminf(a, idm_follow(rec.v, v0, y_rear - rec.x, rec.v - y_v, P));
        }
        // ballistic update with in-step stop
        const float x = rec.x, v = rec.v;
        const float vh = v + a * P.dt;
        float xn, vn;
        if (vh >= 0.0f) {
            xn = x + v * P.dt + 0.5f * a * P.dt * P.dt;
            vn = vh;
        } else {
            xn = x - v * v / (2.0f * a);
            vn = 0.0f;
        }
        // snapshot bounds
        float Bd = TS_INF, vcap = TS_INF;
        const float lr = view.lrear(j);
        if (lr < TS_INF) {
            Bd = lr;
            vcap = view.lv(j);
        }
        if (dec && view.mobil_ex(j)) {
            const float r2 = view.mobil_rear(j), l2v = view.mobil_lv(j);
            if (r2 < Bd) {
                Bd = r2;
                vcap = l2v;
            } else if (r2 == Bd) {
                vcap = fminf(vcap, l2v);
            }
        }
        if (has_y) {
            if (y_rear < Bd) {
                Bd = y_rear;
                vcap = y_v;
            } else if (y_rear == Bd) {
                vcap = fminf(vcap, y_v);
            }
        }
        const int qn = jq_get(jqp, nli - li);   // junction lane from the lane it ends the step in
        if (stop_at(S, nli, next_road(rec), qn, true)) {
            if (len < Bd) {
                Bd = len;
                vcap = 0.0f;
            } else if (len == Bd) {
                vcap = 0.0f;
            }
        }
        if (xn > Bd) {
            xn = fmaxf(Bd, x);
            vn = fminf(vn, vcap);
            atomicAdd(&S.clamps, 1);
        }
        int kind = dec ? 1 : 0;
        int tgt_local = nli;
        // the lane end, or on the trip's last road its end position
        const float xend = (!is_jl && rec.rem == 0) ? word_end(rec.nr) : len;
        if (xn > xend) {
            if (!is_jl && rec.rem == 0) {
                kind = 4;
                D.status[rec.vid] = 2;
                D.finish_step[rec.vid] = (int)t;
                const double tt = (double)(t + 1) * P.dt_d - (double)D.tau[rec.vid];
                atomicAdd(&S.sum_tt, (unsigned long long)llrint(tt * kTimeFx));
                atomicAdd(&S.finished, 1);
            } else if (!is_jl) {
                kind = 2;
                tgt_local = qn;
                xn -= len;
                atomicAdd(&S.transfers, 1);
            } else {
                // feeder priority: an earlier feeder of the out lane whose
                // front vehicle can pass its end this step goes first
                const int g = S.jl_out[li];
                if (gate_of(S.osum[li].gate, B.tg) < S.jl_ext[li]) {
                    xn = len;
                    vn = 0.0f;
                    atomicAdd(&S.fblocks, 1);
                } else {
                    kind = 3;
                    VehRec o;
                    o.x = xn - len;
                    o.v = vn;
                    o.vid = rec.vid;
                    o.len = rec.len;
                    o.f = rec.f;
                    o.rp = rec.rp + 1;
                    o.rem = rec.rem - 1;
                    o.nr = -1;   // filled in by the prepare kernel that appends the entrant
                    atomicAdd(&D.inbox_flag[g], 1);   // no return: the next prepare checks the count
                    D.inbox[g] = o;
                    atomicAdd(&S.transfers, 1);
                    atomicAdd(&S.entries, 1);
                }
            }
        }
        if (dec) atomicAdd(&S.changes, 1);
        // metrics: a vehicle counts for the lane it occupied at the step start
        if (!is_jl) {
            sv_acc += (long long)llrintf(vn * kSpeedFx);
            cv_acc += 1;
        }
        // lane queue length (Section 3.3, waiting at the lane end): the run
        // of vehicles from the lane front, in snapshot order, slower than
        // 0.1 m/s at the step end ends at the first faster one
        if (!(vn < 0.1f)) atomicMin(&S.wait[li], c);
        view.set2(j, xn, vn, kind, tgt_local);
        if (kind == 0) {
            atomicAdd(&S.nstay[li], 1);
        } else if (kind == 1) {
            atomicAdd(&S.nin[nli], 1);
            const int q = atomicAdd(&S.nchg, 1);
            if (q < TS::kChg) {
                S.chg_x[q] = xn;
                S.chg_vid[q] = rec.vid;
                S.chg_lane[q] = nli;
            }
        } else if (kind == 2) {
            if (atomicAdd(&S.nenter[tgt_local], 1) != 0) atomicAdd(&S.errors, 1);
        }
    }
    // the tile's speed sums: a group reduction (integer, so in any order)
    // instead of an LDS atomic per vehicle
    if constexpr (GW <= kWave) {
#pragma unroll
        for (int off = 1; off < GW; off <<= 1) {
            sv_acc += __shfl_xor(sv_acc, off, GW);
            cv_acc += __shfl_xor(cv_acc, off, GW);
        }
        if (gt == 0) {
            S.sumv = (unsigned long long)sv_acc;
            S.cntv = cv_acc;
        }
    } else {
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) {
            sv_acc += __shfl_xor(sv_acc, off);
            cv_acc += __shfl_xor(cv_acc, off);
        }
        if (gt % kWave == 0 && cv_acc != 0) {
            atomicAdd(&S.sumv, (unsigned long long)sv_acc);
            atomicAdd(&S.cntv, cv_acc);
        }
    }
    tile_sync<GW>();
}

// pass 3 of one tile: new per-lane order, records and summaries written
template <int GW, class TS, class V>
__device__ void process_pass3(const DevNet& D, TS& S, V& view, const StepBufs& B, int gt, int gbase, int n)
{
    const KParams& P = D.P;
    const int nroad = S.nroad;
    if constexpr (GW > kWave) {
        // several wavefronts on one tile: wavefront ballots plus a prefix
        // over the wavefronts through LDS (n is the same for the workgroup)
        __shared__ int wc[GW / kWave];
        int carry = 0;
        const int wv = gt / kWave, ln = gt % kWave;
        for (int b0 = 0; b0 < n; b0 += GW) {
            const int j = b0 + gt;
            const bool st = j < n && view.kind(j) == 0;
            const unsigned long long bal = __ballot(st);
            if (ln == 0) wc[wv] = __popcll(bal);
            __syncthreads();
            int pw = 0, tot = 0;
            for (int q = 0; q < GW / kWave; ++q) {
                const int c = wc[q];
                if (q < wv) pw += c;
                tot += c;
            }
            if (j < n) view.set_pref(j, carry + pw + __popcll(bal & ((1ull << ln) - 1ull)));
            carry += tot;
            __syncthreads();
        }
    } else {
        int carry = 0;
        for (int b0 = 0; b0 < n; b0 += GW) {
            const int j = b0 + gt;
            const bool st = j < n && view.kind(j) == 0;
            const unsigned long long bal = __ballot(st);
            unsigned long long mine;
            if constexpr (GW == kWave) mine = bal;
            else mine = (bal >> gbase) & ((1ull << GW) - 1ull);
            if (j < n) view.set_pref(j, carry + __popcll(mine & ((1ull << gt) - 1ull)));
            carry += __popcll(mine);
        }
    }
    tile_sync<GW>();
    const int nchg = S.nchg;
    for (int j = gt; j < n; j += GW) {
        const int kind = view.kind(j);
        if (kind >= 3) continue;
        const int li = view.lane(j);
        const VehRec rec = view.rec(j);
        const float xn = view.nx(j);
        const int nli = view.nlane(j);
        int rank = 0;
        if (kind == 0) {
            rank = view.pref(j) - view.pref(S.start[li]);
        } else if (kind == 1) {
            // stayers of the target lane ahead of the changer (branch-free,
            // so that the unrolled reads issue together)
            const int b2 = S.start[nli], c2 = S.cnt[nli];
#pragma unroll 4
            for (int q = 0; q < c2; ++q) {
                const int j2 = b2 + q;
                rank += (int)(view.kind(j2) == 0) & (int)ahead(view.nx(j2), view.rec(j2).vid, xn, rec.vid);
            }
        } else {
            rank = S.nstay[nli];
        }
        if (kind <= 1 && S.nin[nli] > (kind == 1 ? 1 : 0)) {
            // changers into the same lane ahead of this vehicle
            if (nchg <= TS::kChg) {
#pragma unroll 4
                for (int q = 0; q < nchg; ++q) {
                    const int cv = S.chg_vid[q];
                    rank += (int)(S.chg_lane[q] == nli) & (int)(cv != rec.vid) & (int)ahead(S.chg_x[q], cv, xn, rec.vid);
                }
            } else {
                for (int dd = -1; dd <= 1; dd += 2) {
                    const int k2 = nli + dd;
                    if (k2 < 0 || k2 >= nroad) continue;
                    for (int q = 0; q < S.cnt[k2]; ++q) {
                        const int j2 = S.start[k2] + q;
                        if (view.kind(j2) != 1 || view.nlane(j2) != nli) continue;
                        const int ov = view.rec(j2).vid;
                        if (ov != rec.vid && ahead(view.nx(j2), ov, xn, rec.vid)) rank++;
                    }
                }
            }
        }
        const int mn = S.lane[nli];
        const int total = S.nstay[nli] + S.nin[nli] + S.nenter[nli];
        if (rank < S.cap[nli]) {
            VehRec o = rec;
            o.x = xn;
            o.v = view.nv(j);
            B.wr[S.base[nli] + rank] = o;
            if (rank == 0) {
                const float fr = front_reach(o.x, o.v, S.len[nli], P);
                B.wsum[mn].front_reach = fr;
                if (nli >= nroad) {
                    // this junction lane feeds its out lane next step
                    const int g = S.jl_out[nli];
                    atomicMax((unsigned long long*)&B.wsum[g].fmax, (unsigned long long)fmax_key(B.tg + 1, f2o(fr)));
                    if (fr > 0.0f)
                        atomicMax((unsigned long long*)&B.wsum[g].gate, (unsigned long long)gate_key(B.tg + 1, S.jl_ext[nli]));
                }
            }
            if (rank == total - 1) {
                B.wsum[mn].rear = o.x - o.len;
                B.wsum[mn].rear_v = o.v;
            }
        } else {
            atomicAdd(&S.errors, 1);
        }
    }
}

// the three passes of one tile; n vehicles (0 = nothing to do), run by the
// GW lanes gt of the group starting at wave lane gbase.  Every lane of the
// wavefront passes the same fences whatever its group's n is.
template <int GW, class TS, class V>
__device__ void process_tile(const DevNet& D, TS& S, V& view, const StepBufs& B, long long t, int inst, int gt,
                             int gbase, int n)
{
    process_pass12<GW>(D, S, view, B, t, inst, gt, n);
    process_pass3<GW>(D, S, view, B, gt, gbase, n);
}

// lane summaries, waiting counts and tile totals after a processed tile
template <int GW, class TS>
__device__ __forceinline__ void finish_tile(const DevNet& D, const StepBufs& B, TS& S, const Hdr& h, int gt, int n,
                                            WGPartial& acc)
{
    int c = 0, busy = 0;
    if (gt < h.nl) {
        const int m = h.lb + gt;
        busy = S.cnt[gt] > 0 ? 1 : 0;
        c = S.nstay[gt] + S.nin[gt] + S.nenter[gt];
        B.wsum[m].cnt = c < S.cap[gt] ? c : S.cap[gt];
        if (c == 0) {
            B.wsum[m].rear = TS_INF;
            B.wsum[m].rear_v = 0.0f;
            B.wsum[m].front_reach = -TS_INF;
        }
        D.lane_wait[m] = S.wait[gt];
    }
    // the tile's vehicle count: a group reduction of the lane counts when
    // the group fits in a wavefront (its lanes are active together)
    int tot = c;
    if constexpr (GW <= kWave) {
#pragma unroll
        for (int off = 1; off < GW; off <<= 1) {
            tot += __shfl_xor(tot, off, GW);
            busy += __shfl_xor(busy, off, GW);
        }
    }
    if (gt == 0) {
        if constexpr (GW > kWave) {
            tot = 0;
            busy = 0;
            for (int q = 0; q < h.nl; ++q) {
                tot += S.nstay[q] + S.nin[q] + S.nenter[q];
                busy += S.cnt[q] > 0 ? 1 : 0;
            }
        }
        B.wtn[h.r] = tot;
        D.road_speed[h.r] = S.cntv > 0 ? (float)((double)(long long)S.sumv / (double)kSpeedFx / (double)S.cntv) : -1.0f;
        acc.sumv_fx += (long long)S.sumv;
        acc.cnt += S.cntv;
        acc.active += n;
        acc.changes += S.changes;
        acc.transfers += S.transfers;
        acc.clamps += S.clamps;
        acc.feeder_blocks += S.fblocks;
        acc.finished += S.finished;
        acc.sum_tt_fx += (long long)S.sum_tt;
        acc.errors += S.errors;
        acc.lanes_busy += busy;
        acc.road_entries += S.entries;
    }
}

__device__ __forceinline__ void flush_acc(const DevNet& D, WGPartial& acc, int inst)
{
    if (inst < 0) return;
    unsigned long long* q = (unsigned long long*)&D.inst_acc[inst];
    const long long* a = (const long long*)&acc;
    for (int k = 0; k < kPartWords; ++k)
        if (a[k]) atomicAdd(q + k, (unsigned long long)a[k]);
    acc = WGPartial{};
}

// per-workgroup partial of the step (acc valid in thread 0), folded by the
// next step's prepare kernel (or a fold launched before the host reads the
// metrics); the kernel boundary makes these plain stores visible, so no
// fence or counter is needed.  Every update workgroup also advances the
// global step (all write the same value; no update workgroup reads it).
__device__ __forceinline__ void finish_step(const DevNet& D, const WGPartial& acc, int slot, long long tg)
{
    if (threadIdx.x == 0) {
        D.part[slot] = acc;
        *D.gstep = tg + 1;
    }
}

// folds the last step run (*ustep): sums its update workgroups' partials
// (or, for batches, the per-instance sums) into the metrics.  Run by one
// whole workgroup of NT threads.  The prepare kernel's other workgroups may
// be adding departures and errors to the same metrics, so those fields take
// atomics here.
// the metrics of a single-instance step from its summed partials (thread of
// the caller; fs: the step they belong to)
// gridlock detector: a step with vehicles on the network in which none on a
// road lane ends it moving and none departs, crosses a lane end or finishes
// extends the run of stalled steps; any movement ends it
__device__ __forceinline__ void note_stall(DevMetrics* M, const long long* a)
{
    const bool moved = a[0] > 0 || a[4] > 0 || a[7] > 0 || M->dep_events != M->stall_dep;
    M->stall_dep = M->dep_events;
    M->stall_steps = (a[2] > 0 && !moved) ? M->stall_steps + 1 : 0;
    if (M->stall_steps > M->max_stall) M->max_stall = M->stall_steps;
}

__device__ __forceinline__ void apply_sums(const DevNet& D, const long long* a, long long fs)
{
    DevMetrics* M = D.met;
    note_stall(M, a);
    M->vehicle_steps += a[2];
    M->lane_changes += a[3];
    M->transfers += a[4];
    M->clamps += a[5];
    M->feeder_blocks += a[6];
    M->finished += a[7];
    M->sum_tt_fx += a[8];
    M->lane_steps += a[10];
    M->road_entries += a[11];
    if (a[9]) atomicAdd((unsigned long long*)&M->errors, (unsigned long long)a[9]);
    if (a[1] > 0) {
        M->mean_speed_last = (double)a[0] / (double)kSpeedFx / (double)a[1];
        M->speed_acc += M->mean_speed_last;
        M->speed_steps += 1;
    } else {
        M->mean_speed_last = 0.0;
    }
    M->step = fs - D.inst_t0[0] + 1;
}

// sums partials [lo, hi) over a workgroup of NT threads (result in thread 0)
template <int NT>
__device__ void sum_partials(const DevNet& D, int lo, int hi, long long* a)
{
    __shared__ long long red[NT / kWave][kPartWords];
    const int tid = threadIdx.x;
#pragma unroll
    for (int k = 0; k < kPartWords; ++k) a[k] = 0;
    // partials are kPartWords / 2 16-byte words at 16-byte alignment
#pragma unroll 4
    for (int g = lo + tid; g < hi; g += NT) {
        const longlong2* q = (const longlong2*)&D.part[g];
#pragma unroll
        for (int k = 0; k < kPartWords / 2; ++k) {
            const longlong2 x = q[k];
            a[2 * k] += x.x;
            a[2 * k + 1] += x.y;
        }
    }
#pragma unroll
    for (int k = 0; k < kPartWords; ++k) {
        for (int off = 32; off > 0; off >>= 1) a[k] += __shfl_down(a[k], off);
    }
    if (tid % kWave == 0) {
#pragma unroll
        for (int k = 0; k < kPartWords; ++k) red[tid / kWave][k] = a[k];
    }
    __syncthreads();
    if (tid == 0)
        for (int w = 1; w < NT / kWave; ++w)
            for (int k = 0; k < kPartWords; ++k) a[k] += red[w][k];
}

// the second level of a single-instance fold: the kFoldWGs slice sums the
// prepare kernel wrote, combined by the first wavefront of the calling
// workgroup into the metrics of step *ustep - 1 (run by the update)
__device__ __forceinline__ void fold_finish(const DevNet& D)
{
    if (threadIdx.x >= kWave || D.fold_flag[4] == 0) return;
    const int l = (int)threadIdx.x;
    long long a[kPartWords];
#pragma unroll
    for (int k = 0; k < kPartWords; ++k) a[k] = 0;
    if (l < kFoldWGs) {
        const longlong2* q = (const longlong2*)&D.part2[l];
#pragma unroll
        for (int k = 0; k < kPartWords / 2; ++k) {
            const longlong2 x = q[k];
            a[2 * k] = x.x;
            a[2 * k + 1] = x.y;
        }
    }
#pragma unroll
    for (int k = 0; k < kPartWords; ++k) {
        for (int off = 32; off > 0; off >>= 1) a[k] += __shfl_down(a[k], off);
    }
    if (l == 0) {
        apply_sums(D, a, *D.ustep - 1);
        D.fold_flag[4] = 0;
    }
}

template <int NT>
__device__ void fold_step(const DevNet& D, int total_wg)
{
    const long long fs = *D.ustep;
    const int tid = threadIdx.x;
    if (D.n_inst > 1) {
        for (int i = tid; i < D.n_inst; i += NT) {
            if (fs - D.inst_t0[i] >= D.inst_end[i]) continue;   // frozen instance
            long long* q = (long long*)&D.inst_acc[i];
            long long a[kPartWords];
#pragma unroll
            for (int k = 0; k < kPartWords; ++k) {
                a[k] = q[k];
                q[k] = 0;
            }
            DevMetrics* M = &D.met[i];
            note_stall(M, a);
            M->vehicle_steps += a[2];
            M->lane_changes += a[3];
            M->transfers += a[4];
            M->clamps += a[5];
            M->feeder_blocks += a[6];
            M->finished += a[7];
            M->sum_tt_fx += a[8];
            M->lane_steps += a[10];
            M->road_entries += a[11];
            if (a[9]) atomicAdd((unsigned long long*)&M->errors, (unsigned long long)a[9]);
            if (a[1] > 0) {
                M->mean_speed_last = (double)a[0] / (double)kSpeedFx / (double)a[1];
                M->speed_acc += M->mean_speed_last;
                M->speed_steps += 1;
            } else {
                M->mean_speed_last = 0.0;
            }
            M->step = fs - D.inst_t0[i] + 1;
        }
    } else {
        long long a[kPartWords];
        sum_partials<NT>(D, 0, total_wg, a);
        if (tid == 0) apply_sums(D, a, fs);
    }
}

// folds a step that no prepare kernel has folded yet (launched before the
// host reads metrics); does nothing when none is pending
constexpr int kFoldThreads = 256;

__global__ __launch_bounds__(kFoldThreads) void k_fold(const DevNet D)
{
    // slice sums of the step before the last, if no update combined them
    fold_finish(D);
    const int p = (int)(*D.ustep & 1);
    if (D.fold_flag[2 * p] == 0) return;
    __syncthreads();
    fold_step<kFoldThreads>(D, D.fold_flag[2 * p + 1]);
    __syncthreads();
    if (threadIdx.x == 0) D.fold_flag[2 * p] = 0;
}


// Grouped pass: the step's small-tile list (tiles of at most GW lanes and
// CAP vehicles, built by the prepare kernel), 64 / GW tiles per wavefront,
// one group of GW lanes per tile; the grid strides over the list.
// LDS of one grouped-pass workgroup
template <int GW, int CAP, int CHG, int WPB, int LANES>
struct GroupedLds {
    static constexpr int NG = kWave / GW;
    TileLds<LANES, CAP, CHG> Sg[WPB * NG];
    WGPartial gacc[WPB * NG];
    int pst_all[WPB * NG][GW + 1];      // next tile: lane starts
    uint32_t pbs_all[WPB * NG][GW];     // next tile: lane slab bases
    signed char pvl_all[WPB * NG][CAP]; // next tile: lane of each record
};

// the grouped pass as run by workgroup blk of nblk
template <int GW, int CAP, int CHG, int WPB, int LANES, int LIST>
__device__ __forceinline__ void grouped_pass(const DevNet& D, int a_wg, int blk, int nblk,
                                             GroupedLds<GW, CAP, CHG, WPB, LANES>& L)
{
    constexpr int NG = kWave / GW;
    static_assert(LANES <= GW, "a group covers the lanes of its tile");
    using TS = TileLds<LANES, CAP, CHG>;
    TS* const Sg = L.Sg;
    WGPartial* const gacc = L.gacc;
    const long long tg = *D.ustep;
    const StepBufs B = step_bufs(D, tg);
    // the WPB wavefronts of a workgroup work independently (each its own
    // groups and tiles); they meet only to combine their partial sums
    const int w = (int)threadIdx.x / kWave, tid = (int)threadIdx.x % kWave;
    if (w >= WPB) {
        // a workgroup larger than the pass (fused launch): the extra
        // wavefronts only meet the final barrier
        __syncthreads();
        return;
    }
    const int g = tid / GW, gt = tid % GW, gbase = g * GW;
    TS& S = Sg[w * NG + g];
    const int count = D.list_cnt[((int)(tg & 1) * kNumLists + LIST) * kCntStride];
    const int32_t* const list = LIST == 0   ? D.list_small
                                : LIST == 1 ? D.list_big
                                : LIST == 3 ? D.list_tiny
                                : LIST == 4 ? D.list_med
                                            : D.list_large;
    const int first = (blk * WPB + w) * NG;
    const int stride = nblk * WPB * NG;
    const int rounds = count > first ? (count - first + stride - 1) / stride : 0;

    WGPartial acc{};
    int acc_inst = -1;

    // Software pipeline over the group's tiles: while tile k is processed,
    // the lane tables, out-lane summaries, signal states and records of tile
    // k+1 are loaded into registers (lane gt holds lane gt of the next tile
    // and records gt, gt + GW, ...), so a round starts from data in hand.
    constexpr int RPT = (CAP + GW - 1) / GW;
    static_assert(RPT <= 4, "at most four prefetched records per lane");
    int* const pst = L.pst_all[w * NG + g];
    uint32_t* const pbs = L.pbs_all[w * NG + g];
    signed char* const pvl = L.pvl_all[w * NG + g];
    LaneInfo pL{};
    int pcnt = 0, pfmx = kNoFeeder, pcur = -1, pn = 0;
    int4 poa{}, pob{};   // out-lane summary of the next tile's junction lane gt (LaneSum as two vectors)
    // records as pairs of 16-byte vectors (register-friendly)
    int4 r0a{}, r0b{}, r1a{}, r1b{}, r2a{}, r2b{}, r3a{}, r3b{};

#define TSIM_PF_LANES(H)                                                       \
    do {                                                                       \
        pcnt = 0;                                                              \
        if ((H).r >= 0 && gt < (H).nl) {                                       \
            const int m_ = (H).lb + gt;                                        \
            pL = D.lane_info[m_];                                              \
            pcnt = B.rsum[m_].cnt;                                             \
            pfmx = gt < (H).nroad ? fmax_of(B.rsum[m_].fmax, B.tg) : kNoFeeder; \
        }                                                                      \
    } while (0)
#define TSIM_PF_LANE_OF(J, LI) const int LI = pvl[J]
#define TSIM_PF_LOAD(I, RA, RB)                                                \
    do {                                                                       \
        const int j_ = gt + (I) * GW;                                          \
        if ((I) < RPT && j_ < pn) {                                            \
            TSIM_PF_LANE_OF(j_, li_);                                          \
            const int4* src_ = (const int4*)(B.rd + pbs[li_] + (uint32_t)(j_ - pst[li_])); \
            RA = src_[0];                                                      \
            RB = src_[1];                                                      \
        }                                                                      \
    } while (0)
#define TSIM_PF_STORE(I, RA, RB)                                               \
    do {                                                                       \
        const int j_ = gt + (I) * GW;                                          \
        if ((I) < RPT && j_ < pn) {                                            \
            TSIM_PF_LANE_OF(j_, li_);                                          \
            int4* dst_ = (int4*)&S.rec[j_];                                    \
            dst_[0] = RA;                                                      \
            dst_[1] = RB;                                                      \
            S.vl[j_] = (signed char)li_;                                       \
        }                                                                      \
    } while (0)
    // stage 2 (stage 1 in hand): lane starts, records, out-lane summaries and
    // signal states of tile H
#define TSIM_PF_REST(H)                                                        \
    do {                                                                       \
        int c_ = pcnt;                                                         \
        _Pragma("unroll") for (int off = 1; off < GW; off <<= 1)               \
        {                                                                      \
            const int y_ = __shfl_up(c_, off, GW);                             \
            if (gt >= off) c_ += y_;                                           \
        }                                                                      \
        pst[gt + 1] = c_;                                                      \
        if (gt == 0) pst[0] = 0;                                               \
        pbs[gt] = pL.base;                                                     \
        pn = __shfl(c_, gbase + GW - 1);                                       \
        /* lane map: lane gt marks its own records */                          \
        for (int k_ = c_ - pcnt; k_ < c_ && k_ < CAP; ++k_) pvl[k_] = (signed char)gt; \
        wave_sync();                                                           \
        if (pn <= CAP) {                                                       \
            TSIM_PF_LOAD(0, r0a, r0b);                                         \
            TSIM_PF_LOAD(1, r1a, r1b);                                         \
            TSIM_PF_LOAD(2, r2a, r2b);                                         \
            TSIM_PF_LOAD(3, r3a, r3b);                                         \
        }                                                                      \
        if ((H).r >= 0 && gt < (H).nl && gt >= (H).nroad) {                    \
            poa = ((const int4*)(B.rsum + pL.jl_out))[0];                      \
            pob = ((const int4*)(B.rsum + pL.jl_out))[1];                      \
            pcur = D.junc_cur[pL.jl_junc];                                     \
        }                                                                      \
    } while (0)

    auto pos_of = [&](int round) -> int {
        const int ps = first + round * stride + g;
        return (round < rounds && ps < count) ? ps : -1;
    };

    // headers run two tiles ahead and tile ids three ahead, so that no load
    // of a round waits for a load issued in the same round
    Hdr cur = load_hdr(D, B, pos_of(0) >= 0 ? list[pos_of(0)] : -1);
    Hdr nxt = load_hdr(D, B, pos_of(1) >= 0 ? list[pos_of(1)] : -1);
    int rn2 = pos_of(2) >= 0 ? list[pos_of(2)] : -1;
    TSIM_PF_LANES(cur);
    TSIM_PF_REST(cur);
    for (int round = 0; round < rounds; ++round) {
        const Hdr h = cur;
        const long long t = tg - D.inst_t0[h.inst];
        // the prefetched tile becomes the LDS image of the current tile
        if (h.r >= 0 && gt < h.nl) {
            S.lane[gt] = h.lb + gt;
            S.cnt[gt] = pcnt;
            S.base[gt] = pL.base;
            S.cap[gt] = pL.cap;
            S.len[gt] = pL.len;
            S.lim[gt] = pL.lim;
            S.nstay[gt] = 0;
            S.nin[gt] = 0;
            S.nenter[gt] = 0;
            S.mcnt[gt] = 0;
            S.wait[gt] = pcnt;
            S.jl_out[gt] = pL.jl_out;
            S.jl_out_road[gt] = pL.jl_out_road;
            S.jl_in_local[gt] = pL.jl_in_local;
            S.jl_ext[gt] = pL.jl_ext;
            S.fmx[gt] = pfmx;
            if (gt >= h.nroad) {
                S.green[gt] = (pcur < 0 || ((pL.green_mask >> pcur) & 1u)) ? 1 : 0;
                ((int4*)&S.osum[gt])[0] = poa;
                ((int4*)&S.osum[gt])[1] = pob;
            } else {
                S.green[gt] = 1;
            }
        }
        {
            const unsigned long long rb = __ballot(h.r >= 0 && gt < h.nroad && (pL.flags & 1));
            if constexpr (GW == kWave) {
                if (gt == 0) S.rmask = (uint32_t)rb;
            } else {
                if (gt == 0) S.rmask = (uint32_t)((rb >> gbase) & ((1ull << GW) - 1ull));
            }
        }
        if (gt < LANES) S.start[gt + 1] = pst[gt + 1];
        if (gt == 0) {
            S.start[0] = 0;
            reset_counters(S, h);
            S.n = h.r >= 0 ? pn : 0;
        }
        if (pn <= CAP) {
            TSIM_PF_STORE(0, r0a, r0b);
            TSIM_PF_STORE(1, r1a, r1b);
            TSIM_PF_STORE(2, r2a, r2b);
            TSIM_PF_STORE(3, r3a, r3b);
        }
        wave_sync();
        // the list holds tiles of at most CAP vehicles; a tile count that
        // disagrees with its lanes (only after a capacity error) is skipped
        const int n = S.n <= CAP ? S.n : 0;
        if (S.n > CAP && gt == 0) atomicAdd((unsigned long long*)&D.met[h.inst].errors, 1ull);
        // next tile: lane tables now, the rest after pass 2
        TSIM_PF_LANES(nxt);
        const int rn3 = pos_of(round + 3) >= 0 ? list[pos_of(round + 3)] : -1;
        LdsView<TS> view{S};
        process_pass12<GW>(D, S, view, B, t, h.inst, gt, n);
        TSIM_PF_REST(nxt);
        const Hdr nn = load_hdr(D, B, rn2);
        process_pass3<GW>(D, S, view, B, gt, gbase, n);
        wave_sync();
        if (n > 0) {
            if (gt == 0 && D.n_inst > 1 && h.inst != acc_inst) {
                flush_acc(D, acc, acc_inst);
                acc_inst = h.inst;
            }
            finish_tile<GW>(D, B, S, h, gt, n, acc);
        }
        wave_sync();
        cur = nxt;
        nxt = nn;
        rn2 = rn3;
    }
#undef TSIM_PF_LANES
#undef TSIM_PF_LANE_OF
#undef TSIM_PF_LOAD
#undef TSIM_PF_STORE
#undef TSIM_PF_REST
    if (D.n_inst > 1 && gt == 0) flush_acc(D, acc, acc_inst);
    // group partials -> workgroup partial
    if (gt == 0) gacc[w * NG + g] = acc;
    __syncthreads();
    WGPartial tot{};
    if (threadIdx.x == 0) {
        for (int q = 0; q < WPB * NG; ++q) {
            long long* a = (long long*)&tot;
            const long long* b = (const long long*)&gacc[q];
            for (int k = 0; k < kPartWords; ++k) a[k] += b[k];
        }
    }
    finish_step(D, tot, a_wg + blk, tg);
}

template <int GW, int CAP, int CHG, int WPB, int LANES = GW, int LIST = 0>
__global__ __launch_bounds__(kWave * WPB) void k_update_grouped(const DevNet D, int a_wg)
{
    __shared__ GroupedLds<GW, CAP, CHG, WPB, LANES> L;
    grouped_pass<GW, CAP, CHG, WPB, LANES, LIST>(D, a_wg, (int)blockIdx.x, (int)gridDim.x, L);
}

constexpr int kWideWaves = 2;   // wavefronts per wide-pass workgroup

// Wide pass: one tile of a list per wavefront, its vehicles staged in LDS up
// to CAP (more: global scratch); the first WPB wavefronts of the workgroup
// work, any others only meet the final barrier.  Part slots follow the
// grouped pass's (offset a_wg).
template <int LANES, int CAP, int WPB, int LIST>
__device__ __forceinline__ void wide_pass(const DevNet& D, int a_wg, int blk, int nblk,
                                          TileLds<LANES, CAP, kChangerCap>* Sw, WGPartial* wacc)
{
    using TS = TileLds<LANES, CAP, kChangerCap>;
    const long long tg = *D.ustep;
    const StepBufs B = step_bufs(D, tg);
    const int w = (int)threadIdx.x / kWave, tid = (int)threadIdx.x % kWave;
    const int count = D.list_cnt[((int)(tg & 1) * kNumLists + LIST) * kCntStride];
    const int32_t* list = LIST == 1 ? D.list_big : (LIST == 5 ? D.list_large : D.list_huge);

    WGPartial acc{};
    int acc_inst = -1;
    if (w < WPB) {
        TS& S = Sw[w];
        for (int k = blk * WPB + w; k < count; k += nblk * WPB) {
            const Hdr h = load_hdr(D, B, list[k]);
            const long long t = tg - D.inst_t0[h.inst];
            const LaneRegs lr = load_lanes_a(D, B, S, h, tid);
            {
                const unsigned long long rb = __ballot(lr.restr);
                if (tid == 0) S.rmask = (uint32_t)rb;
            }
            if (tid == 0) reset_counters(S, h);
            wave_sync();
            {
                int c = tid < h.nl ? S.cnt[tid] : 0;
#pragma unroll
                for (int off = 1; off < kWave; off <<= 1) {
                    const int y = __shfl_up(c, off);
                    if (tid >= off) c += y;
                }
                if (tid < h.nl) S.start[tid + 1] = c;
                if (tid == 0) S.start[0] = 0;
                if (tid == kWave - 1) S.n = c;
            }
            wave_sync();
            const int n = S.n;
            load_lanes_b(D, B, S, h, tid, lr);
            if (n <= CAP) {
                for (int j = tid; j < n; j += kWave) {
                    const int li = lane_of(S, j);
                    S.vl[j] = (signed char)li;
                    S.rec[j] = B.rd[S.base[li] + (j - S.start[li])];
                }
                wave_sync();
                LdsView<TS> view{S};
                process_tile<kWave>(D, S, view, B, t, h.inst, tid, 0, n);
            } else {
                wave_sync();
                GlobalView<TS> view{S, D, B.rd};
                process_tile<kWave>(D, S, view, B, t, h.inst, tid, 0, n);
            }
            wave_sync();
            if (tid == 0 && D.n_inst > 1 && h.inst != acc_inst) {
                flush_acc(D, acc, acc_inst);
                acc_inst = h.inst;
            }
            finish_tile<kWave>(D, B, S, h, tid, n, acc);
            wave_sync();
        }
        if (D.n_inst > 1 && tid == 0) flush_acc(D, acc, acc_inst);
        if (tid == 0) wacc[w] = acc;
    }
    __syncthreads();
    WGPartial tot{};
    if (threadIdx.x == 0) {
        for (int q = 0; q < WPB; ++q) {
            long long* a = (long long*)&tot;
            const long long* b = (const long long*)&wacc[q];
            for (int k = 0; k < kPartWords; ++k) a[k] += b[k];
        }
    }
    finish_step(D, tot, a_wg + blk, tg);
}

template <int LANES, int CAP, int WPB, int LIST>
__global__ __launch_bounds__(kWave * WPB) void k_update_wide(const DevNet D, int a_wg)
{
    using TS = TileLds<LANES, CAP, kChangerCap>;
    __shared__ TS Sw[WPB];
    __shared__ WGPartial wacc[WPB];
    wide_pass<LANES, CAP, WPB, LIST>(D, a_wg, (int)blockIdx.x, (int)gridDim.x, Sw, wacc);
}

constexpr int kHugeThreads = 256;   // threads working together on one huge tile

// Huge pass: the step's huge list, one tile per workgroup of TPB threads
// (several wavefronts per tile, barrier-separated passes); up to CAP vehicles
// staged in LDS, more on global per-slot scratch.
// the huge-tile pass as run by workgroup blk of nblk
template <int LANES, int CAP, int TPB, int LIST>
__device__ __forceinline__ void block_pass(const DevNet& D, int a_wg, int blk, int nblk,
                                           TileLds<LANES, CAP, kChangerCap>& S)
{
    static_assert(LANES <= kWave, "lane scan by the first wavefront");
    using TS = TileLds<LANES, CAP, kChangerCap>;
    const long long tg = *D.ustep;
    const StepBufs B = step_bufs(D, tg);
    const int tid = (int)threadIdx.x;
    const int count = D.list_cnt[((int)(tg & 1) * kNumLists + LIST) * kCntStride];
    const int32_t* list = LIST == 1 ? D.list_big : (LIST == 5 ? D.list_large : D.list_huge);

    // the previous step's metrics (every schedule runs this pass's first
    // workgroup; a single instance's fold ends here)
    if (blk == 0) fold_finish(D);
    WGPartial acc{};
    int acc_inst = -1;
    for (int k = blk; k < count; k += nblk) {
        const Hdr h = load_hdr(D, B, list[k]);
        const long long t = tg - D.inst_t0[h.inst];
        const LaneRegs lr = load_lanes_a(D, B, S, h, tid);
        {
            // lanes are held by the first wavefront
            const unsigned long long rb = __ballot(lr.restr);
            if (tid == 0) S.rmask = (uint32_t)rb;
        }
        if (tid == 0) reset_counters(S, h);
        __syncthreads();
        if (tid < kWave) {
            int c = tid < h.nl ? S.cnt[tid] : 0;
#pragma unroll
            for (int off = 1; off < kWave; off <<= 1) {
                const int y = __shfl_up(c, off);
                if (tid >= off) c += y;
            }
            if (tid < h.nl) S.start[tid + 1] = c;
            if (tid == 0) S.start[0] = 0;
            if (tid == kWave - 1) S.n = c;
        }
        __syncthreads();
        const int n = S.n;
        load_lanes_b(D, B, S, h, tid, lr);
        if (n <= CAP) {
            for (int j = tid; j < n; j += TPB) {
                const int li = lane_of(S, j);
                S.vl[j] = (signed char)li;
                S.rec[j] = B.rd[S.base[li] + (j - S.start[li])];
            }
            __syncthreads();
            LdsView<TS> view{S};
            process_tile<TPB>(D, S, view, B, t, h.inst, tid, 0, n);
        } else {
            __syncthreads();
            GlobalView<TS> view{S, D, B.rd};
            process_tile<TPB>(D, S, view, B, t, h.inst, tid, 0, n);
        }
        __syncthreads();
        if (tid == 0 && D.n_inst > 1 && h.inst != acc_inst) {
            flush_acc(D, acc, acc_inst);
            acc_inst = h.inst;
        }
        finish_tile<TPB>(D, B, S, h, tid, n, acc);
        __syncthreads();
    }
    if (D.n_inst > 1 && tid == 0) flush_acc(D, acc, acc_inst);
    finish_step(D, acc, a_wg + blk, tg);
}

template <int LANES, int CAP, int TPB, int LIST>
__global__ __launch_bounds__(TPB) void k_update_block(const DevNet D, int a_wg)
{
    __shared__ TileLds<LANES, CAP, kChangerCap> S;
    block_pass<LANES, CAP, TPB, LIST>(D, a_wg, (int)blockIdx.x, (int)gridDim.x, S);
}

// All update passes of a step in one launch (fused schedule): workgroups
// [0, GC) take the huge tiles (a workgroup per tile), then GL the large ones
// (one per wavefront, the workgroup's last wavefront idle), GB the wide ones
// (one per wavefront), GM the medium ones (two per wavefront), GA the small
// and GT the tiny ones; each range
// strides over its own list, the LDS of each range is carved from one
// dynamic allocation, and the workgroups of later ranges start as earlier
// ones finish (no launches or stream joins between the passes).
// wavefronts per workgroup of the fused launch: two, so that a range's LDS
// per workgroup is half that of four and a workgroup slot, held until its
// last wavefront ends, frees sooner (measured: 4% faster than four)
constexpr int kFusedWaves = 2;
constexpr int kFusedThreads = kFusedWaves * kWave;
using FusedWide = GroupedLds<kWave, kWideCap, kChangerCap, kFusedWaves, kWideLanes>;
using FusedMed = GroupedLds<32, kMedCap, 32, kFusedWaves, kWideLanes>;
using FusedSmall = GroupedLds<16, 32, 16, kFusedWaves, 16>;
using FusedTiny = GroupedLds<8, 16, 8, kFusedWaves, 8>;
constexpr size_t cmax(size_t a, size_t b) { return a > b ? a : b; }
constexpr size_t kFusedGroupedLds =
    cmax(cmax(sizeof(FusedWide), sizeof(FusedMed)), cmax(sizeof(FusedSmall), sizeof(FusedTiny)));
// the huge range stages up to kFusedHugeCap vehicles in LDS: the grouped
// ranges set the launch's LDS size, and a huge tile uses all of it (a tile
// above the cap works on global scratch, much slower)
constexpr int kFusedHugeCap = kFusedWaves == 4 ? 1024 : 448;
using FusedHuge = TileLds<kMaxTileLanes, kFusedHugeCap, kChangerCap>;
static_assert(sizeof(FusedHuge) <= kFusedGroupedLds, "the huge range fits the grouped ranges' LDS");
// the large range: one tile per wavefront (software-pipelined like the
// grouped ones), every wavefront of the workgroup: the tile cap is chosen
// so that two images fit the launch's LDS (measured: 3.8% faster per step
// than one wavefront per workgroup with a cap of 256 vehicles, the other
// wavefront idle)
constexpr int kFusedLargeWaves = kFusedWaves;
using FusedLarge = GroupedLds<kWave, kLargeCap, kChangerCap, kFusedLargeWaves, kLargeLanes>;
static_assert(sizeof(FusedLarge) <= kFusedGroupedLds, "the large range fits the grouped ranges' LDS");
constexpr size_t kFusedLds = cmax(sizeof(FusedHuge), kFusedGroupedLds);

__global__ __launch_bounds__(kFusedThreads) void k_update_fused(const DevNet D)
{
    extern __shared__ __align__(16) char fused_lds[];
    int b = (int)blockIdx.x;
    if (b < D.GC) {
        block_pass<kMaxTileLanes, kFusedHugeCap, kFusedThreads, 2>(D, D.GA + D.GB, b, D.GC,
                                                                 *reinterpret_cast<FusedHuge*>(fused_lds));
        return;
    }
    b -= D.GC;
    if (b < D.GL) {
        grouped_pass<kWave, kLargeCap, kChangerCap, kFusedLargeWaves, kLargeLanes, 5>(
            D, D.GA + D.GB + D.GC + D.GT + D.GM, b, D.GL, *reinterpret_cast<FusedLarge*>(fused_lds));
        return;
    }
    b -= D.GL;
    if (b < D.GB) {
        grouped_pass<kWave, kWideCap, kChangerCap, kFusedWaves, kWideLanes, 1>(D, D.GA, b, D.GB,
                                                                     *reinterpret_cast<FusedWide*>(fused_lds));
        return;
    }
    b -= D.GB;
    if (b < D.GM) {
        grouped_pass<32, kMedCap, 32, kFusedWaves, kWideLanes, 4>(D, D.GA + D.GB + D.GC + D.GT, b, D.GM,
                                                        *reinterpret_cast<FusedMed*>(fused_lds));
        return;
    }
    b -= D.GM;
    if (b < D.GA) {
        grouped_pass<16, 32, 16, kFusedWaves, 16, 0>(D, 0, b, D.GA, *reinterpret_cast<FusedSmall*>(fused_lds));
        return;
    }
    b -= D.GA;
    grouped_pass<8, 16, 8, kFusedWaves, 8, 3>(D, D.GA + D.GB + D.GC, b, D.GT, *reinterpret_cast<FusedTiny*>(fused_lds));
}

// ---------------------------------------------------------------------------
// host-driven helpers
// ---------------------------------------------------------------------------
__global__ void k_set_phases(const DevNet D, const int32_t* ids, const int32_t* ph, int n)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    D.junc_policy[ids[i]] = 2;
    D.junc_manual[ids[i]] = ph[i];
}

// horizon of one instance (local steps after which it is frozen)
__global__ void k_set_end(const DevNet D, int inst, long long end)
{
    D.inst_end[inst] = end;
}

// one phase entry per junction (negative = unchanged)
__global__ void k_set_all_phases(const DevNet D, const int32_t* ph)
{
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= D.NJ || ph[j] < 0) return;
    D.junc_policy[j] = 2;
    D.junc_manual[j] = ph[j];
}

// per-vehicle export of the state at a step boundary (residents + inboxes)
__global__ void k_export(const DevNet D, const int32_t* lane_ext, int32_t* o_lane, float* o_x,
                         float* o_v, int32_t* o_rpos, int32_t* o_rank)
{
    const int m = blockIdx.x * blockDim.x + threadIdx.x;
    if (m >= D.NL) return;
    const long long t = *D.gstep;
    // the buffer holding the lane's latest state: that of the current step,
    // or, for an instance frozen at its horizon, that of its last step (its
    // lanes are not written after it)
    const int inst = D.tile_inst[D.lane_tile[m]];
    const long long t0 = D.inst_t0[inst], loc = t - t0, end = D.inst_end[inst];
    const int p = (int)((t0 + (loc < end ? loc : end)) & 1);
    const VehRec* slab = p ? D.slab1 : D.slab0;
    const LaneSum* sum = p ? D.sum1 : D.sum0;
    const int c = sum[m].cnt;
    for (int q = 0; q < c; ++q) {
        const VehRec z = slab[D.lane_base[m] + q];
        o_lane[z.vid] = lane_ext[m];
        o_x[z.vid] = z.x;
        o_v[z.vid] = z.v;
        o_rpos[z.vid] = z.rp - D.route_begin[z.vid];
        o_rank[z.vid] = q;
    }
    if (D.inbox_flag[m]) {
        const VehRec z = D.inbox[m];
        o_lane[z.vid] = lane_ext[m];
        o_x[z.vid] = z.x;
        o_v[z.vid] = z.v;
        o_rpos[z.vid] = z.rp - D.route_begin[z.vid];
        o_rank[z.vid] = c;
    }
}

// trajectory output (Appendix B.2: every vehicle's motion state saved for
// output): at a step boundary whose step number is a multiple of `every`,
// one record per vehicle on the network (lane residents and inbox entrants),
// appended to the caller's buffer through a counter; records beyond
// `cap` are counted but not written.  Launched after every update while
// recording is on; other steps return at once.
__global__ void k_record(const DevNet D, const int32_t* lane_ext, TrajRec* out, long long cap,
                         unsigned long long* count, int every)
{
    const int m = blockIdx.x * blockDim.x + threadIdx.x;
    if (m >= D.NL) return;
    const long long t = *D.gstep;
    if (t % every != 0) return;
    const int p = (int)(t & 1);
    const VehRec* slab = p ? D.slab1 : D.slab0;
    const LaneSum* sum = p ? D.sum1 : D.sum0;
    const int c = sum[m].cnt;
    const int in = D.inbox_flag[m] != 0 ? 1 : 0;
    if (c + in == 0) return;
    const unsigned long long base = atomicAdd(count, (unsigned long long)(c + in));
    for (int q = 0; q < c + in; ++q) {
        if ((long long)(base + q) >= cap) break;
        const VehRec z = q < c ? slab[D.lane_base[m] + q] : D.inbox[m];
        TrajRec r;
        r.step = t;
        r.vid = z.vid;
        r.lane = lane_ext[m];
        r.x = z.x;
        r.v = z.v;
        out[base + q] = r;
    }
}

hipError_t launch_record(const DevNet& H, const int32_t* lane_ext, TrajRec* out, long long cap,
                         unsigned long long* count, int every, hipStream_t s)
{
    hipLaunchKernelGGL(k_record, dim3((H.NL + 255) / 256), dim3(256), 0, s, H, lane_ext, out, cap, count, every);
    return hipGetLastError();
}

// scatter of host-ordered records into the read slab of the current step
__global__ void k_import(const DevNet D, const uint32_t* slots, const VehRec* recs, int n)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const long long t = *D.gstep;
    VehRec* slab = (t & 1) ? D.slab1 : D.slab0;
    slab[slots[i]] = recs[i];
}

// MAX_PRESSURE signals (Section 3.2 policy list; Appendix B.2: lane pressures
// computed in the prepare phase, junction phases updated from them).  One
// thread per junction, launched before k_prepare while some junction may use
// the policy, so that the lane counts it reads are those of the step start
// (the summaries the last update wrote, plus the entrant waiting in each
// lane's inbox) before any departure or inbox merge of the step.  A
// movement's pressure is n(in lane) - n(out lane), a phase's the sum over the
// movements it makes green; the largest wins, ties to the lowest phase.  A
// junction decides only at the steps in which a multiple of its first phase's
// duration falls (t = 0, then every d0 seconds) and holds the phase in
// junc_manual in between, which the prepare kernel reads like a MANUAL phase.
constexpr int kSignalThreads = 256;

__global__ __launch_bounds__(kSignalThreads) void k_signals(const DevNet D)
{
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= D.NJ || D.junc_policy[j] != 3) return;
    const int inst = D.junc_inst[j];
    const long long tg = *D.gstep;
    const long long t = tg - D.inst_t0[inst];
    if (!(t < D.inst_end[inst])) return;
    const int b = D.junc_phase_begin[j], e = D.junc_phase_begin[j + 1];
    if (e == b) return;
    const double d0 = (double)D.phase_dur[b];
    if (d0 > 0.0 && !(floor((double)t * D.P.dt_d / d0) > floor((double)(t - 1) * D.P.dt_d / d0))) return;
    const LaneSum* sum = (tg & 1) ? D.sum1 : D.sum0;
    const int mb = D.mp_begin[j], me = D.mp_begin[j + 1];
    int best = 0;
    long long best_p = 0;
    for (int p = 0; p < e - b; ++p) {
        long long pr = 0;
        for (int k = mb; k < me; ++k) {
            const int4 mv = D.mp_mov[k];
            if (!(((uint32_t)mv.z >> p) & 1u)) continue;
            pr += (long long)(sum[mv.x].cnt + (D.inbox_flag[mv.x] != 0)) -
                  (long long)(sum[mv.y].cnt + (D.inbox_flag[mv.y] != 0));
        }
        if (p == 0 || pr > best_p) {
            best_p = pr;
            best = p;
        }
    }
    D.junc_manual[j] = best;
}

// Staging of tsim_set_signal_phases_noalloc: junction ids in the first
// kNoAllocMaxUpdates words, phases in the second.  One copy per GPU, held
// until the process ends and shared by every call on that GPU.  In host code
// `scratch` names a host-side stand-in, never the device array: the device
// address comes from noalloc_scratch().
static __device__ __align__(256) int32_t scratch[2 * kNoAllocMaxUpdates];

// The HIP runtime records a file-scope device variable for the devices it
// knows when the library's module constructor registers it; a library loaded
// before the runtime has enumerated the GPUs (an application that only counted
// devices so far) would register `scratch` for none.  This constructor runs
// before the module constructor (lower priority number) and starts the runtime
// first; without a GPU it fails harmlessly.
__attribute__((constructor(101))) static void tsim_runtime_first()
{
    (void)hipInit(0);
}

// device address of the current GPU's scratch, looked up once per device
// (the lookup allocates nothing)
hipError_t noalloc_scratch(int32_t** out)
{
    constexpr int kMaxDevices = 64;
    static std::mutex mu;
    static int32_t* ptr[kMaxDevices] = {};
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lk(mu);
    if (!ptr[dev]) {
        void* p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        ptr[dev] = (int32_t*)p;
    }
    *out = ptr[dev];
    return hipSuccess;
}

// speed limits of some lanes (host-staged internal lane ids and limits):
// the lane record every tile loads and the plain limit table
__global__ void k_set_lane_speed(const DevNet D, const int32_t* ids, const float* lim, int n)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int m = ids[i];
    const_cast<LaneInfo*>(D.lane_info)[m].lim = lim[i];
    const_cast<float*>(D.lane_lim)[m] = lim[i];
}

hipError_t launch_set_lane_speed(const DevNet& H, const int32_t* ids, const float* lim, int n, hipStream_t s)
{
    hipLaunchKernelGGL(k_set_lane_speed, dim3((n + 255) / 256), dim3(256), 0, s, H, ids, lim, n);
    return hipGetLastError();
}

// signal policies of some junctions (host-staged ids and policies)
__global__ void k_set_policy(const DevNet D, const int32_t* ids, const int32_t* pol, int n)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    D.junc_policy[ids[i]] = pol[i];
}

// launch wrappers (host side); Dd is the device copy of the view, H the host copy
hipError_t launch_prepare(const DevNet* Dd, const DevNet& H, hipStream_t s)
{
    if (H.mp_any)
        hipLaunchKernelGGL(k_signals, dim3((H.NJ + kSignalThreads - 1) / kSignalThreads), dim3(kSignalThreads), 0, s,
                           H);
    const int n = H.R + H.NJ;
    int lanes = 0, cap = 0, tl = 0, tc = 0;
    switch (H.sched) {
    case kSched8and16:
    case kSchedFused: lanes = 16; cap = 32; tl = 8; tc = 16; break;
    case kSched16x32:
    case kSched16x32P: lanes = 16; cap = 32; break;
    case kSched16x64: lanes = 16; cap = 64; break;
    case kSched32x64: lanes = 32; cap = 64; break;
    case kSched8x16: lanes = 8; cap = 16; break;
    default: break;
    }
    hipLaunchKernelGGL(k_prepare, dim3(kFoldWGs + (n + kPrepThreads - 1) / kPrepThreads), dim3(kPrepThreads), 0, s, H,
                       lanes, cap,
                       tl, tc, H.GT + H.GA + H.GB + H.GC + H.GM + H.GL);
    return hipGetLastError();
}

hipError_t launch_update(const DevNet* Dd, const DevNet& H, hipStream_t s, const PassStreams* ps)
{
    const int total = H.GT + H.GA + H.GB + H.GC + H.GM + H.GL;
    if (H.sched == kSchedFused) {
        hipLaunchKernelGGL(k_update_fused, dim3(total), dim3(kFusedThreads), kFusedLds, s, H);
        return hipGetLastError();
    }
    // pass streams: the wide pass on the step's stream, the huge, grouped and
    // tiny passes on the side streams when they are enabled
    hipStream_t sw = s, sh = s, sg = s, st = s;
    const int naux = ps ? ps->n : 0;
    if (naux > 0) {
        hipError_t e = hipEventRecord(ps->fork, s);
        for (int i = 0; i < naux && e == hipSuccess; ++i) e = hipStreamWaitEvent(ps->aux[i], ps->fork, 0);
        if (e != hipSuccess) return e;
        sh = ps->aux[0];
        sg = ps->aux[naux > 1 ? 1 : 0];
        st = ps->aux[naux > 2 ? 2 : naux - 1];
    }
    // huge tiles first: their workgroups run longest
    hipLaunchKernelGGL((k_update_block<kMaxTileLanes, kHugeCap, kHugeThreads, 2>), dim3(H.GC), dim3(kHugeThreads), 0,
                       sh, H, H.GA + H.GB);
    {
        const hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    if (H.sched == kSched16x32P || H.sched == kSched8and16)
        hipLaunchKernelGGL((k_update_grouped<kWave, kWideCap, kChangerCap, kWideWaves, kWideLanes, 1>), dim3(H.GB),
                           dim3(kWideWaves * kWave), 0, sw, H, H.GA);
    else
        hipLaunchKernelGGL((k_update_wide<kWideLanes, kWideCap, kWideWaves, 1>), dim3(H.GB), dim3(kWideWaves * kWave), 0,
                           sw, H, H.GA);
    {
        const hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    if (H.GT > 0) {
        hipLaunchKernelGGL((k_update_grouped<8, 16, 8, 4, 8, 3>), dim3(H.GT), dim3(4 * kWave), 0, st, H, H.GA + H.GB + H.GC);
        const hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    if (H.GA > 0) {
        switch (H.sched) {
        case kSched16x32:
        case kSched16x32P:
        case kSched8and16:
            hipLaunchKernelGGL((k_update_grouped<16, 32, 16, 4>), dim3(H.GA), dim3(4 * kWave), 0, sg, H, 0);
            break;
        case kSched16x64:
            hipLaunchKernelGGL((k_update_grouped<16, 64, 32, 2>), dim3(H.GA), dim3(2 * kWave), 0, sg, H, 0);
            break;
        case kSched32x64:
            hipLaunchKernelGGL((k_update_grouped<32, 64, 32, 4>), dim3(H.GA), dim3(4 * kWave), 0, sg, H, 0);
            break;
        case kSched8x16:
            hipLaunchKernelGGL((k_update_grouped<8, 16, 8, 4>), dim3(H.GA), dim3(4 * kWave), 0, sg, H, 0);
            break;
        default:
            return hipErrorInvalidValue;
        }
        const hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    for (int i = 0; i < naux; ++i) {
        hipError_t e = hipEventRecord(ps->join[i], ps->aux[i]);
        if (e == hipSuccess) e = hipStreamWaitEvent(s, ps->join[i], 0);
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

hipError_t prepare_update_kernels()
{
    return hipFuncSetAttribute((const void*)k_update_fused, hipFuncAttributeMaxDynamicSharedMemorySize, (int)kFusedLds);
}

hipError_t launch_fold(const DevNet& H, hipStream_t s)
{
    hipLaunchKernelGGL(k_fold, dim3(1), dim3(kFoldThreads), 0, s, H);
    return hipGetLastError();
}

// resident workgroups per compute unit of the update kernels (sched -1: the
// wide pass, -2: the huge pass, -3: the software-pipelined wide pass), from
// the compiled kernels' register and LDS use
int update_blocks_per_cu(int sched)
{
    int nb = 0;
    hipError_t e = hipSuccess;
    switch (sched) {
    case kSched16x32:
    case kSched16x32P:
    case kSched8and16:
        e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_update_grouped<16, 32, 16, 4>, 4 * kWave, 0);
        break;
    case -4:
        e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_update_grouped<8, 16, 8, 4, 8, 3>, 4 * kWave, 0);
        break;
    case kSchedFused:
        e = prepare_update_kernels();
        if (e == hipSuccess)
            e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_update_fused, kFusedThreads, kFusedLds);
        break;
    case -3:
        e = hipOccupancyMaxActiveBlocksPerMultiprocessor(
            &nb, k_update_grouped<kWave, kWideCap, kChangerCap, kWideWaves, kWideLanes, 1>, kWideWaves * kWave, 0);
        break;
    case kSched16x64:
        e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_update_grouped<16, 64, 32, 2>, 2 * kWave, 0);
        break;
    case kSched32x64:
        e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_update_grouped<32, 64, 32, 4>, 4 * kWave, 0);
        break;
    case kSched8x16:
        e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_update_grouped<8, 16, 8, 4>, 4 * kWave, 0);
        break;
    default:
        e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_update_wide<kWideLanes, kWideCap, kWideWaves, 1>,
                                                         kWideWaves * kWave, 0);
        break;
    case -2:
        e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_update_block<kMaxTileLanes, kHugeCap, kHugeThreads, 2>,
                                                         kHugeThreads, 0);
        break;
    }
    return e == hipSuccess ? nb : 0;
}

hipError_t launch_set_phases(const DevNet* Dd, const DevNet& H, const int32_t* ids, const int32_t* ph, int n, hipStream_t s)
{
    hipLaunchKernelGGL(k_set_phases, dim3((n + 255) / 256), dim3(256), 0, s, H, ids, ph, n);
    return hipGetLastError();
}

hipError_t launch_set_policy(const DevNet* Dd, const DevNet& H, const int32_t* ids, const int32_t* pol, int n, hipStream_t s)
{
    hipLaunchKernelGGL(k_set_policy, dim3((n + 255) / 256), dim3(256), 0, s, H, ids, pol, n);
    return hipGetLastError();
}

hipError_t launch_set_all_phases(const DevNet* Dd, const DevNet& H, const int32_t* ph, hipStream_t s)
{
    hipLaunchKernelGGL(k_set_all_phases, dim3((H.NJ + 255) / 256), dim3(256), 0, s, H, ph);
    return hipGetLastError();
}

hipError_t launch_set_end(const DevNet& H, int inst, long long end, hipStream_t s)
{
    hipLaunchKernelGGL(k_set_end, dim3(1), dim3(1), 0, s, H, inst, end);
    return hipGetLastError();
}

hipError_t launch_export(const DevNet* Dd, const DevNet& H, const int32_t* lane_ext, int32_t* o_lane, float* o_x,
                         float* o_v, int32_t* o_rpos, int32_t* o_rank, hipStream_t s)
{
    hipLaunchKernelGGL(k_export, dim3((H.NL + 255) / 256), dim3(256), 0, s, H, lane_ext, o_lane, o_x, o_v, o_rpos,
                       o_rank);
    return hipGetLastError();
}

hipError_t launch_import(const DevNet* Dd, const DevNet& H, const uint32_t* slots, const VehRec* recs, int n, hipStream_t s)
{
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_import, dim3((n + 255) / 256), dim3(256), 0, s, H, slots, recs, n);
    return hipGetLastError();
}

}  // namespace tsim
