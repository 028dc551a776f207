// Device kernels of the gfx950 microscopic traffic stepper.
//
// One simulation step (Section 3.1 two-phase process, Appendix B.2):
//   k_prepare  one thread per junction: phase of the step (Section 3.2
//              FIXED_TIME / MANUAL / NONE); one thread per road: append the
//              junction-to-road entrant held in each road lane's inbox, then
//              release due departures into the origin road's lanes when safe.
//   k_update   one wavefront per road tile, grid-stride over tiles.  Pass 1:
//              own leader (or two-lane lookahead), lane group, stop obstacle,
//              own IDM acceleration, merge target.  Pass 2: randomized MOBIL
//              (Appendix B.3), Philox draw, ballistic integration with snapshot
//              bounds, lane-end transfer.  Pass 3: new per-lane order (stayers
//              keep theirs, changers merge by position) written to the other
//              slab buffer.  The last workgroup folds the step's metrics.
// Reads of the step come only from slab buffer t&1 and its counts; writes go
// to buffer (t+1)&1, the inboxes and per-vehicle status, so the update is free
// of read/write races without any lock.
#include "tsim_internal.h"

namespace tsim {

#define TS_INF __builtin_huge_valf()

struct Lead {
    float rear;  // rear bumper in the follower's lane coordinate
    float v;
    bool ex;
};

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
__device__ __forceinline__ float idm_free_term(float v, float v0, const KParams& P)
{
    const float r = v / v0;
    const float q = P.delta_is_4 ? (r * r) * (r * r) : powf(r, P.delta);
    return 1.0f - q;
}

__device__ __forceinline__ float idm_follow(float v, float v0, float s, float dv, const KParams& P)
{
    if (!(s > 0.0f)) return -P.a_emerg;
    const float fr = idm_free_term(v, v0, P);
    const float ss = P.s0 + fmaxf(0.0f, v * P.T + v * dv * P.inv_2sqrt_ab);
    const float q = ss / s;
    return fmaxf(P.a_max * (fr - q * q), -P.a_emerg);
}

__device__ __forceinline__ float idm_freeroad(float v, float v0, const KParams& P)
{
    return fmaxf(P.a_max * idm_free_term(v, v0, P), -P.a_emerg);
}

__device__ __forceinline__ float accel(float v, float v0, float x, Lead ld, bool stop, float len, const KParams& P)
{
    float a = ld.ex ? idm_follow(v, v0, ld.rear - x, v - ld.v, P) : idm_freeroad(v, v0, P);
    if (stop) a = fminf(a, idm_follow(v, v0, len - x, v, P));
    return a;
}

__device__ __forceinline__ bool jl_green(const DevNet& D, int g)
{
    const int cur = D.junc_cur[D.jl_junc[g]];
    return cur < 0 || ((D.jl_green_mask[g] >> cur) & 1u);
}

// junction lane leaving road lane m toward road nr, or -1
__device__ __forceinline__ int out_toward(const DevNet& D, int m, int nr)
{
    if (nr < 0) return -1;
    for (int e = D.out_begin[m]; e < D.out_begin[m + 1]; ++e) {
        const int g = D.out_jl[e];
        if (D.jl_out_road[g] == nr) return g;
    }
    return -1;
}

// leader substitution when lane m has nobody ahead: rearmost vehicle of the
// next lane of the route, else of the lane after it
__device__ Lead lookahead(const DevNet& D, const VehRec* slab, const int32_t* cnt, int m, bool m_is_jl, int nr,
                          int rp, int rem)
{
    Lead L{TS_INF, 0.0f, false};
    const int g1 = m_is_jl ? D.jl_out[m] : out_toward(D, m, nr);
    if (g1 < 0) return L;
    const float off = D.lane_len[m];
    const int c1 = cnt[g1];
    if (c1 > 0) {
        const VehRec z = slab[D.lane_base[g1] + c1 - 1];
        L.ex = true;
        L.rear = off + (z.x - z.len);
        L.v = z.v;
        return L;
    }
    int g2;
    if (m_is_jl) {
        if (rem < 2) return L;
        g2 = out_toward(D, g1, D.route[rp + 2]);
    } else {
        g2 = D.jl_out[g1];
    }
    if (g2 < 0) return L;
    const int c2 = cnt[g2];
    if (c2 > 0) {
        const VehRec z = slab[D.lane_base[g2] + c2 - 1];
        L.ex = true;
        L.rear = (off + D.lane_len[g1]) + (z.x - z.len);
        L.v = z.v;
    }
    return L;
}

// stop obstacle at the end of road lane m: red next junction lane, or (with
// with_wrong) no connection to the next road
__device__ __forceinline__ bool stop_end(const DevNet& D, int m, bool m_is_jl, int nr, bool with_wrong)
{
    if (m_is_jl || nr < 0) return false;
    const int g = out_toward(D, m, nr);
    if (g < 0) return with_wrong;
    return !jl_green(D, g);
}

// ---------------------------------------------------------------------------
// prepare
// ---------------------------------------------------------------------------
__global__ void k_prepare(DevNet D)
{
    const long long t = D.met->step;
    const int p = (int)(t & 1);
    VehRec* slab = p ? D.slab1 : D.slab0;
    int32_t* cnt = p ? D.cnt1 : D.cnt0;
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    const KParams& P = D.P;

    if (i < D.NJ) {
        const int b = D.junc_phase_begin[i], e = D.junc_phase_begin[i + 1];
        int cur = -1;
        const int pol = D.junc_policy[i];
        if (pol != 0 && e > b) {
            if (pol == 2) {
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
    }
    if (i >= D.R) return;
    const int r = i;
    const int lb = D.tile_lane_begin[r];
    const int nrl = D.tile_n_road[r];
    long long errors = 0;
    for (int li = 0; li < nrl; ++li) {
        const int m = lb + li;
        if (D.inbox_flag[m]) {
            const int c = cnt[m];
            if (c < D.lane_cap[m]) {
                slab[D.lane_base[m] + c] = D.inbox[m];
                cnt[m] = c + 1;
            } else {
                errors++;
            }
            D.inbox_flag[m] = 0;
        }
    }
    // departures (FIFO per origin road, one per lane per step, safe entry)
    int head = D.q_head[r];
    const int qe = D.q_begin[r + 1];
    const double now = (double)t * P.dt_d;
    unsigned used = 0u;
    int departed = 0;
    while (head < qe) {
        const int v = D.q_veh[head];
        if (D.status[v] != 0) {
            head++;
            continue;
        }
        if (!((double)D.tau[v] <= now)) break;
        const int rb = D.route_begin[v];
        const int rl = D.route_begin[v + 1] - rb;
        const int nr = rl > 1 ? D.route[rb + 1] : -1;
        const float Lv = D.vlen[v];
        int best = -1;
        float best_room = -TS_INF;
        for (int li = 0; li < nrl; ++li) {
            if (used & (1u << li)) continue;
            const int m = lb + li;
            if (nr >= 0 && out_toward(D, m, nr) < 0) continue;
            bool safe = true;
            for (int e = D.feed_begin[m]; e < D.feed_begin[m + 1]; ++e) {
                const int fl = D.feed_jl[e];
                const int cf = cnt[fl];
                if (cf == 0) continue;
                const VehRec h = slab[D.lane_base[fl]];
                const float mg = -Lv - (h.x + h.v * P.dt + P.reach - D.lane_len[fl]);
                if (!(mg >= 0.0f)) safe = false;
            }
            if (!safe) continue;
            const int c = cnt[m];
            float room = TS_INF;
            if (c > 0) {
                const VehRec z = slab[D.lane_base[m] + c - 1];
                room = z.x - z.len;
            }
            if (room > best_room) {
                best_room = room;
                best = li;
            }
        }
        if (best < 0 || !(best_room >= P.s0)) break;
        const int m = lb + best;
        const int c = cnt[m];
        if (c >= D.lane_cap[m]) {
            errors++;
            break;
        }
        VehRec nrec;
        nrec.x = 0.0f;
        nrec.v = 0.0f;
        nrec.vid = v;
        nrec.len = Lv;
        nrec.f = D.vf[v];
        nrec.rp = rb;
        nrec.rem = rl - 1;
        nrec.nr = nr;
        slab[D.lane_base[m] + c] = nrec;
        cnt[m] = c + 1;
        D.status[v] = 1;
        used |= 1u << best;
        departed++;
        head++;
    }
    D.q_head[r] = head;
    if (departed) {
        atomicAdd((unsigned long long*)&D.met->departed, (unsigned long long)departed);
        atomicAdd((unsigned long long*)&D.met->dep_events, (unsigned long long)departed);
    }
    if (errors) atomicAdd((unsigned long long*)&D.met->errors, (unsigned long long)errors);
}

// ---------------------------------------------------------------------------
// update
// ---------------------------------------------------------------------------
struct DirEval {
    float u;   // utility, -inf when infeasible
    float ta;  // prospective acceleration in the target lane
    Lead lead; // target-lane leader
};

struct TileShared {
    int lane[kMaxTileLanes];
    int cnt[kMaxTileLanes];
    int start[kMaxTileLanes + 1];
    uint32_t base[kMaxTileLanes];
    float len[kMaxTileLanes];
    float lim[kMaxTileLanes];
    int jl_out_road[kMaxTileLanes];
    int jl_in_local[kMaxTileLanes];
    int nstay[kMaxTileLanes];
    int nin[kMaxTileLanes];
    int nenter[kMaxTileLanes];
    int wait[kMaxTileLanes];
    int nlanes, nroad, n;
    int nchg, nmerge;
    float chg_x[kChangerCap];
    int chg_vid[kChangerCap];
    int chg_lane[kChangerCap];
    int mrg_tgt[kMergeCap];
    float mrg_rear[kMergeCap];
    float mrg_v[kMergeCap];
    int mrg_vid[kMergeCap];
    unsigned long long sumv;
    int cntv;
    int changes, transfers, clamps, fblocks, finished, errors;
    unsigned long long sum_tt;
};

__device__ __forceinline__ int lane_of(const TileShared& S, int j)
{
    int li = 0;
    while (j >= S.start[li + 1]) li++;
    return li;
}

// nearest lane of the group (bit set) to local lane li; ties to the left
__device__ __forceinline__ int group_dist(uint32_t gmask, int li, int nroad)
{
    int best = 1 << 20;
    for (int b = 0; b < nroad; ++b)
        if ((gmask >> b) & 1u) {
            const int d = b > li ? b - li : li - b;
            if (d < best) best = d;
        }
    return best;
}

// number of vehicles of tile lane li (front first) ahead of (x, vid)
__device__ __forceinline__ int count_ahead(const TileShared& S, const VehRec* slab, int li, float x, int vid)
{
    int lo = 0, hi = S.cnt[li];
    const uint32_t b = S.base[li];
    while (lo < hi) {
        const int mid = (lo + hi) >> 1;
        const VehRec z = slab[b + mid];
        if (ahead(z.x, z.vid, x, vid)) lo = mid + 1;
        else hi = mid;
    }
    return lo;
}

__global__ __launch_bounds__(kWave) void k_update(DevNet D)
{
    __shared__ TileShared S;
    const long long t = D.met->step;
    const int p = (int)(t & 1);
    const VehRec* rd = p ? D.slab1 : D.slab0;
    VehRec* wr = p ? D.slab0 : D.slab1;
    const int32_t* rcnt = p ? D.cnt1 : D.cnt0;
    int32_t* wcnt = p ? D.cnt0 : D.cnt1;
    const KParams& P = D.P;
    const int tid = threadIdx.x;

    WGPartial acc{};

    for (int ti = blockIdx.x; ti < D.R; ti += gridDim.x) {
        const int r = D.tile_order[ti];
        const int lb = D.tile_lane_begin[r];
        const int nl = D.tile_lane_begin[r + 1] - lb;
        const int nroad = D.tile_n_road[r];
        if (tid < nl) {
            const int m = lb + tid;
            S.lane[tid] = m;
            S.cnt[tid] = rcnt[m];
            S.base[tid] = D.lane_base[m];
            S.len[tid] = D.lane_len[m];
            S.lim[tid] = D.lane_lim[m];
            S.jl_out_road[tid] = tid >= nroad ? D.jl_out_road[m] : -1;
            S.jl_in_local[tid] = tid >= nroad ? D.jl_in_local[m] : -1;
            S.nstay[tid] = 0;
            S.nin[tid] = 0;
            S.nenter[tid] = 0;
            S.wait[tid] = 0;
        }
        if (tid == 0) {
            S.nlanes = nl;
            S.nroad = nroad;
            S.nchg = 0;
            S.nmerge = 0;
            S.sumv = 0ull;
            S.cntv = 0;
            S.changes = S.transfers = S.clamps = S.fblocks = S.finished = S.errors = 0;
            S.sum_tt = 0ull;
        }
        __syncthreads();
        if (tid == 0) {
            int s = 0;
            for (int li = 0; li < nl; ++li) {
                S.start[li] = s;
                s += S.cnt[li];
            }
            S.start[nl] = s;
            S.n = s;
        }
        __syncthreads();
        const int n = S.n;
        if (n == 0) {
            if (tid < nl) {
                wcnt[lb + tid] = 0;
                D.lane_wait[lb + tid] = 0;
            }
            if (tid == 0) D.road_speed[r] = -1.0f;
            __syncthreads();
            continue;
        }

        // ---------------- pass 1 ----------------
        for (int j = tid; j < n; j += kWave) {
            const int li = lane_of(S, j);
            const int c = j - S.start[li];
            const uint32_t slot = S.base[li] + c;
            const VehRec rec = rd[slot];
            const bool is_jl = li >= nroad;
            const int m = S.lane[li];
            uint32_t gmask = 0u;
            if (!is_jl) {
                if (rec.nr < 0) {
                    gmask = nroad >= 32 ? 0xFFFFFFFFu : ((1u << nroad) - 1u);
                } else {
                    for (int q = nroad; q < nl; ++q)
                        if (S.jl_out_road[q] == rec.nr) gmask |= 1u << S.jl_in_local[q];
                }
            }
            Lead ld;
            if (c > 0) {
                const VehRec z = rd[slot - 1];
                ld.ex = true;
                ld.rear = z.x - z.len;
                ld.v = z.v;
            } else {
                ld = lookahead(D, rd, rcnt, m, is_jl, rec.nr, rec.rp, rec.rem);
            }
            const bool stop = stop_end(D, m, is_jl, rec.nr, true);
            const float a = accel(rec.v, rec.f * S.lim[li], rec.x, ld, stop, S.len[li], P);
            int mt = -1;
            if (!is_jl && rec.nr >= 0 && !((gmask >> li) & 1u)) {
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
            D.sh_gmask[slot] = gmask;
            D.sh_aown[slot] = a;
            D.sh_merge[slot] = mt;
            D.sh_lrear[slot] = ld.ex ? ld.rear : TS_INF;
            D.sh_lv[slot] = ld.v;
            if (mt >= 0) {
                const int k = atomicAdd(&S.nmerge, 1);
                if (k < kMergeCap) {
                    S.mrg_tgt[k] = mt;
                    S.mrg_rear[k] = rec.x - rec.len;
                    S.mrg_v[k] = rec.v;
                    S.mrg_vid[k] = rec.vid;
                }
            }
        }
        __syncthreads();

        // ---------------- pass 2 ----------------
        for (int j = tid; j < n; j += kWave) {
            const int li = lane_of(S, j);
            const int c = j - S.start[li];
            const uint32_t slot = S.base[li] + c;
            const VehRec rec = rd[slot];
            const bool is_jl = li >= nroad;
            const int m = S.lane[li];
            const float len = S.len[li];
            const float lim = S.lim[li];
            const float v0 = rec.f * lim;
            const float a_e = D.sh_aown[slot];
            const uint32_t gmask = D.sh_gmask[slot];
            const int my_mt = D.sh_merge[slot];
            const bool in_g = !is_jl && ((gmask >> li) & 1u);
            const int dist_l = (is_jl || in_g) ? 0 : group_dist(gmask, li, nroad);
            // MOBIL for one direction: utility (or -inf), prospective
            // acceleration, and the target-lane leader used as a bound
            auto eval_dir = [&](int d) -> DirEval {
                DirEval o;
                o.u = -TS_INF;
                o.ta = 0.0f;
                o.lead.ex = false;
                o.lead.rear = TS_INF;
                o.lead.v = 0.0f;
                if (is_jl) return o;
                const int k = li + d;
                if (k < 0 || k >= nroad) return o;
                if (in_g) {
                    if (!((gmask >> k) & 1u)) return o;
                } else if (!(group_dist(gmask, k, nroad) < dist_l)) {
                    return o;
                }
                const int pos = count_ahead(S, rd, k, rec.x, rec.vid);
                const int tl = pos > 0 ? (int)(S.base[k] + pos - 1) : -1;
                const int tf = pos < S.cnt[k] ? (int)(S.base[k] + pos) : -1;
                VehRec tlr{}, tfr{};
                if (tl >= 0) tlr = rd[tl];
                if (tf >= 0) tfr = rd[tf];
                // same gap of k held by a vehicle two lanes right (rightward only)
                if (d > 0 && k + 1 < nroad) {
                    const int lo2 = tl >= 0 ? count_ahead(S, rd, k + 1, tlr.x, tlr.vid) : 0;
                    const int hi2 = tf >= 0 ? count_ahead(S, rd, k + 1, tfr.x, tfr.vid) : S.cnt[k + 1];
                    if (lo2 < hi2) return o;
                }
                const int mk = S.lane[k];
                Lead tld;
                if (tl >= 0) {
                    tld.ex = true;
                    tld.rear = tlr.x - tlr.len;
                    tld.v = tlr.v;
                } else {
                    tld = lookahead(D, rd, rcnt, mk, false, rec.nr, rec.rp, rec.rem);
                }
                const float g3 = tld.ex ? tld.rear - rec.x : TS_INF;
                if (!(g3 > 0.0f)) return o;
                const bool tf_yields = tf >= 0 && my_mt == k && (rec.x - rec.len > tfr.x);
                if (tf >= 0 && !tf_yields) {
                    const float g4 = rec.x - rec.len - tfr.x - (tfr.v * P.dt + P.reach);
                    if (!(g4 >= 0.0f)) return o;
                }
                if (tf < 0) {
                    for (int e = D.feed_begin[mk]; e < D.feed_begin[mk + 1]; ++e) {
                        const int fl = D.feed_jl[e];
                        if (rcnt[fl] == 0) continue;
                        const VehRec h = rd[D.lane_base[fl]];
                        const float g = (rec.x - rec.len) - (h.x + h.v * P.dt + P.reach - D.lane_len[fl]);
                        if (!(g >= 0.0f)) return o;
                    }
                }
                const float ta_e = accel(rec.v, v0, rec.x, tld, stop_end(D, mk, false, rec.nr, false), len, P);
                float d_new = 0.0f, d_old = 0.0f;
                if (tf >= 0) {
                    const float a_tf = D.sh_aown[tf];
                    const Lead me_lead{rec.x - rec.len, rec.v, true};
                    const float ta_tf =
                        accel(tfr.v, tfr.f * lim, tfr.x, me_lead, stop_end(D, mk, false, tfr.nr, true), len, P);
                    if (!tf_yields && !(ta_tf + P.b_safe >= 0.0f)) return o;
                    d_new = ta_tf - a_tf;
                }
                if (c + 1 < S.cnt[li]) {
                    const VehRec ofr = rd[slot + 1];
                    const float a_of = D.sh_aown[slot + 1];
                    Lead ol;
                    if (c > 0) {
                        const VehRec z = rd[slot - 1];
                        ol.ex = true;
                        ol.rear = z.x - z.len;
                        ol.v = z.v;
                    } else {
                        ol = lookahead(D, rd, rcnt, m, false, ofr.nr, ofr.rp, ofr.rem);
                    }
                    const float ta_of = accel(ofr.v, ofr.f * lim, ofr.x, ol, stop_end(D, m, false, ofr.nr, true), len, P);
                    d_old = ta_of - a_of;
                }
                const float da = (ta_e - a_e) + P.p * (d_new + d_old);
                float ud = da - P.a_th;
                if (!in_g) ud = fmaxf(ud, 1.0f);
                o.u = ud;
                o.ta = ta_e;
                o.lead = tld;
                return o;
            };
            const DirEval eL = eval_dir(-1);
            const DirEval eR = eval_dir(+1);
            // randomized decision
            const float uLp = fmaxf(0.0f, eL.u), uRp = fmaxf(0.0f, eR.u);
            const float uT = uLp + uRp;
            const float pLC = uT >= 1.0f ? P.p_max : (uT > 0.0f ? P.p_min + (P.p_max - P.p_min) * uT : P.p_min);
            const uint32_t w = philox_word0(P.key0, P.key1, (uint32_t)rec.vid, (uint32_t)t);
            const float rr = (float)w * 2.3283064365386963e-10f;  // 2^-32
            int dec = 0;
            if (uT > 0.0f) {
                const float bL = pLC * uLp / uT;
                if (uLp > 0.0f && rr < bL) dec = 1;
                else if (uRp > 0.0f && rr >= bL && rr < pLC) dec = 2;
            } else {
                const bool fL = eL.u > -TS_INF, fR = eR.u > -TS_INF;
                if (fL && fR) {
                    if (rr < 0.5f * P.p_min) dec = 1;
                    else if (rr < P.p_min) dec = 2;
                } else if (fL || fR) {
                    if (rr < P.p_min) dec = fL ? 1 : 2;
                }
            }
            const int nli = dec == 1 ? li - 1 : (dec == 2 ? li + 1 : li);
            float a = dec == 1 ? eL.ta : (dec == 2 ? eR.ta : a_e);
            // cooperative yielding of lane keepers to vehicles merging into their lane
            bool has_y = false;
            float y_rear = TS_INF, y_v = 0.0f;
            if (!is_jl && !dec) {
                int y_vid = 0x7FFFFFFF;
                const int nm = S.nmerge;
                if (nm <= kMergeCap) {
                    for (int q = 0; q < nm; ++q) {
                        if (S.mrg_tgt[q] != li) continue;
                        const float rm = S.mrg_rear[q];
                        if (!(rm > rec.x)) continue;
                        if (!has_y || rm < y_rear || (rm == y_rear && S.mrg_vid[q] < y_vid)) {
                            has_y = true;
                            y_rear = rm;
                            y_v = S.mrg_v[q];
                            y_vid = S.mrg_vid[q];
                        }
                    }
                } else {
                    for (int dd = -1; dd <= 1; dd += 2) {
                        const int k2 = li + dd;
                        if (k2 < 0 || k2 >= nroad) continue;
                        for (int q = 0; q < S.cnt[k2]; ++q) {
                            const uint32_t s2 = S.base[k2] + q;
                            if (D.sh_merge[s2] != li) continue;
                            const VehRec z = rd[s2];
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
            float B = TS_INF, vcap = TS_INF;
            const float lr = D.sh_lrear[slot];
            if (lr < TS_INF) {
                B = lr;
                vcap = D.sh_lv[slot];
            }
            if (dec) {
                const Lead l2 = dec == 1 ? eL.lead : eR.lead;
                if (l2.ex) {
                    if (l2.rear < B) {
                        B = l2.rear;
                        vcap = l2.v;
                    } else if (l2.rear == B) {
                        vcap = fminf(vcap, l2.v);
                    }
                }
            }
            if (has_y) {
                if (y_rear < B) {
                    B = y_rear;
                    vcap = y_v;
                } else if (y_rear == B) {
                    vcap = fminf(vcap, y_v);
                }
            }
            const int mnew = S.lane[nli];
            if (stop_end(D, mnew, is_jl, rec.nr, true)) {
                if (len < B) {
                    B = len;
                    vcap = 0.0f;
                } else if (len == B) {
                    vcap = 0.0f;
                }
            }
            if (xn > B) {
                xn = fmaxf(B, x);
                vn = fminf(vn, vcap);
                atomicAdd(&S.clamps, 1);
            }
            int kind = dec ? 1 : 0;
            int tgt_local = nli;
            if (xn > len) {
                if (!is_jl && rec.rem == 0) {
                    kind = 4;
                    D.status[rec.vid] = 2;
                    D.finish_step[rec.vid] = (int)t;
                    const double tt = (double)(t + 1) * P.dt_d - (double)D.tau[rec.vid];
                    atomicAdd(&S.sum_tt, (unsigned long long)llrint(tt * kTimeFx));
                    atomicAdd(&S.finished, 1);
                } else if (!is_jl) {
                    const int g = out_toward(D, mnew, rec.nr);
                    kind = 2;
                    tgt_local = D.lane_local[g];
                    xn -= len;
                    atomicAdd(&S.transfers, 1);
                } else {
                    const int g = D.jl_out[m];
                    bool blocked = false;
                    const int my_ext = D.jl_ext[m];
                    for (int e = D.feed_begin[g]; e < D.feed_begin[g + 1]; ++e) {
                        const int fl = D.feed_jl[e];
                        if (D.jl_ext[fl] >= my_ext) break;
                        const int cf = rcnt[fl];
                        if (cf == 0) continue;
                        const VehRec h = rd[D.lane_base[fl]];
                        const float reach = h.x + h.v * P.dt + P.reach - D.lane_len[fl];
                        if (reach > 0.0f) blocked = true;
                    }
                    if (blocked) {
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
                        o.nr = rec.rem - 1 > 0 ? D.route[rec.rp + 2] : -1;
                        if (atomicCAS(&D.inbox_flag[g], 0, 1) != 0) atomicAdd(&S.errors, 1);
                        D.inbox[g] = o;
                        atomicAdd(&S.transfers, 1);
                    }
                }
            }
            if (dec) atomicAdd(&S.changes, 1);
            // metrics: a vehicle counts for the lane it occupied at the step start
            if (!is_jl) {
                atomicAdd(&S.sumv, (unsigned long long)(long long)llrintf(vn * kSpeedFx));
                atomicAdd(&S.cntv, 1);
            }
            if (vn < 0.1f) atomicAdd(&S.wait[li], 1);
            D.sh_nx[slot] = xn;
            D.sh_nv[slot] = vn;
            D.sh_kind[slot] = kind;
            D.sh_nlane[slot] = tgt_local;
            if (kind == 0) {
                atomicAdd(&S.nstay[li], 1);
            } else if (kind == 1) {
                atomicAdd(&S.nin[nli], 1);
                const int q = atomicAdd(&S.nchg, 1);
                if (q < kChangerCap) {
                    S.chg_x[q] = xn;
                    S.chg_vid[q] = rec.vid;
                    S.chg_lane[q] = nli;
                }
            } else if (kind == 2) {
                atomicAdd(&S.nenter[tgt_local], 1);
            }
        }
        __syncthreads();

        // ---------------- pass 3 ----------------
        // exclusive prefix count of stayers over the tile enumeration
        {
            int carry = 0;
            for (int b0 = 0; b0 < n; b0 += kWave) {
                const int j = b0 + tid;
                bool st = false;
                uint32_t slot = 0;
                if (j < n) {
                    const int li = lane_of(S, j);
                    slot = S.base[li] + (j - S.start[li]);
                    st = D.sh_kind[slot] == 0;
                }
                const unsigned long long bal = __ballot(st);
                const int pre = carry + __popcll(bal & ((1ull << tid) - 1ull));
                if (j < n) D.sh_pref[slot] = pre;
                carry += __popcll(bal);
            }
        }
        __syncthreads();
        const int nchg = S.nchg;
        for (int j = tid; j < n; j += kWave) {
            const int li = lane_of(S, j);
            const int c = j - S.start[li];
            const uint32_t slot = S.base[li] + c;
            const int kind = D.sh_kind[slot];
            if (kind >= 3) continue;
            const VehRec rec = rd[slot];
            const float xn = D.sh_nx[slot];
            const int nli = D.sh_nlane[slot];
            int rank = 0;
            if (kind == 0) {
                rank = D.sh_pref[slot] - D.sh_pref[S.base[li]];
            } else if (kind == 1) {
                for (int q = 0; q < S.cnt[nli]; ++q) {
                    const uint32_t s2 = S.base[nli] + q;
                    if (D.sh_kind[s2] != 0) continue;
                    if (ahead(D.sh_nx[s2], rd[s2].vid, xn, rec.vid)) rank++;
                }
            } else {
                rank = S.nstay[nli];
            }
            if (kind <= 1) {
                // changers into the same lane ahead of this vehicle
                if (nchg <= kChangerCap) {
                    for (int q = 0; q < nchg; ++q)
                        if (S.chg_lane[q] == nli && S.chg_vid[q] != rec.vid && ahead(S.chg_x[q], S.chg_vid[q], xn, rec.vid))
                            rank++;
                } else {
                    for (int dd = -1; dd <= 1; dd += 2) {
                        const int k2 = nli + dd;
                        if (k2 < 0 || k2 >= nroad) continue;
                        for (int q = 0; q < S.cnt[k2]; ++q) {
                            const uint32_t s2 = S.base[k2] + q;
                            if (D.sh_kind[s2] != 1 || D.sh_nlane[s2] != nli) continue;
                            const int ov = rd[s2].vid;
                            if (ov != rec.vid && ahead(D.sh_nx[s2], ov, xn, rec.vid)) rank++;
                        }
                    }
                }
            }
            const int mn = S.lane[nli];
            if (rank < D.lane_cap[mn]) {
                VehRec o = rec;
                o.x = xn;
                o.v = D.sh_nv[slot];
                wr[S.base[nli] + rank] = o;
            } else {
                atomicAdd(&S.errors, 1);
            }
        }
        __syncthreads();
        if (tid < nl) {
            const int m = lb + tid;
            const int c = S.nstay[tid] + S.nin[tid] + S.nenter[tid];
            wcnt[m] = c < D.lane_cap[m] ? c : D.lane_cap[m];
            D.lane_wait[m] = S.wait[tid];
        }
        if (tid == 0) {
            D.road_speed[r] = S.cntv > 0 ? (float)((double)(long long)S.sumv / (double)kSpeedFx / (double)S.cntv) : -1.0f;
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
        }
        __syncthreads();
    }

    // per-workgroup partials; the last workgroup folds the step
    if (tid == 0) {
        D.part[blockIdx.x] = acc;
        __threadfence();
        const unsigned int old = atomicAdd(D.done_ctr, 1u);
        S.n = (old == gridDim.x - 1) ? 1 : 0;
    }
    __syncthreads();
    if (S.n) {
        __threadfence();
        long long a[10] = {0, 0, 0, 0, 0, 0, 0, 0, 0, 0};
        for (int g = tid; g < (int)gridDim.x; g += kWave) {
            const volatile long long* q = (const volatile long long*)&D.part[g];
            for (int k = 0; k < 10; ++k) a[k] += q[k];
        }
        for (int k = 0; k < 10; ++k) {
            for (int off = 32; off > 0; off >>= 1) a[k] += __shfl_down(a[k], off);
        }
        if (tid == 0) {
            DevMetrics* M = D.met;
            M->vehicle_steps += a[2];
            M->lane_changes += a[3];
            M->transfers += a[4];
            M->clamps += a[5];
            M->feeder_blocks += a[6];
            M->finished += a[7];
            M->sum_tt_fx += a[8];
            M->errors += a[9];
            if (a[1] > 0) {
                M->mean_speed_last = (double)a[0] / (double)kSpeedFx / (double)a[1];
                M->speed_acc += M->mean_speed_last;
                M->speed_steps += 1;
            } else {
                M->mean_speed_last = 0.0;
            }
            M->step = t + 1;
            *D.done_ctr = 0u;
        }
    }
}

// ---------------------------------------------------------------------------
// host-driven helpers
// ---------------------------------------------------------------------------
__global__ void k_set_phases(DevNet D, const int32_t* ids, const int32_t* ph, int n)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    D.junc_policy[ids[i]] = 2;
    D.junc_manual[ids[i]] = ph[i];
}

// per-vehicle export of the state at a step boundary (residents + inboxes)
__global__ void k_export(DevNet D, const int32_t* lane_ext, int32_t* o_lane, float* o_x, float* o_v, int32_t* o_rpos,
                         int32_t* o_rank)
{
    const int m = blockIdx.x * blockDim.x + threadIdx.x;
    if (m >= D.NL) return;
    const long long t = D.met->step;
    const int p = (int)(t & 1);
    const VehRec* slab = p ? D.slab1 : D.slab0;
    const int32_t* cnt = p ? D.cnt1 : D.cnt0;
    const int c = cnt[m];
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

// scatter of host-ordered records into the read slab of the current step
__global__ void k_import(DevNet D, const uint32_t* slots, const VehRec* recs, int n)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const long long t = D.met->step;
    VehRec* slab = (t & 1) ? D.slab1 : D.slab0;
    slab[slots[i]] = recs[i];
}

// launch wrappers (host side)
hipError_t launch_prepare(const DevNet& D, hipStream_t s)
{
    const int n = D.R > D.NJ ? D.R : D.NJ;
    hipLaunchKernelGGL(k_prepare, dim3((n + 255) / 256), dim3(256), 0, s, D);
    return hipGetLastError();
}

hipError_t launch_update(const DevNet& D, hipStream_t s)
{
    hipLaunchKernelGGL(k_update, dim3(D.G), dim3(kWave), 0, s, D);
    return hipGetLastError();
}

hipError_t launch_set_phases(const DevNet& D, const int32_t* ids, const int32_t* ph, int n, hipStream_t s)
{
    hipLaunchKernelGGL(k_set_phases, dim3((n + 255) / 256), dim3(256), 0, s, D, ids, ph, n);
    return hipGetLastError();
}

hipError_t launch_export(const DevNet& D, const int32_t* lane_ext, int32_t* o_lane, float* o_x, float* o_v,
                         int32_t* o_rpos, int32_t* o_rank, hipStream_t s)
{
    hipLaunchKernelGGL(k_export, dim3((D.NL + 255) / 256), dim3(256), 0, s, D, lane_ext, o_lane, o_x, o_v, o_rpos,
                       o_rank);
    return hipGetLastError();
}

hipError_t launch_import(const DevNet& D, const uint32_t* slots, const VehRec* recs, int n, hipStream_t s)
{
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_import, dim3((n + 255) / 256), dim3(256), 0, s, D, slots, recs, n);
    return hipGetLastError();
}

}  // namespace tsim
