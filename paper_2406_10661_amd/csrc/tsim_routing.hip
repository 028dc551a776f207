// Shortest routes on the device for congestion pricing (Section 4
// "Congestion Pricing": once roads carry prices, drivers move to routes of
// lower cost; Appendix F: every road may be priced, prices change every
// 20 s; Appendix E: demand routed by shortest travel time).
//
// Cost of a route: over every road after its first, the fastest open
// junction lane into it (length / limit), plus the road's travel time (its
// length over the highest limit of its lanes, or a time the caller gives),
// plus its price, in FP32.  The cost-to-go of a road is its movement cost
// plus the cost-to-go of the road the movement enters; of successors with
// equal candidate cost the smaller road id is taken.
//
// Kernels:
//   k_route_weights   one thread per movement: the movement's cost.
//   k_route_tree_reg  networks of at most 16,384 movements: one workgroup
//                     per group of up to 16 destinations, the movements
//                     held in registers, every destination's cost-to-go in
//                     LDS; Bellman-Ford sweeps relax every movement with an
//                     LDS atomic minimum until a sweep changes nothing, then
//                     each road's next road toward each destination.
//   k_route_tree      larger networks: one workgroup per destination, the
//                     movements read from memory, each road relaxed from its
//                     successors.
//   k_route_walk      one thread per pair: follows the next roads from the
//                     origin, first counting, then writing the route.
// The costs are non-negative and the candidate sum is monotone, so any order
// of relaxations from +inf settles on the same least costs as Dijkstra's
// order, bit for bit.
#include <algorithm>
#include <cmath>
#include <limits>
#include <numeric>

#include "../../include/tsim.h"
#include "tsim_internal.h"
#include "tsim_route.h"

namespace tsim {

namespace {

constexpr int kTreeThreads = 256;
constexpr int kWalkThreads = 256;

struct RouteDev {
    int R, E;
    const int32_t* road_lane_begin;
    const float* road_len;
    const float* lane_lim;
    const int32_t* e_begin;
    const int32_t* e_to;
    const int32_t* e_jl_begin;
    const float* jl_len;
    const float* jl_lim;
    const float* price;      // or null
    const float* road_time;  // or null
    float* w;                // [E] movement costs
};

__global__ __launch_bounds__(256) void k_route_weights(RouteDev G)
{
    const int e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= G.E) return;
    const int b = G.e_to[e];
    float t;
    if (G.road_time) {
        t = G.road_time[b];
    } else {
        float vmax = 0.0f;
        for (int l = G.road_lane_begin[b]; l < G.road_lane_begin[b + 1]; ++l) vmax = fmaxf(vmax, G.lane_lim[l]);
        t = G.road_len[b] / vmax;
    }
    const int q0 = G.e_jl_begin[e], q1 = G.e_jl_begin[e + 1];
    float c = G.jl_len[q0] / G.jl_lim[q0];
    for (int q = q0 + 1; q < q1; ++q) c = fminf(c, G.jl_len[q] / G.jl_lim[q]);
    float w = c + t;
    w = w + (G.price ? G.price[b] : 0.0f);
    G.w[e] = w;
}

__global__ __launch_bounds__(kTreeThreads) void k_route_tree(RouteDev G, const int32_t* dests, int32_t* nxt)
{
    extern __shared__ float dist[];
    const int R = G.R, d = dests[blockIdx.x];
    for (int r = threadIdx.x; r < R; r += kTreeThreads) dist[r] = r == d ? 0.0f : INFINITY;
    __syncthreads();
    for (;;) {
        int changed = 0;
        for (int r = threadIdx.x; r < R; r += kTreeThreads) {
            if (r == d) continue;
            const int e0 = G.e_begin[r], e1 = G.e_begin[r + 1];
            const float cur = dist[r];
            float best = cur;
            for (int e = e0; e < e1; ++e) {
                const float c = G.w[e] + dist[G.e_to[e]];
                best = c < best ? c : best;
            }
            if (best < cur) {
                dist[r] = best;
                changed = 1;
            }
        }
        if (!__syncthreads_or(changed)) break;
    }
    int32_t* out = nxt + (size_t)blockIdx.x * R;
    for (int r = threadIdx.x; r < R; r += kTreeThreads) {
        int nx = -1;
        if (r == d) {
            nx = d;
        } else if (dist[r] < INFINITY) {
            float best = INFINITY;
            for (int e = G.e_begin[r]; e < G.e_begin[r + 1]; ++e) {
                const int b = G.e_to[e];
                const float c = G.w[e] + dist[b];
                if (c < best) {
                    best = c;
                    nx = b;
                }
            }
        }
        out[r] = nx;
    }
}

// k_route_tree for networks of at most kRegMoves movements: each of the
// workgroup's 1024 threads holds up to EPT movements (source road, target
// road, cost) in registers for the whole kernel, and the cost-to-go of K
// destinations lives in LDS; a sweep relaxes every movement for every
// destination that changed in the sweep before, lowering the source road's
// cost with an LDS atomic minimum (non-negative floats order as their bit
// patterns).
constexpr int kRegThreads = 1024;
constexpr int kRegMaxK = 16;
constexpr int kRegMoves = 16 * kRegThreads;

template <int EPT>
__global__ __launch_bounds__(kRegThreads) void k_route_tree_reg(RouteDev G, const int32_t* e_from,
                                                                const int32_t* dests, int nd, int K, int32_t* nxt)
{
    extern __shared__ float dist[];   // [K][R]
    __shared__ int chg[2][kRegMaxK];  // destinations changed in the last sweep / this sweep
    const int R = G.R, E = G.E, tid = threadIdx.x;
    int fr[EPT], to[EPT];
    float w[EPT];
#pragma unroll
    for (int j = 0; j < EPT; ++j) {
        const int e = tid + j * kRegThreads;
        const bool ok = e < E;
        fr[j] = ok ? e_from[e] : -1;
        to[j] = ok ? G.e_to[e] : 0;
        w[j] = ok ? G.w[e] : 0.0f;
    }
    const int base = blockIdx.x * K;
    const int nk = min(K, nd - base);
    for (int i = tid; i < nk * R; i += kRegThreads) {
        const int k = i / R, r = i - k * R;
        dist[i] = r == dests[base + k] ? 0.0f : INFINITY;
    }
    if (tid < kRegMaxK) {
        chg[0][tid] = 1;
        chg[1][tid] = 0;
    }
    __syncthreads();
    for (int sweep = 0;; ++sweep) {
        const int cur = sweep & 1;
        for (int k = 0; k < nk; ++k) {
            if (!chg[cur][k]) continue;
            float* dk = dist + (size_t)k * R;
            int changed = 0;
#pragma unroll
            for (int j = 0; j < EPT; ++j) {
                if (fr[j] < 0) continue;
                const float c = w[j] + dk[to[j]];
                if (c < dk[fr[j]]) {
                    const int old = atomicMin((int*)(dk + fr[j]), __float_as_int(c));
                    changed |= __int_as_float(old) > c;
                }
            }
            if (changed) chg[cur ^ 1][k] = 1;
        }
        __syncthreads();
        if (tid < kRegMaxK) chg[cur][tid] = 0;
        int any = 0;
        for (int k = 0; k < nk; ++k) any |= chg[cur ^ 1][k];
        if (!__syncthreads_or(any)) break;
    }
    // each road's next road toward each destination
    for (int i = tid; i < nk * R; i += kRegThreads) {
        const int k = i / R, r = i - k * R, d = dests[base + k];
        const float* dk = dist + (size_t)k * R;
        int nx = -1;
        if (r == d) {
            nx = d;
        } else if (dk[r] < INFINITY) {
            float best = INFINITY;
            for (int e = G.e_begin[r]; e < G.e_begin[r + 1]; ++e) {
                const int b = G.e_to[e];
                const float c = G.w[e] + dk[b];
                if (c < best) {
                    best = c;
                    nx = b;
                }
            }
        }
        nxt[(size_t)(base + k) * R + r] = nx;
    }
}

// pairs p of one chunk (pointers already offset to the chunk's first pair);
// pud[p] - c0 is the pair's destination slot in nxt.  write = 0: plen[p] =
// roads of the route (0: unreachable, or longer than the network has
// roads); write = 1: the route of every pair with plen[p] > 0 to
// stage[poff[p] ..].
__global__ __launch_bounds__(kWalkThreads) void k_route_walk(const int32_t* nxt, int R, int c0, const int32_t* porig,
                                                              const int32_t* pdest, const int32_t* pud, int np,
                                                              int32_t* plen, const int32_t* poff, int32_t* stage,
                                                              int write)
{
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= np) return;
    if (write && plen[p] == 0) return;
    const int32_t* nx = nxt + (size_t)(pud[p] - c0) * R;
    const int d = pdest[p];
    int r = porig[p], len = 0;
    int32_t* o = write ? stage + poff[p] : nullptr;
    if (nx[r] >= 0) {
        for (;;) {
            if (len >= R || r < 0) {
                len = 0;
                break;
            }
            if (write) o[len] = r;
            ++len;
            if (r == d) break;
            r = nx[r];
        }
    }
    if (!write) plen[p] = len;
}

constexpr size_t kAlign = 256;

size_t up_align(size_t x) { return (x + kAlign - 1) / kAlign * kAlign; }

struct Layout {
    size_t rlb, rlen, llim, eb, eto, efr, ejb, jlen, jlim, price, time, w, porig, pdest, pud, plen, poff, dests, nxt,
        stage;
    size_t fixed;   // bytes before nxt
    int C = 0;      // destinations per pass
    long long S = 0;  // staging entries
};

Layout fixed_layout(const RouteGraph& G, long long n)
{
    const size_t R = G.R, L = G.lane_lim.size(), E = G.e_to.size(), J = G.jl_len.size();
    Layout y{};
    size_t o = 0;
    auto take = [&](size_t bytes) {
        const size_t at = o;
        o = up_align(o + std::max<size_t>(bytes, 4));
        return at;
    };
    y.rlb = take((R + 1) * 4);
    y.rlen = take(R * 4);
    y.llim = take(L * 4);
    y.eb = take((R + 1) * 4);
    y.eto = take(E * 4);
    y.efr = take(E * 4);
    y.ejb = take((E + 1) * 4);
    y.jlen = take(J * 4);
    y.jlim = take(J * 4);
    y.price = take(R * 4);
    y.time = take(R * 4);
    y.w = take(E * 4);
    y.porig = take((size_t)n * 4);
    y.pdest = take((size_t)n * 4);
    y.pud = take((size_t)n * 4);
    y.plen = take((size_t)n * 4);
    y.poff = take((size_t)n * 4);
    y.dests = take(std::min<size_t>((size_t)std::max<long long>(n, 1), R) * 4);
    y.fixed = o;
    return y;
}

// nxt for C destinations, then S staging entries
size_t tail_bytes(const RouteGraph& G, int C, long long S)
{
    return up_align((size_t)C * G.R * 4) + (size_t)S * 4;
}

// New routes of vehicles at a step boundary: n_rp[i] >= 0 marks vehicle i,
// whose record (a lane resident, an inbox entrant, or, while it waits, its
// departure queue entry) takes route position n_rp[i], n_rem[i] roads after
// it and next-road word n_nr[i]; a waiting vehicle's queue entry also takes
// the departure lane mask n_mask[i].  One thread per lane, then one per
// queue entry.
__global__ void k_apply_routes(const DevNet D, const int32_t* n_rp, const int32_t* n_rem, const int32_t* n_nr,
                               const uint32_t* n_mask, int n_queue)
{
    const int id = blockIdx.x * blockDim.x + threadIdx.x;
    if (id < D.NL) {
        const int m = id;
        const long long t = *D.gstep;
        const int inst = D.tile_inst[D.lane_tile[m]];
        const long long t0 = D.inst_t0[inst], loc = t - t0, end = D.inst_end[inst];
        const int p = (int)((t0 + (loc < end ? loc : end)) & 1);
        VehRec* slab = (p ? D.slab1 : D.slab0) + D.lane_base[m];
        const int c = (p ? D.sum1 : D.sum0)[m].cnt;
        for (int q = 0; q <= c; ++q) {
            VehRec* z = q < c ? slab + q : (D.inbox_flag[m] ? D.inbox + m : nullptr);
            if (!z) break;
            const int i = z->vid;
            if (n_rp[i] >= 0) {
                z->rp = n_rp[i];
                z->rem = n_rem[i];
                z->nr = n_nr[i];
            }
        }
        return;
    }
    const int e = id - D.NL;
    if (e >= n_queue) return;
    QRec* r = const_cast<QRec*>(D.q_rec) + e;
    const int i = r->vid;
    if (n_rp[i] < 0 || D.status[i] != TSIM_WAITING) return;
    r->rp = n_rp[i];
    r->rem = n_rem[i];
    r->nr = n_nr[i];
    r->mask = n_mask[i];
}

}  // namespace

hipError_t launch_apply_routes(const DevNet& H, const int32_t* n_rp, const int32_t* n_rem, const int32_t* n_nr,
                               const uint32_t* n_mask, int n_queue, hipStream_t s)
{
    const int n = H.NL + n_queue;
    if (n > 0) k_apply_routes<<<(n + 255) / 256, 256, 0, s>>>(H, n_rp, n_rem, n_nr, n_mask, n_queue);
    return hipGetLastError();
}

size_t route_workspace_min(const RouteGraph& G, long long n)
{
    return fixed_layout(G, n).fixed + tail_bytes(G, 1, G.R);
}

size_t route_workspace_hint(const RouteGraph& G, long long n)
{
    const long long R = std::max(G.R, 1);
    const long long nd = std::max<long long>(1, std::min<long long>(n, R));
    const int C = (int)std::min<long long>(nd, std::max<long long>(1, (64ll << 20) / (4 * R)));
    const long long S = std::max<long long>(R, std::min<long long>({n * R, std::max<long long>(R, n * 64), 1ll << 24}));
    return fixed_layout(G, n).fixed + tail_bytes(G, C, S);
}

#define RCHK(call)                                                                        \
    do {                                                                                  \
        hipError_t e_ = (call);                                                           \
        if (e_ != hipSuccess) {                                                           \
            *err = std::string("HIP error in route kernels: ") + hipGetErrorString(e_);   \
            return TSIM_EDEVICE;                                                          \
        }                                                                                 \
    } while (0)

int route_pairs(const RouteGraph& G, const float* price, const float* road_time, const int32_t* origin,
                const int32_t* dest, int n, hipStream_t stream, void* ws, size_t ws_bytes,
                std::vector<int64_t>& begin, RouteSink& sink, int* n_unreachable, std::string* err)
{
    const int R = G.R;
    const int E = (int)G.e_to.size();
    if (n < 0 || (n > 0 && (!origin || !dest))) {
        *err = "bad pair arrays";
        return TSIM_EINVAL;
    }
    if (R < 1 || R > kRouteMaxRoads) {
        *err = "the network has no roads or more than the route kernels take (32768)";
        return TSIM_EINVAL;
    }
    for (int p = 0; p < n; ++p)
        if (origin[p] < 0 || origin[p] >= R || dest[p] < 0 || dest[p] >= R) {
            *err = "road id of a pair out of range";
            return TSIM_EINVAL;
        }
    for (int r = 0; r < R; ++r)
        if ((price && !(price[r] >= 0.0f)) || (road_time && !(road_time[r] >= 0.0f))) {
            *err = "prices and road times must be non-negative";
            return TSIM_EINVAL;
        }
    begin.assign((size_t)n + 1, 0);
    if (n_unreachable) *n_unreachable = 0;
    if (n == 0) return TSIM_OK;
    Layout y = fixed_layout(G, n);
    if (!ws || ws_bytes < y.fixed + tail_bytes(G, 1, R)) {
        *err = "route workspace too small";
        return TSIM_ENOMEM;
    }
    // pairs by destination (counting sort, stable), distinct destinations
    // in increasing id
    std::vector<int32_t> order(n), at_d((size_t)R + 1, 0);
    for (int p = 0; p < n; ++p) ++at_d[dest[p] + 1];
    for (int r = 0; r < R; ++r) at_d[r + 1] += at_d[r];
    for (int p = 0; p < n; ++p) order[at_d[dest[p]]++] = p;
    std::vector<int32_t> so(n), sd(n), sud(n), ud;
    for (int c = 0; c < n; ++c) {
        const int p = order[c];
        so[c] = origin[p];
        sd[c] = dest[p];
        if (ud.empty() || ud.back() != dest[p]) ud.push_back(dest[p]);
        sud[c] = (int32_t)ud.size() - 1;
    }
    const int nud = (int)ud.size();
    // destinations per pass from what is left, at least R staging entries
    const size_t left = ws_bytes - y.fixed;
    long long C = std::min<long long>(nud, (long long)((left - (size_t)R * 4 - kAlign) / ((size_t)R * 4)));
    if (C < 1) C = 1;
    y.C = (int)C;
    y.nxt = y.fixed;
    y.stage = y.nxt + up_align((size_t)C * R * 4);
    y.S = std::min<long long>((long long)((ws_bytes - y.stage) / 4), std::numeric_limits<int32_t>::max());

    char* base = (char*)ws;
    auto at = [&](size_t off) { return (void*)(base + off); };
    auto put = [&](size_t off, const void* src, size_t bytes) {
        return bytes ? hipMemcpyAsync(at(off), src, bytes, hipMemcpyHostToDevice, stream) : hipSuccess;
    };
    RCHK(put(y.rlb, G.road_lane_begin.data(), G.road_lane_begin.size() * 4));
    RCHK(put(y.rlen, G.road_len.data(), G.road_len.size() * 4));
    RCHK(put(y.llim, G.lane_lim.data(), G.lane_lim.size() * 4));
    RCHK(put(y.eb, G.e_begin.data(), G.e_begin.size() * 4));
    RCHK(put(y.eto, G.e_to.data(), G.e_to.size() * 4));
    RCHK(put(y.ejb, G.e_jl_begin.data(), G.e_jl_begin.size() * 4));
    RCHK(put(y.jlen, G.jl_len.data(), G.jl_len.size() * 4));
    RCHK(put(y.jlim, G.jl_lim.data(), G.jl_lim.size() * 4));
    if (price) RCHK(put(y.price, price, (size_t)R * 4));
    if (road_time) RCHK(put(y.time, road_time, (size_t)R * 4));
    RCHK(put(y.porig, so.data(), (size_t)n * 4));
    RCHK(put(y.pdest, sd.data(), (size_t)n * 4));
    RCHK(put(y.pud, sud.data(), (size_t)n * 4));

    RouteDev D;
    D.R = R;
    D.E = E;
    D.road_lane_begin = (const int32_t*)at(y.rlb);
    D.road_len = (const float*)at(y.rlen);
    D.lane_lim = (const float*)at(y.llim);
    D.e_begin = (const int32_t*)at(y.eb);
    D.e_to = (const int32_t*)at(y.eto);
    D.e_jl_begin = (const int32_t*)at(y.ejb);
    D.jl_len = (const float*)at(y.jlen);
    D.jl_lim = (const float*)at(y.jlim);
    D.price = price ? (const float*)at(y.price) : nullptr;
    D.road_time = road_time ? (const float*)at(y.time) : nullptr;
    D.w = (float*)at(y.w);
    if (E > 0) {
        k_route_weights<<<(E + 255) / 256, 256, 0, stream>>>(D);
        RCHK(hipGetLastError());
    }
    // the tree kernel: movements held in registers with up to 16
    // destinations per workgroup (enough workgroups to cover the GPU twice)
    // when there are at most kRegMoves of them, else read from memory with
    // one destination per workgroup
    int dev = 0, lds_max = 0, n_cu = 0;
    RCHK(hipGetDevice(&dev));
    if (hipDeviceGetAttribute(&lds_max, hipDeviceAttributeSharedMemPerBlockOptin, dev) != hipSuccess || lds_max <= 0)
        RCHK(hipDeviceGetAttribute(&lds_max, hipDeviceAttributeMaxSharedMemoryPerBlock, dev));
    RCHK(hipDeviceGetAttribute(&n_cu, hipDeviceAttributeMultiprocessorCount, dev));
    const int ept = (E + kRegThreads - 1) / kRegThreads;
    int K = 0;
    if (E <= kRegMoves) {
        const long long fit = std::min<long long>(kRegMaxK, (long long)(lds_max - 256) / ((long long)R * 4));
        const long long want = (std::min<long long>(C, nud) + 2LL * std::max(n_cu, 1) - 1) / (2LL * std::max(n_cu, 1));
        K = (int)std::max<long long>(0, std::min(fit, std::max<long long>(want, 1)));
    }
    const size_t lds = K ? (size_t)K * R * 4 : (size_t)R * 4;
    if (lds > (size_t)lds_max) {
        *err = "the network's cost-to-go does not fit in LDS";
        return TSIM_EINVAL;
    }
    auto reg_kernel = [&]() -> const void* {
        if (ept <= 4) return (const void*)k_route_tree_reg<4>;
        if (ept <= 8) return (const void*)k_route_tree_reg<8>;
        return (const void*)k_route_tree_reg<16>;
    };
    RCHK(hipFuncSetAttribute(K ? reg_kernel() : (const void*)k_route_tree, hipFuncAttributeMaxDynamicSharedMemorySize,
                             (int)lds));
    std::vector<int32_t> e_from(E);
    for (int r = 0; r < R; ++r)
        for (int e = G.e_begin[r]; e < G.e_begin[r + 1]; ++e) e_from[e] = r;
    RCHK(put(y.efr, e_from.data(), (size_t)E * 4));
    const int32_t* d_efr = (const int32_t*)at(y.efr);

    int32_t* nxt = (int32_t*)at(y.nxt);
    int32_t* stage = (int32_t*)at(y.stage);
    int32_t* d_plen = (int32_t*)at(y.plen);
    int32_t* d_poff = (int32_t*)at(y.poff);
    const int32_t* d_po = (const int32_t*)at(y.porig);
    const int32_t* d_pd = (const int32_t*)at(y.pdest);
    const int32_t* d_pu = (const int32_t*)at(y.pud);
    // chunks of C destinations and their pairs (contiguous in sorted order)
    const int n_chunks = (int)((nud + C - 1) / C);
    std::vector<int> chunk_pa(n_chunks + 1, n);
    for (int c = n - 1; c >= 0; --c) chunk_pa[sud[c] / C] = c;
    for (int k = n_chunks - 1; k >= 0; --k) chunk_pa[k] = std::min(chunk_pa[k], chunk_pa[k + 1]);
    auto tree = [&](int k) {
        const int c0 = (int)(k * C), c1 = (int)std::min<long long>(nud, c0 + C);
        RCHK(put(y.dests, ud.data() + c0, (size_t)(c1 - c0) * 4));
        const int32_t* dd = (const int32_t*)at(y.dests);
        const int nwg = K ? (c1 - c0 + K - 1) / K : 0;
        if (K && ept <= 4)
            k_route_tree_reg<4><<<nwg, kRegThreads, lds, stream>>>(D, d_efr, dd, c1 - c0, K, nxt);
        else if (K && ept <= 8)
            k_route_tree_reg<8><<<nwg, kRegThreads, lds, stream>>>(D, d_efr, dd, c1 - c0, K, nxt);
        else if (K)
            k_route_tree_reg<16><<<nwg, kRegThreads, lds, stream>>>(D, d_efr, dd, c1 - c0, K, nxt);
        else
            k_route_tree<<<c1 - c0, kTreeThreads, lds, stream>>>(D, (const int32_t*)at(y.dests), nxt);
        RCHK(hipGetLastError());
        return TSIM_OK;
    };
    auto walk = [&](int k, int q0, int q1, int write) {
        const int np = q1 - q0;
        if (np <= 0) return TSIM_OK;
        k_route_walk<<<(np + kWalkThreads - 1) / kWalkThreads, kWalkThreads, 0, stream>>>(
            nxt, R, (int)(k * C), d_po + q0, d_pd + q0, d_pu + q0, np, d_plen + q0, d_poff + q0, stage, write);
        RCHK(hipGetLastError());
        return TSIM_OK;
    };
    // pass 1: each chunk's cost-to-go trees, then the lengths of its routes
    for (int k = 0; k < n_chunks; ++k) {
        int rc = tree(k);
        if (!rc) rc = walk(k, chunk_pa[k], chunk_pa[k + 1], 0);
        if (rc) return rc;
    }
    std::vector<int32_t> hlen(n);
    RCHK(hipMemcpyAsync(hlen.data(), d_plen, (size_t)n * 4, hipMemcpyDeviceToHost, stream));
    RCHK(hipStreamSynchronize(stream));
    int bad = 0;
    for (int c = 0; c < n; ++c) {
        begin[(size_t)order[c] + 1] = hlen[c];
        bad += hlen[c] == 0;
    }
    for (int p = 0; p < n; ++p) begin[p + 1] += begin[p];
    if (n_unreachable) *n_unreachable = bad;
    const int64_t total = begin[n];
    int32_t* out = sink.reserve(total);
    if (!out && total > 0) {
        *err = "no room for the routes (" + std::to_string(total) + " roads)";
        return TSIM_ENOMEM;
    }
    if (total == 0) return TSIM_OK;
    // pass 2: the routes, the last chunk first (its trees are still in
    // place), every other chunk's trees computed again
    std::vector<int32_t> hoff(n);
    if (total <= y.S) {
        // every route written at its place in the callers' order: one copy
        for (int c = 0; c < n; ++c) hoff[c] = (int32_t)begin[order[c]];
        RCHK(put(y.poff, hoff.data(), (size_t)n * 4));
        for (int k = n_chunks - 1; k >= 0; --k) {
            int rc = k == n_chunks - 1 ? TSIM_OK : tree(k);
            if (!rc) rc = walk(k, chunk_pa[k], chunk_pa[k + 1], 1);
            if (rc) return rc;
        }
        RCHK(hipMemcpyAsync(out, stage, (size_t)total * 4, hipMemcpyDeviceToHost, stream));
        RCHK(hipStreamSynchronize(stream));
        return TSIM_OK;
    }
    // the staging buffer holds part of the routes: batches of pairs, each
    // copied down and placed
    std::vector<int32_t> tmp;
    for (int k = n_chunks - 1; k >= 0; --k) {
        if (k != n_chunks - 1) {
            const int rc = tree(k);
            if (rc) return rc;
        }
        int q = chunk_pa[k];
        while (q < chunk_pa[k + 1]) {
            long long used = 0;
            int q2 = q;
            while (q2 < chunk_pa[k + 1] && used + hlen[q2] <= y.S) {
                hoff[q2] = (int32_t)used;
                used += hlen[q2];
                ++q2;
            }
            RCHK(put(y.poff + (size_t)q * 4, hoff.data() + q, (size_t)(q2 - q) * 4));
            const int rc = walk(k, q, q2, 1);
            if (rc) return rc;
            tmp.resize((size_t)used);
            if (used)
                RCHK(hipMemcpyAsync(tmp.data(), stage, (size_t)used * 4, hipMemcpyDeviceToHost, stream));
            RCHK(hipStreamSynchronize(stream));
            for (int c = q; c < q2; ++c)
                std::copy(tmp.begin() + hoff[c], tmp.begin() + hoff[c] + hlen[c], out + begin[order[c]]);
            q = q2;
        }
    }
    return TSIM_OK;
}

}  // namespace tsim
