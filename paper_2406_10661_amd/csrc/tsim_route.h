// Shortest routes on the device: the movement graph the host gathers from a
// network (values only; every cost is computed by the kernels) and the
// driver that runs the route kernels over a caller's workspace.
#pragma once
#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>
#include <string>
#include <vector>

namespace tsim {

// Largest network the route kernels take: the cost-to-go of every road is
// held in LDS (4 bytes per road) by the workgroup of one destination.
constexpr int kRouteMaxRoads = 32768;

// Movement graph with local road ids 0..R-1.  A movement r -> b exists when
// an open junction lane leads from a lane of r into a lane of b; its
// junction lanes' lengths and limits are listed for the kernels to take the
// fastest.  Road travel time: the road's length over the highest limit of
// its lanes.
struct RouteGraph {
    int R = 0;
    std::vector<int32_t> road_lane_begin;  // [R+1] CSR into lane_lim
    std::vector<float> road_len;           // [R] metres
    std::vector<float> lane_lim;           // road lanes' limits, m/s
    std::vector<int32_t> e_begin;          // [R+1] movements leaving road r
    std::vector<int32_t> e_to;             // [E] target road, ascending within a road
    std::vector<int32_t> e_jl_begin;       // [E+1] CSR into jl_len / jl_lim
    std::vector<float> jl_len, jl_lim;     // junction lanes of each movement
};

// Workspace a call needs at least, and the size that routes n pairs with
// few passes.
size_t route_workspace_min(const RouteGraph& G, long long n);
size_t route_workspace_hint(const RouteGraph& G, long long n);

// Where the routes go: room for `total` road ids, or null when the caller
// cannot hold them.
struct RouteSink {
    virtual int32_t* reserve(int64_t total) = 0;
    virtual ~RouteSink() = default;
};

struct VectorSink : RouteSink {
    std::vector<int32_t> roads;
    int32_t* reserve(int64_t total) override
    {
        roads.resize((size_t)total);
        return roads.data();
    }
};

// Routes for n (origin, destination) pairs of local road ids under prices
// price[R] and road times road_time[R] (either may be null): begin[n+1] (CSR
// in the callers' order) and the roads written to sink.reserve(begin[n])
// (origin first, destination last, empty when unreachable).  Returns a
// TSIM_* status (message in *err; TSIM_ENOMEM with begin filled when the
// sink has no room); synchronises the stream.
int route_pairs(const RouteGraph& G, const float* price, const float* road_time, const int32_t* origin,
                const int32_t* dest, int n, hipStream_t stream, void* ws, size_t ws_bytes,
                std::vector<int64_t>& begin, RouteSink& sink, int* n_unreachable, std::string* err);

}  // namespace tsim
