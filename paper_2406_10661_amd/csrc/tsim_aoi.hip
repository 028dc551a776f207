// Areas of interest on the device: occupancy counts of the AOIs where trips
// start and end (Appendix B.1: an AOI is an area with connections to the
// road network; Appendix B.2: it holds the vehicles whose trips start there
// until they depart and takes in those whose trips end there).  Launched on
// demand between steps, never inside a step.
#include "tsim_internal.h"

namespace tsim {

// one thread per vehicle of the range [v0, v0 + nv) (an instance's);
// counts[a] the waiting vehicles of origin AOI a, counts[n_aoi + a] the
// finished ones of destination AOI a (counts cleared by the caller; AOI ids
// indexed from v0, < 0: none)
__global__ void k_aoi_counts(const DevNet D, int v0, int nv, const int32_t* origin, const int32_t* dest, int n_aoi,
                             int32_t* counts)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= nv) return;
    const int st = D.status[v0 + i];
    const int o = origin[i], d = dest[i];
    if (st == 0 && o >= 0) atomicAdd(&counts[o], 1);
    if (st == 2 && d >= 0) atomicAdd(&counts[n_aoi + d], 1);
}

hipError_t launch_aoi_counts(const DevNet& H, int v0, int nv, const int32_t* origin, const int32_t* dest, int n_aoi,
                             int32_t* counts, hipStream_t s)
{
    if (nv > 0)
        hipLaunchKernelGGL(k_aoi_counts, dim3((nv + 255) / 256), dim3(256), 0, s, H, v0, nv, origin, dest, n_aoi,
                           counts);
    return hipGetLastError();
}

}  // namespace tsim
