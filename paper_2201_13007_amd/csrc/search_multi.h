// The general search kernel, one wavefront per worker (see search_body.h): every case
// with two or more workers, and one worker with an LDS visited table.
#pragma once
#include "search_body.h"

#include <atomic>

namespace sa {
namespace search_detail {

// workgroup b runs job b in workspace region b.  Up to two queue slots per lane the gather
// passes take two vectors per lane group: sixteen registers more, which stay within the 128
// of a 1024-lane workgroup without scratch there (not at four lanes per vector, nor at four
// slots, where the compiler spills); +5% at M = 4 and 8, L = 128, on 1M SIFT-shaped rows.
template <int LPV, int NI, int DT>
__global__ void __launch_bounds__(1024) search_multi(KArgs A)
{
    search_body<LPV, NI, DT, NI <= 2 && LPV != 4 ? 2 : 1>(A, blockIdx.x, blockIdx.x);
}

// Persistent form: each resident workgroup takes jobs from the device counter until none
// is left, every one in its own workspace region (see KArgs::jobctr).  One vector per lane
// group and pass: the loop's registers leave no room for two.
template <int LPV, int NI, int DT>
__global__ void __launch_bounds__(1024) search_multi_loop(KArgs A)
{
    extern __shared__ __attribute__((aligned(16))) unsigned char smem[];
    Ctrl *const C = reinterpret_cast<Ctrl *>(smem + A.o_ctrl);
    for (;;) {
        __syncthreads();
        if (threadIdx.x == 0) C->job = atomicAdd(A.jobctr, 1);
        __syncthreads();
        const int job = C->job;
        if (job >= A.njobs) break;
        search_body<LPV, NI, DT>(A, job, blockIdx.x);
    }
    __syncthreads();
    if (threadIdx.x == 0) release_jobs(A.jobctr);
}

template <int LPV, int NI, int DT>
hipError_t launch1(const KArgs &A, int64_t nq, int M, uint32_t lds, hipStream_t s)
{
    auto k = A.jobctr ? search_multi_loop<LPV, NI, DT> : search_multi<LPV, NI, DT>;
    // the dynamic LDS limit is raised to the whole 160 KB once per kernel and device, not
    // on every launch (the latency path launches one query at a time); one mask per form
    static std::atomic<uint64_t> raised[2] = {{0}, {0}};
    std::atomic<uint64_t> &done = raised[A.jobctr ? 1 : 0];
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    const uint64_t bit = 1ull << (dev & 63);
    if (!(done.load(std::memory_order_acquire) & bit)) {
        e = hipFuncSetAttribute(reinterpret_cast<const void *>(k), hipFuncAttributeMaxDynamicSharedMemorySize,
                                160 * 1024);
        if (e != hipSuccess) return e;
        done.fetch_or(bit, std::memory_order_acq_rel);
    }
    int64_t grid = nq;
    if (A.jobctr) {
        e = resident_grid(reinterpret_cast<const void *>(k), 64 * M, lds, nq, &grid);
        if (e != hipSuccess) return e;
    }
    hipLaunchKernelGGL(k, dim3((unsigned)grid), dim3(64 * M), lds, s, A);
    return hipGetLastError();
}

template <int LPV, int DT>
hipError_t launch1_ni(const KArgs &A, int64_t nq, int M, uint32_t lds, hipStream_t s)
{
    const int ni = (A.L + 63) / 64;
    if (ni <= 1) return launch1<LPV, 1, DT>(A, nq, M, lds, s);
    if (ni <= 2) return launch1<LPV, 2, DT>(A, nq, M, lds, s);
    if (ni <= 4) return launch1<LPV, 4, DT>(A, nq, M, lds, s);
    if (ni <= 6) return launch1<LPV, 6, DT>(A, nq, M, lds, s);
    if (ni <= 8) return launch1<LPV, 8, DT>(A, nq, M, lds, s);
    return launch1<LPV, 16, DT>(A, nq, M, lds, s);
}

// one instantiation per storage type, each in a file of its own (search_multi_*.hip)
template <int DT>
int launch_dt(const KArgs &A, int64_t nq, int M, uint32_t lds, hipStream_t s)
{
    hipError_t e;
    switch (lanes_per_vector(A.d)) {
    case 1: e = launch1_ni<1, DT>(A, nq, M, lds, s); break;
    case 2: e = launch1_ni<2, DT>(A, nq, M, lds, s); break;
    case 4: e = launch1_ni<4, DT>(A, nq, M, lds, s); break;
    case 8: e = launch1_ni<8, DT>(A, nq, M, lds, s); break;
    case 16: e = launch1_ni<16, DT>(A, nq, M, lds, s); break;
    case 32: e = launch1_ni<32, DT>(A, nq, M, lds, s); break;
    default: e = launch1_ni<64, DT>(A, nq, M, lds, s); break;
    }
    if (e != hipSuccess) return hip_fail(e, "search kernel launch");
    return SA_OK;
}

}  // namespace search_detail
}  // namespace sa
