// Kernel launches that serve one plan or a batch of independent systems.
//
// Every kernel is a body B::run(GridPos, const A&...) with B::kThreads threads per block:
// the block's index and the grid size come in as a GridPos instead of blockIdx / gridDim.
// launch<B>(plan, grid, lds, args...) launches it for one plan (k_single, blockIdx as the
// position), or, when the plan records (Plan::rec), stores the arguments and the grid
// instead.  A batch of systems records each system's sequence of launches once; the k-th
// launches of all systems then run as one launch of k_batched, whose blocks are dealt to
// the systems by a block-offset table (system s owns blocks [boff[s], boff[s+1]) and sees
// them as 0 .. its own grid size - 1) and whose arguments come from a table of the
// systems' recorded arguments in device memory.
#pragma once

#include <cstring>
#include <vector>

#include "device_common.hpp"

namespace sog {

struct GridPos {
    int bid;  // block index within the launch (or within its system's share of a batched launch)
    int nb;   // blocks of the launch (or of the system)
};

__device__ __forceinline__ GridPos grid_single() { return GridPos{(int)blockIdx.x, (int)gridDim.x}; }

// The kernel arguments of one launch as a flat aggregate (identical layout in host and
// device code); call() hands them to a functor by const reference.
template <class... A>
struct KArgs;
template <>
struct KArgs<> {
    template <class F, class... D>
    __device__ __forceinline__ void call(F&& f, const D&... d) const {
        f(d...);
    }
};
template <class H, class... T>
struct KArgs<H, T...> {
    H h;
    KArgs<T...> t;
    template <class F, class... D>
    __device__ __forceinline__ void call(F&& f, const D&... d) const {
        t.call(f, d..., h);
    }
};
inline KArgs<> make_kargs() { return KArgs<>{}; }
template <class H, class... T>
inline KArgs<H, T...> make_kargs(const H& h, const T&... t) {
    KArgs<H, T...> r;
    r.h = h;
    r.t = make_kargs(t...);
    return r;
}

template <class B, class... A>
__global__ __launch_bounds__(B::kThreads) void k_single(A... a) {
    B::run(grid_single(), a...);
}

// system of the calling block: boff[s] <= blockIdx.x < boff[s + 1] (binary search, uniform)
__device__ __forceinline__ int batch_system(const int* __restrict__ boff, int nsys) {
    int lo = 0, hi = nsys - 1;
    const int b = blockIdx.x;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (boff[mid] <= b) lo = mid;
        else hi = mid - 1;
    }
    return lo;
}

// A block finds its system (a uniform value) and runs the body on that system's argument
// record, read through the constant address space (scalar loads, as kernel arguments
// are).  The body is forced inline: as a called function it took the calling
// convention's registers (248 VGPRs and one wave per SIMD where the single-plan kernel
// has 124 and four).
template <class B, class... A>
__global__ __launch_bounds__(B::kThreads) void k_batched(const KArgs<A...>* __restrict__ tab,
                                                         const int* __restrict__ boff, int nsys) {
    const int s = __builtin_amdgcn_readfirstlane(batch_system(boff, nsys));
    const int b0 = __builtin_amdgcn_readfirstlane(boff[s]), b1 = __builtin_amdgcn_readfirstlane(boff[s + 1]);
    const GridPos g{(int)blockIdx.x - b0, b1 - b0};
    typedef const __attribute__((address_space(4))) KArgs<A...>* cptr;
    const cptr rec = (cptr)tab + s;
    ((const KArgs<A...>*)rec)->call([&](const A&... a) __attribute__((always_inline)) {
        [[clang::always_inline]] B::run(g, a...);
    });
}

// One recorded launch.
struct RecLaunch {
    const void* id = nullptr;            // the k_batched instantiation (identifies body and argument types)
    std::vector<unsigned char> args;     // the KArgs<A...> of the launch
    size_t align = 8;
    unsigned grid = 0, block = 0;
    size_t lds = 0;
    // launches k_batched for a table of nsys argument records at dtab (device)
    hipError_t (*batched)(const void* dtab, const int* boff, int nsys, unsigned blocks, size_t lds,
                          hipStream_t s) = nullptr;
};

template <class B, class... A>
hipError_t launch_batched_thunk(const void* dtab, const int* boff, int nsys, unsigned blocks, size_t lds,
                                hipStream_t s) {
    k_batched<B, A...><<<blocks, B::kThreads, lds, s>>>(static_cast<const KArgs<A...>*>(dtab), boff, nsys);
    return hipGetLastError();
}

// Launch body B on the plan's stream, or record the launch when the plan records.
// BATCH = false: a kernel that no batch runs (recording it is an error), and k_batched
// is not instantiated for it.
template <class B, bool BATCH = true, class... A>
hipError_t launch(Plan& p, unsigned grid, size_t lds, const A&... a) {
    if (grid == 0) return hipSuccess;
    if (p.rec) {
        if constexpr (!BATCH) {
            return hipErrorNotSupported;
        } else {
            RecLaunch r;
            const KArgs<A...> k = make_kargs(a...);
            r.id = reinterpret_cast<const void*>(&k_batched<B, A...>);
            r.args.resize(sizeof(k));
            std::memcpy(r.args.data(), &k, sizeof(k));
            r.align = alignof(KArgs<A...>);
            r.grid = grid;
            r.block = B::kThreads;
            r.lds = lds;
            r.batched = &launch_batched_thunk<B, A...>;
            p.rec->push_back(std::move(r));
            return hipSuccess;
        }
    }
    k_single<B, A...><<<grid, B::kThreads, lds, p.stream>>>(a...);
    return hipGetLastError();
}

// The XCD-aware logical block of xcd_logical_block for a block position of a launch (or of
// a system's share of a batched launch): the nb = 8 ceil(nwork / 8) blocks in groups of 8
// go to the 8 XCDs round-robin; -1 for the spare blocks.
__device__ __forceinline__ int xcd_logical(int nwork, GridPos g) {
    const int per = (nwork + 7) >> 3;
    const int logical = (g.bid & 7) * per + (g.bid >> 3);
    return logical < nwork ? logical : -1;
}

}  // namespace sog
