// Deferred and grouped launches: several solves advanced together.
//
// While a Recorder is installed on the calling thread, the launch helpers
// below append each operation of a unit of PCG work (a kernel launch, a copy,
// an event record) to it instead of issuing it.  The recordings of several
// solves whose units have the same shape -- the same kernels in the same
// order -- are then replayed position by position: every kernel that has a
// grouped form runs as ONE launch over all the solves (a ragged grid: the
// blocks of solve g follow those of solve g - 1, each block finds its solve
// in the table of block offsets and runs the single-solve body with that
// solve's arguments); copies and event records run solve by solve.  The
// arithmetic of each solve is that of its own launches, so the results are
// bitwise those of the solve advanced alone.
//
// The table travels as a kernel argument (at most kGroupMax solves per
// launch; a larger group is launched in slices), so a grouped launch needs no
// device memory of its own.
#pragma once

#include <cstring>
#include <functional>
#include <vector>

#include "afn_internal.h"

namespace afn {

constexpr int kGroupMax = 16;

template <class A>
struct GroupTable {
    int32_t G;
    int32_t gx[kGroupMax];             // grid width of each solve's launch
    int64_t blk0[kGroupMax + 1];       // first block of each solve; blk0[G] = total
    A a[kGroupMax];
};

// Where block blockIdx.x of a grouped launch sits: solve g, its own block
// coordinates (bx, by) in a grid gx wide.
struct GroupPos {
    int g;
    int64_t bx, by, gx;
};

template <class A>
__device__ __forceinline__ GroupPos group_pos(const GroupTable<A> &t)
{
    const int64_t b = blockIdx.x;
    int g = 0;
    while (g + 1 < t.G && b >= t.blk0[g + 1]) ++g;
    const int64_t l = b - t.blk0[g];
    const int64_t gx = t.gx[g];
    return GroupPos{g, l % gx, l / gx, gx};
}

struct DeferredOp {
    std::function<hipError_t(hipStream_t)> run;     // issue it alone on a stream
    // grouped form (null if none): launches ops[0..G) as one kernel
    hipError_t (*group)(const DeferredOp *const *ops, int G, hipStream_t s) = nullptr;
    dim3 grid{1, 1, 1};
    size_t lds = 0;
    alignas(16) unsigned char args[256];
};

struct Recorder {
    std::vector<DeferredOp> ops;
};

// The calling thread's recorder (nullptr: operations are issued at once).
Recorder *&recorder();

// Issue at once while alive (the autotuner's timed runs, for instance).
struct RecorderPause {
    Recorder *saved;
    RecorderPause() : saved(recorder()) { recorder() = nullptr; }
    ~RecorderPause() { recorder() = saved; }
};

// A has: static void launch1(const A &, dim3 grid, size_t lds, hipStream_t)
// (the single-solve kernel) and static void launchG(const GroupTable<A> &,
// unsigned blocks, size_t lds, hipStream_t) (its grouped form).
template <class A>
hipError_t group_launch(const DeferredOp *const *ops, int G, hipStream_t s)
{
    GroupTable<A> t{};
    t.G = G;
    int64_t b = 0;
    size_t lds = 0;
    for (int g = 0; g < G; ++g) {
        t.gx[g] = (int32_t)ops[g]->grid.x;
        t.blk0[g] = b;
        b += (int64_t)ops[g]->grid.x * ops[g]->grid.y;
        std::memcpy((void *)&t.a[g], ops[g]->args, sizeof(A));
        lds = ops[g]->lds > lds ? ops[g]->lds : lds;
    }
    t.blk0[G] = b;
    if (b == 0) return hipSuccess;
    A::launchG(t, (unsigned)b, lds, s);
    return hipGetLastError();
}

template <class A>
afn_status dlaunch(dim3 grid, size_t lds, hipStream_t s, const A &a)
{
    static_assert(sizeof(A) <= sizeof(DeferredOp::args), "launch arguments too large to record");
    if (Recorder *r = recorder()) {
        DeferredOp op;
        op.run = [a, grid, lds](hipStream_t st) {
            A::launch1(a, grid, lds, st);
            return hipGetLastError();
        };
        op.group = &group_launch<A>;
        op.grid = grid;
        op.lds = lds;
        std::memcpy(op.args, (const void *)&a, sizeof(A));
        r->ops.push_back(std::move(op));
        return AFN_OK;
    }
    A::launch1(a, grid, lds, s);
    AFN_HIP(hipGetLastError());
    return AFN_OK;
}

// An operation without a grouped form, deferred like the rest.
afn_status defer(hipStream_t s, std::function<hipError_t(hipStream_t)> f);

// Replay the recordings of G solves on stream s.  Recordings of the same
// length are replayed position by position; at each position the solves whose
// operation is the same kernel (with a grouped form) share one launch, the
// others run one by one.  Each solve's operations stay in their order on s,
// so any such merge is correct.  merged[g] = 1 if solve g shared a launch.
afn_status replay_grouped(Recorder *const *recs, int G, hipStream_t s, char *merged);

}  // namespace afn
