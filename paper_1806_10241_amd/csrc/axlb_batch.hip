// Batched stepping of many independent lattices of uneven size.  A step of
// many members runs as one fused launch over a work-list of (member, tile)
// pairs (chunks of a member's edge nodes, then its tiles).  100-step bundles
// are captured as HIP graphs; within a bundle, consecutive members whose
// state fits half the Infinity Cache together form a group that takes all
// 100 steps before the next group of its chain starts, and groups alternate
// between two chains (streams) that run side by side, so the states of the
// two running groups stay in that cache and one group's launch ramp and
// tail overlap the other's work (the members are independent, so their
// steps need no common order).  The tile shape and the launch schedule come from an
// autotuner.  The node update is the one of the single-lattice kernels
// (axlb_node.h), so a member's result does not depend on whether it ran
// alone or in a batch.
#include <hip/hip_runtime.h>

#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "../../include/axlb.h"
#include "axlb_internal.h"
#include "axlb_launch.h"
#include "axlb_node.h"

namespace axlb {

// State bytes of the members that one group holds: two groups run at once,
// together below MI355X's 256 MB Infinity Cache with room for the other
// traffic of a step.
constexpr size_t GROUP_BYTES = 80u << 20;

// Per-member descriptor in device memory.
struct InstDesc {
    KParams P;
    void *pop;
    char *lag[2];     // lagged-field blocks (format of the storage type)
    int parity0;     // member step count at batch creation, mod 2
    int tile_begin;  // first work-list entry of this member
    int gx;          // tiles along r
    int nedge;       // edge chunks, the member's first work-list entries
    Planes pl[2];    // plane addresses of the even (0) and odd (1) AA phase
};

// Work-list entries are dealt to the 8 XCDs in 8 contiguous chunks, so that
// the tiles of one member (and their neighbour rows) share an L2; within a
// chunk the blocks of that XCD stride over the entries.  With as many blocks
// as entries every block takes one tile; with fewer, blocks persist and loop.
template <class S, int BX, int BY>
__global__ void __launch_bounds__(BX *BY)
    k_step_batch(const InstDesc *__restrict__ D, const int *__restrict__ tile_inst, int t0,
                 int ntiles, int phase) {
    const int G = gridDim.x, b = blockIdx.x;
    const int xcd = b & 7, k = b >> 3;
    const int nbx = (G >> 3) + (xcd < (G & 7) ? 1 : 0);
    const int lo = t0 + (int)((long long)ntiles * xcd / 8);
    const int hi = t0 + (int)((long long)ntiles * (xcd + 1) / 8);
    for (int t = lo + k; t < hi; t += nbx) {
        const InstDesc *d = D + tile_inst[t];
        const int local = t - d->tile_begin;
        const bool odd = (d->parity0 ^ phase) == 0;
        S *A = (S *)d->pop;
        // edge nodes have entries of their own in the odd phase and, with
        // 16-bit storage, in the even phase too (as in the single-lattice
        // kernel; with FP32 the even phase's extra edge entries cost more than
        // the tiles' boundary code: 22.1k against 23.5k MLUPS on the 256
        // uneven annuli)
        constexpr bool SPLIT_EVEN = sizeof(S) == 2;
        if (local < d->nedge) {
            const int e = local * (BX * BY) + (int)threadIdx.x;
            if ((!odd && !SPLIT_EVEN) || e >= edge_count(d->P.Nr, d->P.Nz)) continue;
            int i, j;
            edge_node(d->P, e, i, j);
            if (odd)
                update_node<S, MODE_AA_ODD>(d->P, A, A, d->lag[0], d->lag[1], i, j, false);
            else
                update_node<S, MODE_AA_EVEN>(d->P, A, A, d->lag[1], d->lag[0], i, j, false);
            continue;
        }
        const int u = local - d->nedge;
        const int j = (u % d->gx) * BX + (int)threadIdx.x % BX;
        const int i = (u / d->gx) * BY + (int)threadIdx.x / BX;
        if (odd || SPLIT_EVEN) {
            if (!interior_node(d->P, i, j)) continue;  // edge nodes and the ragged tail
            update_planes<S>(d->P, d->pl[odd ? 1 : 0], i, j, true);
        } else {
            if (i >= d->P.Nz || j >= d->P.Nr) continue;
            update_planes<S>(d->P, d->pl[0], i, j, interior_node(d->P, i, j));
        }
    }
}

#define AXLB_BATCH_TILES(X) X(0, 64, 4) X(1, 64, 2) X(2, 64, 8) X(3, 128, 2) X(4, 256, 1) \
    X(5, 64, 1) X(6, 128, 4) X(7, 32, 8)

template <class S>
static hipError_t launch_batch_t(int tile, int blocks, const InstDesc *D, const int *tiles,
                                 int t0, int ntiles, int phase, hipStream_t st) {
    switch (tile) {
#define AXLB_CASE(id, bx, by)                                                               \
    case id:                                                                                \
        k_step_batch<S, bx, by><<<blocks, bx * by, 0, st>>>(D, tiles, t0, ntiles, phase); \
        break;
        AXLB_BATCH_TILES(AXLB_CASE)
#undef AXLB_CASE
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

static hipError_t launch_batch(int storage, int tile, int blocks, const InstDesc *D,
                               const int *tiles, int t0, int ntiles, int phase, hipStream_t st) {
    if (storage == STORE_F16)
        return launch_batch_t<__half>(tile, blocks, D, tiles, t0, ntiles, phase, st);
    if (storage == STORE_BF16)
        return launch_batch_t<__hip_bfloat16>(tile, blocks, D, tiles, t0, ntiles, phase, st);
    return launch_batch_t<float>(tile, blocks, D, tiles, t0, ntiles, phase, st);
}

// Whole members: members of at most WHOLE_MAX_NODES nodes may instead run
// one per workgroup, which takes the member through `nsteps` steps in one
// launch (a bundle's 100 steps in one kernel) with a workgroup barrier
// between steps: no launch per step, and the member's edge nodes run in the
// same workgroup as its interior (the first threads take them, in both
// phases, so that the interior loop runs the fast path alone: 15.1k against
// 14.2k MLUPS on 1024 small annuli in FP32).  Every node of an AA phase reads and
// writes only its own 19 slots, so the threads of a step need no order
// among themselves; the barrier (with its workgroup-scope fences) makes a
// step's stores visible to the next step's loads.  Thread k of the
// workgroup takes nodes k, k + WHOLE_THREADS, ... in row-major order.
constexpr int WHOLE_THREADS = 1024;
constexpr long long WHOLE_MAX_NODES = AXLB_WHOLE_MAX_NODES;

template <class S>
__global__ void __launch_bounds__(WHOLE_THREADS)
    k_batch_whole(const InstDesc *__restrict__ D, const int *__restrict__ whole, int nwhole,
                  int phase0, int nsteps) {
    const int tid = (int)threadIdx.x;
    for (int w = (int)blockIdx.x; w < nwhole; w += (int)gridDim.x) {
        const InstDesc *d = D + whole[w];
        S *A = (S *)d->pop;
        const int Nr = d->P.Nr, N = Nr * d->P.Nz, ne = edge_count(Nr, d->P.Nz);
        const int di = WHOLE_THREADS / Nr, dj = WHOLE_THREADS % Nr;
        const int i0 = tid / Nr, j0 = tid % Nr;
        for (int s = 0; s < nsteps; ++s) {
            const bool odd = (d->parity0 ^ ((phase0 + s) & 1)) == 0;
            for (int e = tid; e < ne; e += WHOLE_THREADS) {
                int i, j;
                edge_node(d->P, e, i, j);
                if (odd)
                    update_node<S, MODE_AA_ODD>(d->P, A, A, d->lag[0], d->lag[1], i, j, false);
                else
                    update_node<S, MODE_AA_EVEN>(d->P, A, A, d->lag[1], d->lag[0], i, j, false);
            }
            int i = i0, j = j0;
            const Planes &pl = d->pl[odd ? 1 : 0];
            for (int k = tid; k < N; k += WHOLE_THREADS) {
                if (interior_node(d->P, i, j)) update_planes<S>(d->P, pl, i, j, true);
                i += di;
                j += dj;
                if (j >= Nr) {
                    j -= Nr;
                    ++i;
                }
            }
            __syncthreads();
        }
    }
}

static hipError_t launch_whole(int storage, const InstDesc *D, const int *whole, int nwhole,
                               int phase0, int nsteps, hipStream_t st) {
    if (nwhole == 0) return hipSuccess;
    const dim3 grid(nwhole), block(WHOLE_THREADS);
    if (storage == STORE_F16)
        k_batch_whole<__half><<<grid, block, 0, st>>>(D, whole, nwhole, phase0, nsteps);
    else if (storage == STORE_BF16)
        k_batch_whole<__hip_bfloat16><<<grid, block, 0, st>>>(D, whole, nwhole, phase0, nsteps);
    else
        k_batch_whole<float><<<grid, block, 0, st>>>(D, whole, nwhole, phase0, nsteps);
    return hipGetLastError();
}

}  // namespace axlb

using namespace axlb;

struct axlb_batch {
    int device = 0;
    hipStream_t stream = nullptr;
    // a bundle runs its groups on two chains, the batch stream and `side`,
    // forked and joined by these events, so that two groups share the
    // device and one group's launch ramp and tail overlap the other's work
    hipStream_t side = nullptr;
    hipEvent_t fork = nullptr, join = nullptr;
    // whole members (AA): those of at most whole_max nodes run one per
    // workgroup (d_whole lists them, nwhole of them), on the chain `aux`
    // during a bundle; the work-list holds the others
    long long whole_max = 0;
    int *d_whole = nullptr;
    int nwhole = 0;
    hipStream_t aux = nullptr;
    hipEvent_t join_aux = nullptr;
    std::vector<axlb_lattice *> members;
    std::vector<hipStream_t> member_streams;
    int storage = 0;
    int layout = AXLB_LAYOUT_AA;
    int tile = 0;
    int blocks = 0;  // 0: one block per work-list entry; else persistent blocks
    InstDesc *d_desc = nullptr;
    // two-buffer members (AXLB_LAYOUT_AB2): two steps per launch; a member
    // reads buffer pair cur0 ^ phase, and phase flips with every launch
    TwoDesc *d_two = nullptr;
    int2 *d_two_tiles = nullptr;
    int phase = 0;
    int *d_tiles = nullptr;
    int ntiles = 0;
    // work-list ranges of consecutive members whose state fits the
    // Infinity Cache together: a bundle runs all its steps on one group
    // before the next; group g is entries [group[g], group[g + 1])
    std::vector<int> group;
    long steps = 0;
    hipGraphExec_t graph[2] = {nullptr, nullptr};
    std::string err;
};

static thread_local std::string g_batch_error;

static int bfail(axlb_batch *b, int code, const std::string &m) {
    if (b) b->err = m;
    else g_batch_error = m;
    return code;
}

#define BHIP(b, expr)                                                                    \
    do {                                                                                 \
        hipError_t e_ = (expr);                                                          \
        if (e_ != hipSuccess) return bfail(b, AXLB_EDEVICE, std::string(#expr) + ": " + \
                                                               hipGetErrorString(e_));   \
    } while (0)

static void drop_batch_graphs(axlb_batch *b) {
    for (int k = 0; k < 2; ++k)
        if (b->graph[k]) {
            (void)hipGraphExecDestroy(b->graph[k]);
            b->graph[k] = nullptr;
        }
}

// Descriptors and work-list of a batch of two-buffer members: every tile
// of the two-step kernel of every member, in one group, in member order
// (which the kernel cuts into its 8 XCD chunks).  Listing each chunk's rim
// tiles first, as the single-lattice launch does, measured slower here
// (21.2k against 24.8k MLUPS for the 256 uneven annuli): a member's rim
// and inner tiles then run apart and lose the L2 reuse of their shared
// rows, and small members are mostly rim.
static int build_worklist_two(axlb_batch *b) {
    int tw, th;
    two_batch_tile_shape(&tw, &th);
    std::vector<TwoDesc> desc(b->members.size());
    std::vector<int2> tiles;
    b->group.clear();
    size_t group_bytes = 0;
    for (size_t m = 0; m < b->members.size(); ++m) {
        axlb_lattice *L = b->members[m];
        TwoDesc &d = desc[m];
        std::memset(&d, 0, sizeof(d));
        d.P = L->P;
        for (int c = 0; c < 2; ++c) {
            d.src[c] = L->pop[c];
            d.lag[c] = L->lag[c];
            d.pl[c] = step_planes(L->P, L->storage, MODE_AB, L->pop[c], L->pop[c ^ 1], L->lag[c],
                                  L->lag[c ^ 1]);
        }
        d.cur0 = L->cur ^ b->phase;
        d.gx = (L->Nr + tw - 1) / tw;
        const int gy = (L->Nz + th - 1) / th;
        const int first = (int)tiles.size();
        for (int t = 0; t < d.gx * gy; ++t) tiles.push_back(make_int2((int)m, t));
        // groups of consecutive members whose states (both buffers) fit
        // GROUP_BYTES, as for AA members
        const size_t bytes = 2 * L->lay.pop_bytes + 2 * L->lay.lag_bytes;
        if (m == 0 || group_bytes + bytes > GROUP_BYTES) {
            b->group.push_back(first);
            group_bytes = 0;
        }
        group_bytes += bytes;
    }
    const int n = (int)tiles.size();
    b->group.push_back(n);
    if (b->d_two) (void)hipFree(b->d_two);
    if (b->d_two_tiles) (void)hipFree(b->d_two_tiles);
    b->d_two = nullptr;
    b->d_two_tiles = nullptr;
    BHIP(b, hipMalloc((void **)&b->d_two, desc.size() * sizeof(TwoDesc)));
    BHIP(b, hipMalloc((void **)&b->d_two_tiles, tiles.size() * sizeof(int2)));
    BHIP(b, hipMemcpyAsync(b->d_two, desc.data(), desc.size() * sizeof(TwoDesc),
                           hipMemcpyHostToDevice, b->stream));
    BHIP(b, hipMemcpyAsync(b->d_two_tiles, tiles.data(), tiles.size() * sizeof(int2),
                           hipMemcpyHostToDevice, b->stream));
    BHIP(b, hipStreamSynchronize(b->stream));
    b->ntiles = n;
    drop_batch_graphs(b);
    return AXLB_OK;
}

// Descriptors and work-list for the current tile shape.
static int build_worklist(axlb_batch *b) {
    if (b->layout == AXLB_LAYOUT_AB2) return build_worklist_two(b);
    int bx, by;
    tile_shape(b->tile, &bx, &by);
    std::vector<InstDesc> desc(b->members.size());
    std::vector<int> tiles, whole;
    b->group.clear();
    size_t group_bytes = 0;
    for (size_t m = 0; m < b->members.size(); ++m) {
        axlb_lattice *L = b->members[m];
        InstDesc &d = desc[m];
        std::memset(&d, 0, sizeof(d));
        d.P = L->P;
        d.pop = L->pop[0];
        d.lag[0] = L->lag[0];
        d.lag[1] = L->lag[1];
        d.pl[0] = step_planes(L->P, L->storage, MODE_AA_EVEN, d.pop, d.pop, d.lag[1], d.lag[0]);
        d.pl[1] = step_planes(L->P, L->storage, MODE_AA_ODD, d.pop, d.pop, d.lag[0], d.lag[1]);
        d.parity0 = (int)((L->steps - b->steps) & 1);
        if ((long long)L->Nr * L->Nz <= b->whole_max) {  // one workgroup takes it whole
            whole.push_back((int)m);
            continue;
        }
        d.gx = (L->Nr + bx - 1) / bx;
        const int gy = (L->Nz + by - 1) / by;
        d.nedge = (edge_count(L->Nr, L->Nz) + bx * by - 1) / (bx * by);
        d.tile_begin = (int)tiles.size();
        tiles.insert(tiles.end(), (size_t)d.nedge + (size_t)d.gx * gy, (int)m);
        const size_t bytes = L->lay.pop_bytes + 2 * L->lay.lag_bytes;
        if (b->group.empty() || group_bytes + bytes > GROUP_BYTES) {
            b->group.push_back(d.tile_begin);
            group_bytes = 0;
        }
        group_bytes += bytes;
    }
    if (b->group.empty()) b->group.push_back(0);
    b->group.push_back((int)tiles.size());
    if (b->d_desc) (void)hipFree(b->d_desc);
    if (b->d_tiles) (void)hipFree(b->d_tiles);
    if (b->d_whole) (void)hipFree(b->d_whole);
    b->d_desc = nullptr;
    b->d_tiles = nullptr;
    b->d_whole = nullptr;
    b->ntiles = 0;
    b->nwhole = 0;
    BHIP(b, hipMalloc((void **)&b->d_desc, desc.size() * sizeof(InstDesc)));
    BHIP(b, hipMalloc((void **)&b->d_tiles, (tiles.size() + 1) * sizeof(int)));
    BHIP(b, hipMalloc((void **)&b->d_whole, (whole.size() + 1) * sizeof(int)));
    BHIP(b, hipMemcpyAsync(b->d_desc, desc.data(), desc.size() * sizeof(InstDesc),
                           hipMemcpyHostToDevice, b->stream));
    if (!tiles.empty())
        BHIP(b, hipMemcpyAsync(b->d_tiles, tiles.data(), tiles.size() * sizeof(int),
                               hipMemcpyHostToDevice, b->stream));
    if (!whole.empty())
        BHIP(b, hipMemcpyAsync(b->d_whole, whole.data(), whole.size() * sizeof(int),
                               hipMemcpyHostToDevice, b->stream));
    BHIP(b, hipStreamSynchronize(b->stream));
    b->ntiles = (int)tiles.size();
    b->nwhole = (int)whole.size();
    drop_batch_graphs(b);
    return AXLB_OK;
}

// One step (parity s & 1) of the work-list entries [t0, t1).
static int batch_launch(axlb_batch *b, long s, int t0, int t1, hipStream_t st) {
    const int n = t1 - t0;
    if (n <= 0) return AXLB_OK;  // every member runs whole
    int blocks = b->blocks > 0 ? b->blocks : n;
    if (blocks < 8) blocks = 8;  // every XCD chunk needs a block
    hipError_t e = launch_batch(b->storage, b->tile, blocks, b->d_desc, b->d_tiles, t0, n,
                                (int)(s & 1), st);
    if (e != hipSuccess) return bfail(b, AXLB_EDEVICE, std::string("batch launch: ") + hipGetErrorString(e));
    return AXLB_OK;
}

static int batch_launch(axlb_batch *b, long s, int t0, int t1) {
    return batch_launch(b, s, t0, t1, b->stream);
}
static int batch_launch(axlb_batch *b, long s) { return batch_launch(b, s, 0, b->ntiles); }

// `nsteps` steps of the whole members from batch step s, on stream st.
static int whole_launch(axlb_batch *b, long s, int nsteps, hipStream_t st) {
    const hipError_t e = launch_whole(b->storage, b->d_desc, b->d_whole, b->nwhole, (int)(s & 1),
                                      nsteps, st);
    if (e != hipSuccess) return bfail(b, AXLB_EDEVICE, std::string("whole-member launch: ") + hipGetErrorString(e));
    return AXLB_OK;
}

// Steps s .. s + nsteps - 1 of an AA batch as a bundle runs them: the
// whole members in one launch on the chain `aux`, the work-list group by
// group on the two chains `stream` and `side`, joined back into `stream`.
static int bundle_launches(axlb_batch *b, long s, int nsteps) {
    int rc = AXLB_OK;
    hipError_t fe = hipEventRecord(b->fork, b->stream);
    if (fe == hipSuccess) fe = hipStreamWaitEvent(b->side, b->fork, 0);
    if (fe == hipSuccess) fe = hipStreamWaitEvent(b->aux, b->fork, 0);
    if (fe != hipSuccess) return bfail(b, AXLB_EDEVICE, "batch fork failed");
    if (b->nwhole > 0) rc = whole_launch(b, s, nsteps, b->aux);
    for (size_t g = 0; g + 1 < b->group.size() && rc == AXLB_OK; ++g)
        for (long k = 0; k < nsteps && rc == AXLB_OK; ++k)
            rc = batch_launch(b, s + k, b->group[g], b->group[g + 1], g % 2 ? b->side : b->stream);
    fe = hipEventRecord(b->join, b->side);
    if (fe == hipSuccess) fe = hipStreamWaitEvent(b->stream, b->join, 0);
    if (fe == hipSuccess) fe = hipEventRecord(b->join_aux, b->aux);
    if (fe == hipSuccess) fe = hipStreamWaitEvent(b->stream, b->join_aux, 0);
    if (fe != hipSuccess && rc == AXLB_OK) rc = bfail(b, AXLB_EDEVICE, "batch join failed");
    return rc;
}

static void advance_members(axlb_batch *b, long n) {
    b->steps += n;
    for (axlb_lattice *L : b->members) L->steps += n;
}

// One two-step launch of the work-list entries [t0, t1) of a two-buffer
// batch (every member by default).
static int two_launch(axlb_batch *b, int phase, int t0, int t1, hipStream_t st) {
    const hipError_t e = launch_step_two_batch(b->storage, b->d_two, b->d_two_tiles, t0, t1 - t0,
                                               phase, st);
    if (e != hipSuccess) return bfail(b, AXLB_EDEVICE, std::string("batch launch: ") + hipGetErrorString(e));
    return AXLB_OK;
}
static int two_launch(axlb_batch *b, int phase) { return two_launch(b, phase, 0, b->ntiles, b->stream); }

// After `launches` two-step launches: two steps each, one buffer flip each.
static void advance_two(axlb_batch *b, long launches) {
    advance_members(b, 2 * launches);
    if (launches & 1) {
        b->phase ^= 1;
        for (axlb_lattice *L : b->members) L->cur ^= 1;
    }
}

// n steps of a two-buffer batch: 100-step bundles as graphs of 50 launches
// (keyed by the phase they start from), pairs of steps as plain launches,
// and a last odd step as one single step of each member (which flips its
// buffers as a launch does).
static int batch_step_two(axlb_batch *b, long n) {
    while (n > 0) {
        if (n >= BUNDLE) {
            const int k = b->phase;
            if (!b->graph[k]) {
                BHIP(b, hipStreamBeginCapture(b->stream, hipStreamCaptureModeThreadLocal));
                // group by group, alternating between two chains, as for AA
                // members: a group's two buffers stay in the Infinity Cache
                // through its 50 launches
                int rc = AXLB_OK;
                hipError_t fe = hipEventRecord(b->fork, b->stream);
                if (fe == hipSuccess) fe = hipStreamWaitEvent(b->side, b->fork, 0);
                if (fe != hipSuccess) rc = bfail(b, AXLB_EDEVICE, "batch graph fork failed");
                for (size_t gi = 0; gi + 1 < b->group.size() && rc == AXLB_OK; ++gi)
                    for (long s = 0; s < BUNDLE / 2 && rc == AXLB_OK; ++s)
                        rc = two_launch(b, (int)((k + s) & 1), b->group[gi], b->group[gi + 1],
                                        gi % 2 ? b->side : b->stream);
                fe = hipEventRecord(b->join, b->side);
                if (fe == hipSuccess) fe = hipStreamWaitEvent(b->stream, b->join, 0);
                if (fe != hipSuccess && rc == AXLB_OK) rc = bfail(b, AXLB_EDEVICE, "batch graph join failed");
                hipGraph_t g = nullptr;
                hipError_t e = hipStreamEndCapture(b->stream, &g);
                if (rc != AXLB_OK) {
                    if (g) (void)hipGraphDestroy(g);
                    return rc;
                }
                if (e != hipSuccess) return bfail(b, AXLB_EDEVICE, "batch graph capture failed");
                e = hipGraphInstantiate(&b->graph[k], g, nullptr, nullptr, 0);
                (void)hipGraphDestroy(g);
                if (e != hipSuccess) {
                    b->graph[k] = nullptr;
                    return bfail(b, AXLB_EDEVICE, "batch graph instantiate failed");
                }
            }
            BHIP(b, hipGraphLaunch(b->graph[k], b->stream));
            advance_two(b, BUNDLE / 2);
            n -= BUNDLE;
        } else if (n >= 2) {
            const int rc = two_launch(b, b->phase);
            if (rc) return rc;
            advance_two(b, 1);
            n -= 2;
        } else {
            for (axlb_lattice *L : b->members) {
                const int rc = lattice_step_once(L);
                if (rc) return bfail(b, rc, L->err);
            }
            b->steps += 1;
            b->phase ^= 1;
            n -= 1;
        }
    }
    return AXLB_OK;
}

extern "C" {

int axlb_batch_create(axlb_lattice *const *lats, int n, axlb_batch **out) {
    if (!out) return bfail(nullptr, AXLB_EINVAL, "out is NULL");
    *out = nullptr;
    if (!lats || n <= 0) return bfail(nullptr, AXLB_EINVAL, "empty batch");
    const int dev = lats[0] ? lats[0]->device : 0;
    for (int m = 0; m < n; ++m) {
        axlb_lattice *L = lats[m];
        if (!L) return bfail(nullptr, AXLB_EINVAL, "NULL member");
        if (L->device != dev) return bfail(nullptr, AXLB_EINVAL, "members on different devices");
        if (L->layout != AXLB_LAYOUT_AA && L->layout != AXLB_LAYOUT_AB2)
            return bfail(nullptr, AXLB_EINVAL, "batches need the AA or the AB2 layout");
        if (L->layout != lats[0]->layout) return bfail(nullptr, AXLB_EINVAL, "mixed layouts in a batch");
        if (L->storage != lats[0]->storage) return bfail(nullptr, AXLB_EINVAL, "mixed storage in a batch");
        if (L->batched) return bfail(nullptr, AXLB_ESTATE, "lattice already in a batch");
        for (int k = 0; k < m; ++k)
            if (lats[k] == L) return bfail(nullptr, AXLB_EINVAL, "lattice listed twice");
    }
    axlb_batch *b = new (std::nothrow) axlb_batch();
    if (!b) return bfail(nullptr, AXLB_ENOMEM, "host allocation failed");
    b->device = dev;
    b->storage = lats[0]->storage;
    b->layout = lats[0]->layout;
    if (hipSetDevice(dev) != hipSuccess ||
        hipStreamCreateWithFlags(&b->stream, hipStreamNonBlocking) != hipSuccess ||
        hipStreamCreateWithFlags(&b->side, hipStreamNonBlocking) != hipSuccess ||
        hipStreamCreateWithFlags(&b->aux, hipStreamNonBlocking) != hipSuccess ||
        hipEventCreateWithFlags(&b->fork, hipEventDisableTiming) != hipSuccess ||
        hipEventCreateWithFlags(&b->join, hipEventDisableTiming) != hipSuccess ||
        hipEventCreateWithFlags(&b->join_aux, hipEventDisableTiming) != hipSuccess) {
        if (b->join_aux) (void)hipEventDestroy(b->join_aux);
        if (b->join) (void)hipEventDestroy(b->join);
        if (b->fork) (void)hipEventDestroy(b->fork);
        if (b->aux) (void)hipStreamDestroy(b->aux);
        if (b->side) (void)hipStreamDestroy(b->side);
        if (b->stream) (void)hipStreamDestroy(b->stream);
        delete b;
        return bfail(nullptr, AXLB_EDEVICE, "stream creation failed");
    }
    for (int m = 0; m < n; ++m) {
        axlb_lattice *L = lats[m];
        // lock the boundary rules as a first step would
        const int rc = lattice_start(L);
        if (rc != AXLB_OK) {
            const std::string msg = std::string("member ") + std::to_string(m) + ": " + L->err;
            axlb_batch_destroy(b);
            return bfail(nullptr, rc, msg);
        }
        (void)hipStreamSynchronize(L->stream);
        b->members.push_back(L);
        b->member_streams.push_back(L->stream);
        L->stream = b->stream;  // all member work is ordered on the batch stream
        L->batched = true;
    }
    int rc = build_worklist(b);
    if (rc != AXLB_OK) {
        const std::string msg = b->err;
        axlb_batch_destroy(b);
        return bfail(nullptr, rc, msg);
    }
    *out = b;
    return AXLB_OK;
}

int axlb_batch_size(const axlb_batch *b, int *members, long long *nodes) {
    if (!b) return bfail(nullptr, AXLB_EINVAL, "batch is NULL");
    long long s = 0;
    for (const axlb_lattice *L : b->members) s += (long long)L->Nr * L->Nz;
    if (members) *members = (int)b->members.size();
    if (nodes) *nodes = s;
    return AXLB_OK;
}

int axlb_batch_set_schedule(axlb_batch *b, int tile, int blocks) {
    if (!b) return bfail(nullptr, AXLB_EINVAL, "batch is NULL");
    if (tile < 0 || tile >= tile_count() || blocks < 0) return bfail(b, AXLB_EINVAL, "bad schedule");
    if (b->layout == AXLB_LAYOUT_AB2)
        return bfail(b, AXLB_EINVAL, "a batch of AB2 members has one schedule");
    BHIP(b, hipSetDevice(b->device));
    BHIP(b, hipStreamSynchronize(b->stream));
    const bool rebuild = tile != b->tile;
    b->tile = tile;
    b->blocks = blocks;
    drop_batch_graphs(b);
    return rebuild ? build_worklist(b) : AXLB_OK;
}

int axlb_batch_get_schedule(const axlb_batch *b, int *tile, int *blocks) {
    if (!b) return bfail(nullptr, AXLB_EINVAL, "batch is NULL");
    if (tile) *tile = b->tile;
    if (blocks) *blocks = b->blocks;
    return AXLB_OK;
}

int axlb_batch_set_whole(axlb_batch *b, long long max_nodes) {
    if (!b) return bfail(nullptr, AXLB_EINVAL, "batch is NULL");
    if (max_nodes < 0 || max_nodes > WHOLE_MAX_NODES)
        return bfail(b, AXLB_EINVAL, "max_nodes must lie in [0, AXLB_WHOLE_MAX_NODES]");
    if (b->layout == AXLB_LAYOUT_AB2)
        return bfail(b, AXLB_EINVAL, "whole members are for AA members");
    BHIP(b, hipSetDevice(b->device));
    BHIP(b, hipStreamSynchronize(b->stream));
    b->whole_max = max_nodes;
    return build_worklist(b);
}

int axlb_batch_get_whole(const axlb_batch *b, long long *max_nodes, int *members) {
    if (!b) return bfail(nullptr, AXLB_EINVAL, "batch is NULL");
    if (max_nodes) *max_nodes = b->whole_max;
    if (members) *members = b->nwhole;
    return AXLB_OK;
}

int axlb_batch_step(axlb_batch *b, long n) {
    if (!b) return bfail(nullptr, AXLB_EINVAL, "batch is NULL");
    if (n < 0) return bfail(b, AXLB_EINVAL, "negative step count");
    BHIP(b, hipSetDevice(b->device));
    if (b->layout == AXLB_LAYOUT_AB2) return batch_step_two(b, n);
    while (n > 0) {
        if (n >= BUNDLE) {
            const int k = (int)(b->steps & 1);
            if (!b->graph[k]) {
                BHIP(b, hipStreamBeginCapture(b->stream, hipStreamCaptureModeThreadLocal));
                // group by group, alternate groups on two chains: each
                // group's state stays in the Infinity Cache for the whole
                // bundle, and two groups run side by side; the whole
                // members take the bundle in one launch on a third chain
                const int rc = bundle_launches(b, k, (int)BUNDLE);
                hipGraph_t g = nullptr;
                hipError_t e = hipStreamEndCapture(b->stream, &g);
                if (rc != AXLB_OK) {
                    if (g) (void)hipGraphDestroy(g);
                    return rc;
                }
                if (e != hipSuccess) return bfail(b, AXLB_EDEVICE, "batch graph capture failed");
                e = hipGraphInstantiate(&b->graph[k], g, nullptr, nullptr, 0);
                (void)hipGraphDestroy(g);
                if (e != hipSuccess) {
                    b->graph[k] = nullptr;
                    return bfail(b, AXLB_EDEVICE, "batch graph instantiate failed");
                }
            }
            BHIP(b, hipGraphLaunch(b->graph[k], b->stream));
            advance_members(b, BUNDLE);
            n -= BUNDLE;
        } else {
            int rc = whole_launch(b, b->steps, 1, b->stream);
            if (rc == AXLB_OK) rc = batch_launch(b, b->steps);
            if (rc) return rc;
            advance_members(b, 1);
            n -= 1;
        }
    }
    return AXLB_OK;
}

int axlb_batch_sync(axlb_batch *b) {
    if (!b) return bfail(nullptr, AXLB_EINVAL, "batch is NULL");
    BHIP(b, hipSetDevice(b->device));
    BHIP(b, hipStreamSynchronize(b->stream));
    return AXLB_OK;
}

int axlb_batch_autotune(axlb_batch *b, int steps_per_trial, double *ms_per_step, int *best_tile,
                        int *best_blocks) {
    if (!b) return bfail(nullptr, AXLB_EINVAL, "batch is NULL");
    if (steps_per_trial < 2) return bfail(b, AXLB_EINVAL, "steps_per_trial must be >= 2");
    BHIP(b, hipSetDevice(b->device));
    if (b->layout == AXLB_LAYOUT_AB2) {
        // one schedule: nothing to choose
        if (ms_per_step)
            for (int k = 0; k < tile_count() * AXLB_NSCHEDULES; ++k) ms_per_step[k] = 0.0;
        if (best_tile) *best_tile = b->tile;
        if (best_blocks) *best_blocks = b->blocks;
        return AXLB_OK;
    }
    int dev_cu = 0;
    BHIP(b, hipDeviceGetAttribute(&dev_cu, hipDeviceAttributeMultiprocessorCount, b->device));
    const int sched[AXLB_NSCHEDULES] = {0, 4 * dev_cu, 8 * dev_cu, 16 * dev_cu};
    // keep every member's state; the trials step them
    std::vector<char *> keep(b->members.size(), nullptr);
    auto release = [&]() {
        for (char *p : keep)
            if (p) (void)hipFree(p);
    };
    for (size_t m = 0; m < b->members.size(); ++m) {
        axlb_lattice *L = b->members[m];
        const size_t bytes = L->lay.pop_bytes + 2 * L->lay.lag_bytes;
        if (hipMalloc((void **)&keep[m], bytes) != hipSuccess) {
            release();
            return bfail(b, AXLB_ENOMEM, "autotune snapshot");
        }
        BHIP(b, hipMemcpyAsync(keep[m], L->pop[0], bytes, hipMemcpyDeviceToDevice, b->stream));
    }
    hipEvent_t e0, e1;
    BHIP(b, hipEventCreate(&e0));
    BHIP(b, hipEventCreate(&e1));
    const long steps0 = b->steps;
    const int tile0 = b->tile, blocks0 = b->blocks;
    const long long whole0 = b->whole_max;
    double best_ms = 1e300;
    int bt = b->tile, bb = b->blocks, rc = AXLB_OK;
    long long bw = 0;
    b->whole_max = 0;  // the work-list schedules first, every member in the list
    for (int t = 0; t < tile_count() && rc == AXLB_OK; ++t) {
        b->tile = t;
        rc = build_worklist(b);
        for (int sidx = 0; sidx < AXLB_NSCHEDULES && rc == AXLB_OK; ++sidx) {
            b->blocks = sched[sidx];
            for (int s = 0; s < 2 && rc == AXLB_OK; ++s, ++b->steps) rc = batch_launch(b, b->steps);
            // the trial steps group by group, as a bundle does
            (void)hipEventRecord(e0, b->stream);
            for (size_t g = 0; g + 1 < b->group.size() && rc == AXLB_OK; ++g)
                for (int s = 0; s < steps_per_trial && rc == AXLB_OK; ++s)
                    rc = batch_launch(b, b->steps + s, b->group[g], b->group[g + 1]);
            b->steps += steps_per_trial;
            (void)hipEventRecord(e1, b->stream);
            float ms = 0.f;
            if (rc == AXLB_OK && (hipEventSynchronize(e1) != hipSuccess ||
                                  hipEventElapsedTime(&ms, e0, e1) != hipSuccess))
                rc = bfail(b, AXLB_EDEVICE, "autotune timing");
            const double per = ms / steps_per_trial;
            if (ms_per_step) ms_per_step[t * AXLB_NSCHEDULES + sidx] = per;
            if (rc == AXLB_OK && per < best_ms) {
                best_ms = per;
                bt = t;
                bb = sched[sidx];
            }
        }
    }
    // then the best schedule without and with whole members, each timed as
    // a bundle runs (the chains side by side)
    bool any_small = false;
    for (const axlb_lattice *L : b->members)
        any_small = any_small || (long long)L->Nr * L->Nz <= WHOLE_MAX_NODES;
    if (any_small && rc == AXLB_OK) {
        b->tile = bt;
        b->blocks = bb;
        double per_mode[2] = {0.0, 0.0};
        for (int mode = 0; mode < 2 && rc == AXLB_OK; ++mode) {
            b->whole_max = mode ? WHOLE_MAX_NODES : 0;
            rc = build_worklist(b);
            if (rc == AXLB_OK) rc = bundle_launches(b, b->steps, 2);
            b->steps += 2;
            (void)hipEventRecord(e0, b->stream);
            if (rc == AXLB_OK) rc = bundle_launches(b, b->steps, steps_per_trial);
            b->steps += steps_per_trial;
            (void)hipEventRecord(e1, b->stream);
            float ms = 0.f;
            if (rc == AXLB_OK && (hipEventSynchronize(e1) != hipSuccess ||
                                  hipEventElapsedTime(&ms, e0, e1) != hipSuccess))
                rc = bfail(b, AXLB_EDEVICE, "autotune timing");
            per_mode[mode] = ms / steps_per_trial;
        }
        if (rc == AXLB_OK && per_mode[1] < per_mode[0]) bw = WHOLE_MAX_NODES;
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    // restore every member and the batch step count
    for (size_t m = 0; m < b->members.size(); ++m) {
        axlb_lattice *L = b->members[m];
        const size_t bytes = L->lay.pop_bytes + 2 * L->lay.lag_bytes;
        (void)hipMemcpyAsync(L->pop[0], keep[m], bytes, hipMemcpyDeviceToDevice, b->stream);
    }
    (void)hipStreamSynchronize(b->stream);
    release();
    b->steps = steps0;
    if (rc != AXLB_OK) {  // keep the schedule the batch had
        b->tile = tile0;
        b->blocks = blocks0;
        b->whole_max = whole0;
        (void)build_worklist(b);
        return rc;
    }
    b->tile = bt;
    b->blocks = bb;
    b->whole_max = bw;
    rc = build_worklist(b);
    if (rc != AXLB_OK) return rc;
    if (best_tile) *best_tile = bt;
    if (best_blocks) *best_blocks = bb;
    return AXLB_OK;
}

void axlb_batch_destroy(axlb_batch *b) {
    if (!b) return;
    (void)hipSetDevice(b->device);
    if (b->stream) (void)hipStreamSynchronize(b->stream);
    drop_batch_graphs(b);
    for (size_t m = 0; m < b->members.size(); ++m) {
        b->members[m]->stream = b->member_streams[m];
        b->members[m]->batched = false;
    }
    if (b->d_desc) (void)hipFree(b->d_desc);
    if (b->d_two) (void)hipFree(b->d_two);
    if (b->d_two_tiles) (void)hipFree(b->d_two_tiles);
    if (b->d_tiles) (void)hipFree(b->d_tiles);
    if (b->d_whole) (void)hipFree(b->d_whole);
    if (b->join_aux) (void)hipEventDestroy(b->join_aux);
    if (b->join) (void)hipEventDestroy(b->join);
    if (b->fork) (void)hipEventDestroy(b->fork);
    if (b->aux) (void)hipStreamDestroy(b->aux);
    if (b->side) (void)hipStreamDestroy(b->side);
    if (b->stream) (void)hipStreamDestroy(b->stream);
    delete b;
}

const char *axlb_batch_last_error(const axlb_batch *b) {
    return b ? b->err.c_str() : g_batch_error.c_str();
}

int axlb_step_each(axlb_lattice *const *lats, int n, long steps) {
    if (!lats || n <= 0 || steps < 0) return bfail(nullptr, AXLB_EINVAL, "bad arguments");
    for (long s = 0; s < steps; ++s)
        for (int m = 0; m < n; ++m) {
            if (!lats[m] || lats[m]->batched) return bfail(nullptr, AXLB_EINVAL, "bad member");
            const int rc = lattice_step_once(lats[m]);
            if (rc != AXLB_OK) return bfail(nullptr, rc, lats[m]->err);
        }
    return AXLB_OK;
}

}  // extern "C"
