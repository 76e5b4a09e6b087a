// Two time steps per launch on two population buffers (gfx950), with the
// lagged derivatives of the single-step kernels.  A workgroup has one thread
// per cell of a CW x CH block: a tile of (CW - 2) x (CH - 2) nodes and the
// one-node ring around it.  Step t: every thread takes its cell from the
// state before t (populations and lagged fields in device memory) and keeps
// the post-collision populations and the half-step fields in LDS, rounded
// exactly as a store to device memory would round them.  A ring cell is
// computed again by the workgroup that owns it (the price of the fusion); a
// cell beyond a periodic z face holds the periodic image.  Step t + 1: the
// tile's threads take their nodes from LDS alone and write the state after
// t + 1.  The per-node arithmetic is the single-step kernels' (axlb_node.h),
// so the result equals two single steps bit for bit, while the state crosses
// HBM once per pair.  Interior nodes (all eight neighbours fluid) read
// device memory through the plane addresses of a two-buffer pull (Planes)
// and LDS through fixed stencil offsets; only nodes on the lattice's edge
// take the general boundary rules.
#include "axlb_device.h"
#include "axlb_launch.h"
#include "axlb_node.h"

namespace axlb {

// Cell block of a workgroup: one thread per cell; a wavefront holds two rows
// of 32 cells.  Every thread computes one cell of step t; the 30 x 22 tile
// of step t + 1 is 86% of them.  The block's LDS (19 population planes and
// 4 lagged-field planes, 70.7 KB in FP32) lets two workgroups, 24
// wavefronts, share a compute unit, as three 32 x 16 blocks did; the
// taller block recomputes less of its ring (1024 x 2048 FP32: 101.8 us
// per two steps against 104.8 us for 32 x 16).
constexpr int TWO_CW = 32, TWO_CH = 24;
constexpr int TWO_TW = TWO_CW - 2, TWO_TH = TWO_CH - 2;
// The batch kernel keeps 32 x 16 blocks (three per compute unit): its
// members are 48 to 512 nodes tall, and a taller block wastes more of its
// rows on them (256 uneven annuli: 24.7k MLUPS against 24.3k).
constexpr int BATCH_CH = 16, BATCH_TH = BATCH_CH - 2;

// The LDS block of post-collision populations as a population source for
// pull_all: node (i, j) sits in cell (i - i0 + 1, j - j0 + 1).  With offset
// encoding the cell's own lagged fields (LDS block Lg) decode its slots.
template <class S, int H, int W>
struct TilePops {
    const S (&A)[NPOP][H][W];
    const float (&Lg)[NLAG][H][W];
    int i0, j0;
    __device__ __forceinline__ float operator()(int p, int i, int j) const {
        const int a = i - i0 + 1, b = j - j0 + 1;
        float v = Conv<S>::ld(&A[p][a][b]);
        if constexpr (kEnc<S>)
            v = v + plane_off<false>(p, Lag4{Lg[0][a][b], Lg[1][a][b], Lg[2][a][b], Lg[3][a][b]});
        return v;
    }
};

// Pull of population Q of distribution FLD from the LDS block for an
// interior node in cell (a, b): the post-collision value of the neighbour
// x - e_Q (two-buffer convention, plane Q), decoded with that neighbour's
// lagged fields.
template <class S, int FLD, int Q, int H, int W>
__device__ __forceinline__ float pull_lds(const S (&A)[NPOP][H][W], const float (&Lg)[NLAG][H][W],
                                          int a, int b) {
    using L = Lat<FLD>;
    const int sa = a - L::ex(Q), sb = b - L::ey(Q);
    float v = Conv<S>::ld(&A[L::OFF + Q][sa][sb]);
    if constexpr (kEnc<S>)
        v = v + pop_off<FLD>(Q, Lag4{Lg[0][sa][sb], Lg[1][sa][sb], Lg[2][sa][sb], Lg[3][sa][sb]});
    return v;
}

template <class S, int H, int W>
__device__ __forceinline__ void pull_lds_all(const S (&A)[NPOP][H][W],
                                             const float (&Lg)[NLAG][H][W], int a, int b,
                                             float (&f)[9], float (&g)[5], float (&h)[5]) {
    f[0] = pull_lds<S, FLOW, 0>(A, Lg, a, b);
    f[1] = pull_lds<S, FLOW, 1>(A, Lg, a, b);
    f[2] = pull_lds<S, FLOW, 2>(A, Lg, a, b);
    f[3] = pull_lds<S, FLOW, 3>(A, Lg, a, b);
    f[4] = pull_lds<S, FLOW, 4>(A, Lg, a, b);
    f[5] = pull_lds<S, FLOW, 5>(A, Lg, a, b);
    f[6] = pull_lds<S, FLOW, 6>(A, Lg, a, b);
    f[7] = pull_lds<S, FLOW, 7>(A, Lg, a, b);
    f[8] = pull_lds<S, FLOW, 8>(A, Lg, a, b);
    g[0] = pull_lds<S, SWIRL, 0>(A, Lg, a, b);
    g[1] = pull_lds<S, SWIRL, 1>(A, Lg, a, b);
    g[2] = pull_lds<S, SWIRL, 2>(A, Lg, a, b);
    g[3] = pull_lds<S, SWIRL, 3>(A, Lg, a, b);
    g[4] = pull_lds<S, SWIRL, 4>(A, Lg, a, b);
    h[0] = pull_lds<S, THERMAL, 0>(A, Lg, a, b);
    h[1] = pull_lds<S, THERMAL, 1>(A, Lg, a, b);
    h[2] = pull_lds<S, THERMAL, 2>(A, Lg, a, b);
    h[3] = pull_lds<S, THERMAL, 3>(A, Lg, a, b);
    h[4] = pull_lds<S, THERMAL, 4>(A, Lg, a, b);
}

// Two steps of the tile whose first node is (i0, j0), with the workgroup's
// LDS block.  A: plane addresses of the launch (populations of src, the
// lagged fields of Mprev, and the write planes of dst and Mnext); src and
// Mprev also serve the general path of the lattice's edge cells.  Every
// thread reaches the barrier and the end (no early return), so a workgroup
// may call it for one tile after another.
template <class S, int H>
__device__ __forceinline__ void step_two_tile(const KParams &P, const Planes &A, const S *src,
                                              const char *__restrict__ Mprev, int i0, int j0,
                                              S (&pop)[NPOP][H][TWO_CW],
                                              float (&lag)[NLAG][H][TWO_CW]) {
    constexpr int W = TWO_CW, TH = H - 2;
    const int a = (int)threadIdx.x / W, b = (int)threadIdx.x % W;

    // step t for this thread's cell
    {
        int ci = i0 - 1 + a;
        const int cj = j0 - 1 + b;
        bool live = (unsigned)cj < (unsigned)P.Nr;
        if (live && (unsigned)ci >= (unsigned)P.Nz) {
            // beyond a z face: the periodic image, or nothing
            live = kind_of(P, ci < 0 ? Z_LO : Z_HI, FLOW) == PERIODIC;
            ci += ci < 0 ? P.Nz : -P.Nz;
            live = live && (unsigned)ci < (unsigned)P.Nz;
        }
        if (live) {
            const bool interior = interior_node(P, ci, cj);
            float f[9], g[5], h[5], d[5];
            if (interior) {
                const unsigned cn = (unsigned)ci * (unsigned)P.pitch + (unsigned)cj;
                gather_planes<S>(A, cn * (unsigned)sizeof(S), f, g, h);
                if constexpr (kEnc<S>) decode_planes<S>(P, A, cn, f, g, h);
            } else {
                gather<S, MODE_AB>(P, src, Mprev, ci, cj, false, f, g, h);
            }
            derivatives<S>(P, Mprev, ci, cj, interior, d);
            const Half Hs = relax_node(P, cj, f, g, h, d);
            const unsigned w0 = node_word(f, g, h, ci + P.row0, cj);
            const Lag4 Ln = lag_stored<S>(Hs.ux, Hs.uy, Hs.psi * Hs.irho, Hs.dphi);
            float ef[9], eg[5], eh[5];
            encode<kEnc<S>>(f, g, h, Ln, ef, eg, eh);
#pragma unroll
            for (int p = 0; p < 9; ++p) Conv<S>::st(&pop[p][a][b], ef[p], slot_word(w0, p));
#pragma unroll
            for (int p = 0; p < 5; ++p) {
                Conv<S>::st(&pop[GOFF + p][a][b], eg[p], slot_word(w0, GOFF + p));
                Conv<S>::st(&pop[HOFF + p][a][b], eh[p], slot_word(w0, HOFF + p));
            }
            lag[0][a][b] = Ln.ux;
            lag[1][a][b] = Ln.uy;
            lag[2][a][b] = Ln.ut;
            lag[3][a][b] = Ln.dT;
        }
    }
    __syncthreads();

    // step t + 1 for the tile's own nodes, from LDS
    const int i = i0 - 1 + a, j = j0 - 1 + b;
    if (a >= 1 && a <= TH && b >= 1 && b <= TWO_TW && i < P.Nz && j < P.Nr) {
        float f[9], g[5], h[5], d[5];
        if (interior_node(P, i, j)) {
            pull_lds_all<S>(pop, lag, a, b, f, g, h);
            d[0] = 0.5f * (lag[1][a + 1][b] - lag[1][a - 1][b]);
            d[1] = 0.5f * (lag[0][a][b + 1] - lag[0][a][b - 1]);
            d[2] = 0.5f * (lag[1][a][b + 1] - lag[1][a][b - 1]);
            d[3] = 0.5f * (lag[2][a][b + 1] - lag[2][a][b - 1]);
            d[4] = 0.5f * (lag[3][a][b + 1] - lag[3][a][b - 1]);
        } else {
            pull_all<false>(P, TilePops<S, H, W>{pop, lag, i0, j0}, i, j, f, g, h);
            differences(P, TileSource<H, W>{lag, a, b}, i, j, d);
        }
        const Half Hs = relax_node(P, j, f, g, h, d);
        using F = LagFmt<S>;
        const unsigned n = (unsigned)i * (unsigned)P.pitch + (unsigned)j;
        const unsigned so = local_offset(n * (unsigned)sizeof(S)), sov = local_offset(n * F::VB);
        const unsigned so4 = local_offset(n * 4u);
        scatter_planes<S>(A, so, i + P.row0, j, f, g, h,
                          lag_stored<S>(Hs.ux, Hs.uy, Hs.psi * Hs.irho, Hs.dphi));
        gstore(A.lwr[0], sov, F::enc(Hs.ux));
        gstore(A.lwr[1], sov, F::enc(Hs.uy));
        gstore(A.lwr[2], sov, F::enc(Hs.psi * Hs.irho));
        gstore(A.lwr[3], so4, Hs.dphi);
    }
}

// Workgroups of a two-step launch over a gx x gy grid of tiles: the tiles
// on the rim of the grid (which hold the lattice's edge nodes and run the
// general boundary code) come first, padded to a multiple of 8 so that the
// inner tiles after them start on XCD 0; the inner tiles are dealt to the
// XCDs in 8 contiguous bands, as tile_of deals a single-step grid.  With
// the boundary code confined to the first workgroups, the instruction
// cache of every compute unit holds only the inner path for the rest of
// the launch: at 1024 x 2048 (FP32) the two steps take 104.4 us instead of
// 113.0 us in one banded order.
__host__ __device__ inline int two_rim_tiles(int gx, int gy) {
    return (gx <= 2 || gy <= 2) ? 0 : 2 * gx + 2 * (gy - 2);
}
__host__ __device__ inline int two_grid_blocks(int gx, int gy) {
    const int nE = two_rim_tiles(gx, gy);
    return nE == 0 ? gx * gy : ((nE + 7) & ~7) + (gx - 2) * (gy - 2);
}
// Tile (tx, ty) of workgroup bid; false for a padding workgroup.
__device__ inline bool two_tile_of(int gx, int gy, int bid, int &tx, int &ty) {
    const int nE = two_rim_tiles(gx, gy);
    if (nE == 0) {  // small grids: every tile is on the rim; XCD bands
        const int nb = gx * gy, xcd = bid & 7, k = bid >> 3, q = nb >> 3, r = nb & 7;
        const int t = xcd * q + (xcd < r ? xcd : r) + k;
        tx = t % gx;
        ty = t / gx;
        return true;
    }
    const int nEp = (nE + 7) & ~7;
    if (bid < nEp) {
        if (bid >= nE) return false;
        if (bid < 2 * gx) {  // first and last row of tiles
            tx = bid % gx;
            ty = bid < gx ? 0 : gy - 1;
        } else {  // first and last column, between them
            const int e = bid - 2 * gx;
            tx = e < gy - 2 ? 0 : gx - 1;
            ty = 1 + (e < gy - 2 ? e : e - (gy - 2));
        }
        return true;
    }
    const int b = bid - nEp, nI = (gx - 2) * (gy - 2);
    const int xcd = b & 7, k = b >> 3, q = nI >> 3, r = nI & 7;
    const int t = xcd * q + (xcd < r ? xcd : r) + k;
    tx = 1 + t % (gx - 2);
    ty = 1 + t / (gx - 2);
    return true;
}

template <class S>
__global__ void __launch_bounds__(TWO_CW *TWO_CH) k_step_two(const KParams P, const Planes A,
                                                              const S *src,
                                                              const char *__restrict__ Mprev) {
    __shared__ S pop[NPOP][TWO_CH][TWO_CW];
    __shared__ float lag[NLAG][TWO_CH][TWO_CW];
    const int gx = (P.Nr + TWO_TW - 1) / TWO_TW, gy = (P.Nz + TWO_TH - 1) / TWO_TH;
    int tx, ty;
    if (!two_tile_of(gx, gy, (int)blockIdx.x, tx, ty)) return;  // padding: the whole workgroup
    step_two_tile<S, TWO_CH>(P, A, src, Mprev, ty * TWO_TH, tx * TWO_TW, pop, lag);
}

// Two steps of many lattices (a batch of two-buffer members): one
// workgroup per work-list entry (member, tile index within the member),
// the entries dealt to the 8 XCDs in 8 contiguous chunks so that a
// member's tiles share an L2.  A member reads buffer pair
// cur0 ^ phase (its state when the batch was made, flipped once per
// launch).
// Six waves per SIMD (three workgroups per CU, as the LDS allows) need at
// most 80 VGPRs; left alone the compiler takes 84 for the parameters it
// reads from the descriptors.
template <class S>
__global__ void __launch_bounds__(TWO_CW *BATCH_CH, 6) k_step_two_batch(const TwoDesc *__restrict__ D,
                                                                    const int2 *__restrict__ tile_inst,
                                                                    int t0, int ntiles, int phase) {
    __shared__ S pop[NPOP][BATCH_CH][TWO_CW];
    __shared__ float lag[NLAG][BATCH_CH][TWO_CW];
    const int G = gridDim.x, bk = blockIdx.x;
    const int xcd = bk & 7, k = bk >> 3;
    // chunk sizes follow the block counts per XCD, so that with one block
    // per entry every block takes exactly one
    const int nbx = (G >> 3) + (xcd < (G & 7) ? 1 : 0);
    const int q = ntiles >> 3, r = ntiles & 7;
    const int lo = t0 + xcd * q + (xcd < r ? xcd : r);
    const int hi = lo + q + (xcd < r ? 1 : 0);
    for (int t = lo + k; t < hi; t += nbx) {
        const int2 e = tile_inst[t];
        const TwoDesc *d = D + e.x;
        const int c = d->cur0 ^ phase;
        const int local = e.y;
        step_two_tile<S, BATCH_CH>(d->P, d->pl[c], static_cast<const S *>(d->src[c]), d->lag[c],
                                   (local / d->gx) * BATCH_TH, (local % d->gx) * TWO_TW, pop, lag);
        __syncthreads();  // the LDS block is refilled by the next entry
    }
}

template <class S>
static hipError_t step_two_t(const KParams &P, const void *src, void *dst, const char *Mprev,
                             char *Mnext, hipStream_t st) {
    const int gx = (P.Nr + TWO_TW - 1) / TWO_TW, gy = (P.Nz + TWO_TH - 1) / TWO_TH;
    const Planes A = step_planes(P, store_of<S>(), MODE_AB, src, dst, Mprev, Mnext);
    k_step_two<S><<<dim3(two_grid_blocks(gx, gy)), dim3(TWO_CW * TWO_CH), 0, st>>>(
        P, A, (const S *)src, Mprev);
    return hipGetLastError();
}

void two_batch_tile_shape(int *tw, int *th) {
    *tw = TWO_TW;
    *th = BATCH_TH;
}

hipError_t launch_step_two_batch(int storage, const TwoDesc *D, const int2 *tiles, int t0,
                                 int ntiles, int phase, hipStream_t st) {
    const int blocks = ntiles < 8 ? 8 : ntiles;  // every XCD chunk needs a block
    const dim3 grid(blocks), block(TWO_CW * BATCH_CH);
    if (storage == STORE_F16)
        k_step_two_batch<__half><<<grid, block, 0, st>>>(D, tiles, t0, ntiles, phase);
    else if (storage == STORE_BF16)
        k_step_two_batch<__hip_bfloat16><<<grid, block, 0, st>>>(D, tiles, t0, ntiles, phase);
    else
        k_step_two_batch<float><<<grid, block, 0, st>>>(D, tiles, t0, ntiles, phase);
    return hipGetLastError();
}

hipError_t launch_step_two(const KParams &P, int storage, const void *src, void *dst,
                           const char *Mprev, char *Mnext, hipStream_t st) {
    if (storage == STORE_F16) return step_two_t<__half>(P, src, dst, Mprev, Mnext, st);
    if (storage == STORE_BF16) return step_two_t<__hip_bfloat16>(P, src, dst, Mprev, Mnext, st);
    return step_two_t<float>(P, src, dst, Mprev, Mnext, st);
}

}  // namespace axlb
