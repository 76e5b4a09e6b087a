// Two time steps per launch on two population buffers (gfx950), with the
// lagged derivatives of the single-step kernels.  A workgroup owns a tile of
// TWO_BX x TWO_BY nodes.  It first takes the tile and a one-node ring around
// it through step t, reading the populations and lagged fields of the state
// before t from device memory, and keeps the post-collision populations and
// the half-step fields of every cell in LDS, rounded exactly as a store to
// device memory would round them.  The ring cells are computed again by the
// workgroups that own them (the price of the fusion); a cell beyond a
// periodic z face holds the periodic image.  Then it takes its tile through
// step t + 1 from LDS alone and writes the state after t + 1.  The per-node
// arithmetic is the single-step kernels' (axlb_node.h), so the result equals
// two single steps bit for bit, while the state crosses HBM once per pair.
// Interior cells read, and the tile writes, through the plane addresses of
// a two-buffer pull (Planes).
#include "axlb_device.h"
#include "axlb_launch.h"
#include "axlb_node.h"

namespace axlb {

constexpr int TWO_BX = 32, TWO_BY = 8;

// The LDS tile of post-collision populations as a population source for
// pull_all: node (i, j) sits in cell (i - i0 + 1, j - j0 + 1).
template <class S, int H, int W>
struct TilePops {
    const S (&A)[NPOP][H][W];
    int i0, j0;
    __device__ __forceinline__ float operator()(int p, int i, int j) const {
        return Conv<S>::ld(&A[p][i - i0 + 1][j - j0 + 1]);
    }
};

template <class S, int BX, int BY>
__global__ void __launch_bounds__(BX * BY) k_step_two(const KParams P, const Planes A,
                                                       const S *src, S *dst,
                                                       const char *__restrict__ Mprev,
                                                       char *__restrict__ Mnext) {
    constexpr int W = BX + 2, H = BY + 2, NC = W * H;
    __shared__ S pop[NPOP][H][W];
    __shared__ float lag[NLAG][H][W];
    int i, j;
    tile_of<BX, BY>(P, i, j);
    const int tx = (int)threadIdx.x % BX, ty = (int)threadIdx.x / BX;
    const int i0 = i - ty, j0 = j - tx;

    // step t for every fluid cell of the tile and its ring: the interior
    // nodes row by row (coalesced, pass 0), then the lattice's edge nodes
    // column by column (pass 1), so that an edge column's cells share a few
    // wavefronts and only those run the boundary code
    for (int pass = 0; pass < 2; ++pass)
    for (int c = (int)threadIdx.x; c < NC; c += BX * BY) {
        const int a = pass == 0 ? c / W : c % H, b = pass == 0 ? c % W : c / H;
        int ci = i0 - 1 + a;
        const int cj = j0 - 1 + b;
        if ((unsigned)cj >= (unsigned)P.Nr) continue;
        if ((unsigned)ci >= (unsigned)P.Nz) {
            if (kind_of(P, ci < 0 ? Z_LO : Z_HI, FLOW) != PERIODIC) continue;
            ci += ci < 0 ? P.Nz : -P.Nz;
            if ((unsigned)ci >= (unsigned)P.Nz) continue;
        }
        const bool interior = interior_node(P, ci, cj);
        if (interior != (pass == 0)) continue;
        float f[9], g[5], h[5], d[5];
        if (interior)
            gather_planes<S>(A, ((unsigned)ci * (unsigned)P.pitch + (unsigned)cj) *
                                    (unsigned)sizeof(S), f, g, h);
        else
            gather<S, MODE_AB>(P, src, ci, cj, false, f, g, h);
        derivatives<S>(P, Mprev, ci, cj, interior, d);
        const Half Hs = relax_node(P, cj, f, g, h, d);
#pragma unroll
        for (int q = 0; q < 9; ++q) Conv<S>::st(&pop[q][a][b], f[q], skey(ci, cj, q));
#pragma unroll
        for (int q = 0; q < 5; ++q) {
            Conv<S>::st(&pop[GOFF + q][a][b], g[q], skey(ci, cj, GOFF + q));
            Conv<S>::st(&pop[HOFF + q][a][b], h[q], skey(ci, cj, HOFF + q));
        }
        lag[0][a][b] = lag_round<S>(0, Hs.ux);
        lag[1][a][b] = lag_round<S>(1, Hs.uy);
        lag[2][a][b] = lag_round<S>(2, Hs.psi * Hs.irho);
        lag[3][a][b] = lag_round<S>(3, Hs.dphi);
    }
    __syncthreads();
    if (i >= P.Nz || j >= P.Nr) return;

    // step t + 1 for the tile's own node, from LDS
    float f[9], g[5], h[5], d[5];
    pull_all<false>(P, TilePops<S, H, W>{pop, i0, j0}, i, j, f, g, h);
    differences(P, TileSource<H, W>{lag, ty + 1, tx + 1}, i, j, d);
    const Half Hs = relax_node(P, j, f, g, h, d);
    const unsigned n = (unsigned)i * (unsigned)P.pitch + (unsigned)j;
    scatter_planes<S>(A, local_offset(n * (unsigned)sizeof(S)), i, j, f, g, h);
    lag_st<S>(Mnext, 0, P.plane, n, Hs.ux);
    lag_st<S>(Mnext, 1, P.plane, n, Hs.uy);
    lag_st<S>(Mnext, 2, P.plane, n, Hs.psi * Hs.irho);
    lag_st<S>(Mnext, 3, P.plane, n, Hs.dphi);
}

template <class S>
static hipError_t step_two_t(const KParams &P, const void *src, void *dst, const char *Mprev,
                             char *Mnext, hipStream_t st) {
    const int gx = (P.Nr + TWO_BX - 1) / TWO_BX, gy = (P.Nz + TWO_BY - 1) / TWO_BY;
    const Planes A = step_planes(P, store_of<S>(), MODE_AB, src, dst, Mprev, Mnext);
    k_step_two<S, TWO_BX, TWO_BY><<<dim3(gx * gy), dim3(TWO_BX * TWO_BY), 0, st>>>(
        P, A, (const S *)src, (S *)dst, Mprev, Mnext);
    return hipGetLastError();
}

hipError_t launch_step_two(const KParams &P, int storage, const void *src, void *dst,
                           const char *Mprev, char *Mnext, hipStream_t st) {
    if (storage == STORE_F16) return step_two_t<__half>(P, src, dst, Mprev, Mnext, st);
    if (storage == STORE_BF16) return step_two_t<__hip_bfloat16>(P, src, dst, Mprev, Mnext, st);
    return step_two_t<float>(P, src, dst, Mprev, Mnext, st);
}

}  // namespace axlb
