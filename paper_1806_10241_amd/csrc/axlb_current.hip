// Time step with current-step derivatives (gfx950): the central differences
// of the geometric sources (eq. 4, 7, 9) take the output fields u_x, u_y,
// u_theta = psi/rho, T of the same step (after streaming, before the source
// half step), as the oracle's current-field mode does.  Those fields of a
// neighbour exist only once the neighbour has streamed, so this form needs
// two population buffers (pull from src, write dst): each workgroup streams
// its tile plus a one-node ring around it, keeps the four output fields of
// all of them in LDS, and then differences from LDS.  The ring nodes are
// streamed again by their own workgroups (reads that mostly hit L2); no
// lagged-field buffer is read or written (and so this form takes FP32 or
// binary16 storage, not the offset-encoded bfloat16).
#include "axlb_device.h"
#include "axlb_launch.h"
#include "axlb_node.h"

namespace axlb {

// Pull of node (i, j): through the plane addresses when every source is a
// fluid node, else with the boundary rules.
template <class S>
__device__ __forceinline__ void pull_node(const KParams &P, const Planes &A, const S *src, int i,
                                          int j, bool interior, float (&f)[9], float (&g)[5],
                                          float (&h)[5]) {
    if (interior)
        gather_planes<S>(A, ((unsigned)i * (unsigned)P.pitch + (unsigned)j) * (unsigned)sizeof(S),
                         f, g, h);
    else
        gather<S, MODE_AB, false>(P, src, nullptr, i, j, false, f, g, h);
}

// Output fields of a node into the LDS tile F[4][H][W] at (a, b).
template <int H, int W>
__device__ __forceinline__ void put_fields(float (&F)[4][H][W], int a, int b, const Moments &m) {
    const float ir = rcp(1.f + m.drho);
    F[0][a][b] = m.jx * ir;
    F[1][a][b] = m.jy * ir;
    F[2][a][b] = m.psi * ir;
    F[3][a][b] = m.dphi;
}

// Streams node (i, j) of src (or its periodic image along z) into the LDS
// cell (a, b); positions outside the fluid that are not a periodic image are
// left alone (their ghosts come from the wall and axis rules).
template <class S, int H, int W>
__device__ __forceinline__ void fill_cell(const KParams &P, const Planes &A, const S *src,
                                          float (&F)[4][H][W], int a, int b, int i, int j) {
    if ((unsigned)j >= (unsigned)P.Nr) return;
    if ((unsigned)i >= (unsigned)P.Nz) {
        if (kind_of(P, i < 0 ? Z_LO : Z_HI, FLOW) != PERIODIC) return;
        i += i < 0 ? P.Nz : -P.Nz;
        if ((unsigned)i >= (unsigned)P.Nz) return;
    }
    float f[9], g[5], h[5];
    pull_node<S>(P, A, src, i, j, interior_node(P, i, j), f, g, h);
    put_fields(F, a, b, moments(f, g, h));
}

// One step (STEP) or the reported fields (!STEP) of every node.
template <class S, int BX, int BY, bool STEP>
__global__ void __launch_bounds__(BX * BY) k_current(const KParams P, const Planes A,
                                                      const S *src, S *dst,
                                                      double *__restrict__ out) {
    constexpr int W = BX + 2, H = BY + 2, RING = 2 * BX + 2 * BY;
    __shared__ float F[4][H][W];
    int i, j;
    tile_of<BX, BY>(P, i, j);
    const int tx = (int)threadIdx.x % BX, ty = (int)threadIdx.x / BX;
    const int i0 = i - ty, j0 = j - tx;
    const bool live = i < P.Nz && j < P.Nr;
    const bool interior = live && interior_node(P, i, j);
    float f[9], g[5], h[5];
    Moments m{};
    if (live) {
        pull_node<S>(P, A, src, i, j, interior, f, g, h);
        m = moments(f, g, h);
        put_fields(F, ty + 1, tx + 1, m);
    } else {
        fill_cell<S>(P, A, src, F, ty + 1, tx + 1, i, j);  // periodic image beyond the domain
    }
    // the ring without its corners (the differences only look along the
    // axes): rows 0 and H-1, then columns 0 and W-1
    for (int t = (int)threadIdx.x; t < RING; t += BX * BY) {
        int a, b;
        if (t < 2 * BX) {
            a = t < BX ? 0 : H - 1;
            b = 1 + (t < BX ? t : t - BX);
        } else {
            const int u = t - 2 * BX;
            a = 1 + (u >> 1);
            b = (u & 1) ? W - 1 : 0;
        }
        fill_cell<S>(P, A, src, F, a, b, i0 - 1 + a, j0 - 1 + b);
    }
    __syncthreads();
    if (!live) return;
    float d[5];
    differences(P, TileSource<H, W>{F, ty + 1, tx + 1}, i, j, d);
    const float iy = rcp(P.r0 + (float)j + 0.5f);
    const Half Hs = half_step(P, iy, m.drho, m.jx, m.jy, m.psi, m.dphi, d);
    if (STEP) {
        collide_f(P, f, Hs);
        collide_adv(g, Hs.ux, Hs.uy, Hs.psi, Hs.psi, Hs.hSpsi, P.og12, P.og3, P.og4);
        collide_adv(h, Hs.ux, Hs.uy, P.Tref + Hs.dphi, Hs.dphi, Hs.hSphi, P.oh12, P.oh3, P.oh4);
        if (interior)
            scatter_planes<S, false>(
                A, local_offset(((unsigned)i * (unsigned)P.pitch + (unsigned)j) * (unsigned)sizeof(S)),
                i + P.row0, j, f, g, h, Lag4{});
        else
            scatter<S, MODE_AB, false>(P, dst, i, j, false, f, g, h, Lag4{});
    } else {
        const long long N = (long long)P.Nr * P.Nz, k = (long long)i * P.Nr + j;
        out[k] = 1.0 + (double)Hs.drho;
        out[N + k] = (double)Hs.uy;
        out[2 * N + k] = (double)Hs.ux;
        out[3 * N + k] = (double)(Hs.psi * Hs.irho);
        out[4 * N + k] = (double)P.Tref + (double)Hs.dphi;
    }
}

template <class S>
static hipError_t step_current_t(const KParams &P, int tile, const void *src, void *dst,
                                 hipStream_t st) {
    const S *a = (const S *)src;
    S *b = (S *)dst;
    const Planes A = step_planes(P, store_of<S>(), MODE_AB, src, dst, nullptr, nullptr);
    switch (tile) {
#define AXLB_CASE(id, bx, by)                                                                 \
    case id:                                                                                  \
        k_current<S, bx, by, true><<<dim3(((P.Nr + bx - 1) / bx) * ((P.Nz + by - 1) / by)), \
                                     dim3(bx * by), 0, st>>>(P, A, a, b, nullptr);            \
        break;
        AXLB_TILES(AXLB_CASE)
#undef AXLB_CASE
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

template <class S>
static hipError_t fields_current_t(const KParams &P, const void *src, double *out, hipStream_t st) {
    // reads only: the write planes are never used
    const Planes A = step_planes(P, store_of<S>(), MODE_AB, src, const_cast<void *>(src),
                                 nullptr, nullptr);
    k_current<S, 64, 4, false><<<dim3(((P.Nr + 63) / 64) * ((P.Nz + 3) / 4)), dim3(256), 0, st>>>(
        P, A, (const S *)src, nullptr, out);
    return hipGetLastError();
}

hipError_t launch_step_current(const KParams &P, int storage, int tile, const void *src,
                               void *dst, hipStream_t st) {
    if (storage == STORE_F16) return step_current_t<__half>(P, tile, src, dst, st);
    if (storage == STORE_BF16) return hipErrorInvalidValue;  // refused at lattice creation
    return step_current_t<float>(P, tile, src, dst, st);
}

hipError_t launch_fields_current(const KParams &P, int storage, const void *src, double *out,
                                 hipStream_t st) {
    if (storage == STORE_F16) return fields_current_t<__half>(P, src, out, st);
    if (storage == STORE_BF16) return hipErrorInvalidValue;
    return fields_current_t<float>(P, src, out, st);
}

}  // namespace axlb
