// HIP kernels (gfx950) of the axisymmetric cascaded central-moment LB step
// of arXiv 1806.10241, Section 2: one fused, memory-bound pass per node over
// the D2Q9 f, the D2Q5 g (psi = rho u_theta) and the D2Q5 h (T).
//
// Data layout in HBM (structure of arrays, r fastest, rows padded to
// `pitch`): 19 population planes pop[q][iz][ir] holding shifted populations
// f - w_q (rho_0 = 1), g, and h - w_q T_ref, in FP32, binary16 or bfloat16,
// and two blocks (time levels) of lagged derivative fields, each three
// velocity planes (FP32 with FP32 populations, scaled binary16 with 16-bit
// ones) and one FP32 temperature plane.  All arithmetic is FP32; reductions
// are FP64.
//
// Streaming layouts:
//  * AA (one buffer, in place).  Even phase: node n reads its own slots
//    A[q][n] = f_q(n) and writes f*_q(n) to A[opp q][n].  Odd phase: node n
//    reads f_q(n) = A[opp q][n - e_q] and writes f*_q(n) to A[q][n + e_q].
//    In both phases every node reads and writes the same 19 slots, so the
//    update is race-free without a second buffer; all boundary rules live in
//    the odd phase.
//  * AB (two buffers): pull f_q(n) = src[q][n - e_q], write dst[q][n].
#include "axlb_device.h"
#include "axlb_launch.h"
#include "axlb_node.h"
#include "axlb_reduce.h"

namespace axlb {

// Edge nodes per edge workgroup: one wavefront's worth whatever the tile
// shape, so that the slow, uncoalesced boundary code is spread over more
// compute units (the other wavefronts of an edge workgroup exit at once).
constexpr int EDGE_PER_BLOCK = 64;

// Whether a step of slot convention `mode` runs the lattice's edge nodes in
// workgroups of their own.
template <class S>
__host__ __device__ constexpr bool split_edges(int mode) {
    return mode != MODE_AA_EVEN || sizeof(S) == 2;
}

// One time step for every node of one lattice.  Where boundary rules apply
// to the streaming (AA odd phase, AB), the first workgroups take
// EDGE_PER_BLOCK consecutive edge nodes each (their count rounded up to a
// multiple of 8, so that the hardware deals them to all eight XCDs and the
// tiles after them keep their XCD alignment), and the tile workgroups skip
// the edge nodes; the AA even phase streams within each node's own slots, so its
// tiles take every node, except with 16-bit storage: offset-encoded bfloat16
// finds the writer of an edge node's slots through the boundary rules (that
// code in every tile workgroup cost 10 us of 51 per even step at 1024 x 2048),
// and binary16's even step also runs faster without its edge code in the
// tiles (38.9 us against 40.6 us); FP32's runs slower (59.7 against 58.8 us).
// Tile workgroups are XCD-remapped as in tile_of
// and reach every value through the launch's plane addresses (Planes); edge
// workgroups take the general per-node path.
template <class S, int MODE, int BX, int BY>
__global__ void __launch_bounds__(BX * BY) k_step(const KParams P, const Planes A,
                                                   const S *src, S *dst,
                                                   const char *__restrict__ Mprev,
                                                   char *__restrict__ Mnext) {
    constexpr bool SPLIT = split_edges<S>(MODE);
    const int gx = (P.Nr + BX - 1) / BX;
    const int ne = SPLIT ? edge_blocks(P.Nr, P.Nz, EDGE_PER_BLOCK) : 0;
    const int b = (int)blockIdx.x;
    if (SPLIT && b < ne) {
        if ((int)threadIdx.x >= EDGE_PER_BLOCK) return;
        const int e = b * EDGE_PER_BLOCK + (int)threadIdx.x;
        if (e >= edge_count(P.Nr, P.Nz)) return;
        int i, j;
        edge_node(P, e, i, j);
        update_node<S, MODE>(P, src, dst, Mprev, Mnext, i, j, false);
        return;
    }
    const int nb = (int)gridDim.x - ne, bt = b - ne;
    const int xcd = bt & 7, k = bt >> 3, q = nb >> 3, r = nb & 7;
    const int u = xcd * q + (xcd < r ? xcd : r) + k;
    const int j = (u % gx) * BX + (int)threadIdx.x % BX;
    const int i = (u / gx) * BY + (int)threadIdx.x / BX;
    if (SPLIT) {
        if (!interior_node(P, i, j)) return;  // edge nodes and the ragged tail
        update_planes<S>(P, A, i, j, true);
    } else {
        if (i >= P.Nz || j >= P.Nr) return;
        update_planes<S>(P, A, i, j, interior_node(P, i, j));
    }
}

// The fields the next step's collision sees, without changing the state:
// out = [rho, u_r, u_z, u_theta, T] planes of Nz*Nr doubles.
template <class S, int MODE>
__global__ void __launch_bounds__(TX * TY) k_fields(const KParams P, const S *src,
                                                     const char *__restrict__ Mprev,
                                                     double *__restrict__ out) {
    int i, j;
    tile_of<TX, TY>(P, i, j);
    if (i >= P.Nz || j >= P.Nr) return;
    const bool interior = interior_node(P, i, j);
    float f[9], g[5], h[5];
    gather<S, MODE>(P, src, Mprev, i, j, interior, f, g, h);
    const Moments m = moments(f, g, h);
    float d[5];
    derivatives<S>(P, Mprev, i, j, interior, d);
    const float iy = rcp(P.r0 + (float)j + 0.5f);
    const Half H = half_step(P, iy, m.drho, m.jx, m.jy, m.psi, m.dphi, d);
    const long long N = (long long)P.Nr * P.Nz, k = (long long)i * P.Nr + j;
    out[k] = 1.0 + (double)H.drho;
    out[N + k] = (double)H.uy;
    out[2 * N + k] = (double)H.ux;
    out[3 * N + k] = (double)(H.psi * H.irho);
    out[4 * N + k] = (double)P.Tref + (double)H.dphi;
}

// Equilibria of the given fields (their central moments are the Maxwellian
// ones: a product of the 1-D weights {1 - cs2 - u^2, (cs2 + u^2 +- u)/2}
// per axis for D2Q9; the D2Q5 weights of s (cs2 + u_a^2 +- u_a)/2 and the
// remainder at rest), computed in FP64 and stored shifted.  AA stores them
// as the even phase would (post-collision in plane opp q), AB in plane q.
// The lagged fields start as the given fields; ENC stores the populations
// offset-encoded with them (bfloat16 with lagged derivatives).
__device__ __forceinline__ double w1(int e, double u) {
    const double c = 1.0 / 3.0 + u * u;
    return e == 0 ? 1.0 - c : 0.5 * (c + e * u);
}

template <class S, bool AA, bool ENC>
__global__ void __launch_bounds__(TX * TY) k_init(const KParams P, S *A,
                                                   const double *__restrict__ in, char *M) {
    int i, j;
    tile_of<TX, TY>(P, i, j);
    if (i >= P.Nz || j >= P.Nr) return;
    const long long N = (long long)P.Nr * P.Nz, k = (long long)i * P.Nr + j;
    const long long n = (long long)i * P.pitch + j;
    const double rho = in[k], ur = in[N + k], uz = in[2 * N + k], uth = in[3 * N + k];
    const double T = in[4 * N + k];
    const double Tref = (double)P.Tref;
    const Lag4 L0 = lag_stored<S>((float)uz, (float)ur, (float)uth, (float)(T - Tref));
#pragma unroll
    for (int q = 0; q < 9; ++q) {
        const int ex = Lat<FLOW>::ex(q), ey = Lat<FLOW>::ey(q);
        const double feq = rho * w1(ex, uz) * w1(ey, ur);
        const double w = w1(ex, 0.0) * w1(ey, 0.0);
        const int slot = AA ? Lat<FLOW>::opp(q) : q;
        const float x = (float)(feq - w);
        float e = x;
        if (ENC) e = x - pop_off<FLOW>(q, L0);
        Conv<S>::st(A + slot * P.plane + n, e, sr_single(x, skey(i + P.row0, j, q)));
    }
    const double psi = rho * uth;
    double ge[5], he[5];
    ge[1] = 0.5 * psi * (1.0 / 3.0 + uz * uz + uz);
    ge[3] = 0.5 * psi * (1.0 / 3.0 + uz * uz - uz);
    ge[2] = 0.5 * psi * (1.0 / 3.0 + ur * ur + ur);
    ge[4] = 0.5 * psi * (1.0 / 3.0 + ur * ur - ur);
    ge[0] = psi - (ge[1] + ge[2] + ge[3] + ge[4]);
    he[1] = 0.5 * T * (1.0 / 3.0 + uz * uz + uz);
    he[3] = 0.5 * T * (1.0 / 3.0 + uz * uz - uz);
    he[2] = 0.5 * T * (1.0 / 3.0 + ur * ur + ur);
    he[4] = 0.5 * T * (1.0 / 3.0 + ur * ur - ur);
    he[0] = T - (he[1] + he[2] + he[3] + he[4]);
#pragma unroll
    for (int q = 0; q < 5; ++q) {
        const double w = q == 0 ? 1.0 / 3.0 : 1.0 / 6.0;
        const int slot = AA ? Lat<SWIRL>::opp(q) : q;
        const float xg = (float)ge[q], xh = (float)(he[q] - w * Tref);
        float eg = xg, eh = xh;
        if (ENC) {
            eg = xg - pop_off<SWIRL>(q, L0);
            eh = xh - pop_off<THERMAL>(q, L0);
        }
        const int gi = i + P.row0;
        Conv<S>::st(A + (GOFF + slot) * P.plane + n, eg, sr_single(xg, skey(gi, j, GOFF + q)));
        Conv<S>::st(A + (HOFF + slot) * P.plane + n, eh, sr_single(xh, skey(gi, j, HOFF + q)));
    }
    lag_st<S>(M, 0, P.plane, n, (float)uz);
    lag_st<S>(M, 1, P.plane, n, (float)ur);
    lag_st<S>(M, 2, P.plane, n, (float)uth);
    lag_st<S>(M, 3, P.plane, n, (float)(T - Tref));
}

// ----------------------------------------------------------------------------
// FP64 reductions.  Block sums are formed with wavefront shuffles and LDS in
// a fixed order (block_sum), and the per-block partials are summed by one
// workgroup in block order, so the result does not depend on scheduling.

// Residual partials: for the four fields u_r, u_z, u_theta, T (planes 1..4
// of `fld`) the sums of (q - snap)^2 and q^2, plus the count of non-finite
// values.
__global__ void __launch_bounds__(RED_THREADS) k_residual_partial(const double *__restrict__ fld,
                                                                  const double *__restrict__ snap,
                                                                  long long N, double *part) {
    __shared__ double sh[9 * (RED_THREADS / 64)];
    double v[9];
#pragma unroll
    for (int c = 0; c < 9; ++c) v[c] = 0.0;
    for (long long k = (long long)blockIdx.x * RED_THREADS + threadIdx.x; k < N;
         k += (long long)gridDim.x * RED_THREADS) {
#pragma unroll
        for (int c = 0; c < 4; ++c) {
            const double q = fld[(c + 1) * N + k], s = snap[c * N + k];
            v[2 * c] += (q - s) * (q - s);
            v[2 * c + 1] += q * q;
        }
        if (!isfinite(fld[k]) || !isfinite(fld[N + k]) || !isfinite(fld[2 * N + k]) ||
            !isfinite(fld[3 * N + k]) || !isfinite(fld[4 * N + k]))
            v[8] += 1.0;
    }
    block_sum<9>(v, sh);
    if (threadIdx.x == 0)
        for (int c = 0; c < 9; ++c) part[blockIdx.x * 9 + c] = v[c];
}

__global__ void __launch_bounds__(RED_THREADS) k_sum_partials(const double *part, int nblocks,
                                                              int width, double *out) {
    __shared__ double sh[16 * (RED_THREADS / 64)];
    // width <= 16 columns
    double v[16];
#pragma unroll
    for (int c = 0; c < 16; ++c) v[c] = 0.0;
    for (int b = threadIdx.x; b < nblocks; b += RED_THREADS)
        for (int c = 0; c < width; ++c) v[c] += part[b * width + c];
    block_sum<16>(v, sh);
    if (threadIdx.x == 0)
        for (int c = 0; c < width; ++c) out[c] = v[c];
}

// Wall gradients of T for the Nusselt numbers: one-sided second-order value
// (-8 T_w + 9 T_1 - T_2)/3 along the inward normal of each half-way wall.
// Annulus: summed over the Nz rows at the inner and outer wall.  Cylinder:
// r-weighted sums over the Nr columns at the bottom and top lids.
__global__ void __launch_bounds__(RED_THREADS) k_nusselt(const double *__restrict__ T, int Nr,
                                                         int Nz, int cylinder, double r0,
                                                         double Ta, double Tb, double *out) {
    __shared__ double sh[2 * (RED_THREADS / 64)];
    double v[2] = {0.0, 0.0};
    if (!cylinder) {
        for (int i = threadIdx.x; i < Nz; i += RED_THREADS) {
            const double *row = T + (long long)i * Nr;
            v[0] += (-8.0 * Ta + 9.0 * row[0] - row[1]) / 3.0;
            v[1] -= (-8.0 * Tb + 9.0 * row[Nr - 1] - row[Nr - 2]) / 3.0;
        }
    } else {
        for (int j = threadIdx.x; j < Nr; j += RED_THREADS) {
            const double y = r0 + j + 0.5;
            v[0] += y * (-8.0 * Ta + 9.0 * T[j] - T[(long long)Nr + j]) / 3.0;
            v[1] -= y * (-8.0 * Tb + 9.0 * T[(long long)(Nz - 1) * Nr + j] -
                         T[(long long)(Nz - 2) * Nr + j]) / 3.0;
        }
    }
    block_sum<2>(v, sh);
    if (threadIdx.x == 0) {
        out[0] = v[0];
        out[1] = v[1];
    }
}

// Stream function of the meridian flow, one thread per row i: psi(i, j) =
// -sum_{k <= j} y_k u_z(i, k) (d psi / d y = -y u_x by the midpoint rule
// over the node cells, 0 on the inner face), and the row's smallest and
// largest value (row_range[2 i], row_range[2 i + 1]).
__global__ void __launch_bounds__(RED_THREADS) k_stream(const double *__restrict__ uz, int Nr,
                                                        int Nz, double r0, double *psi,
                                                        double *row_range) {
    const int i = (int)blockIdx.x * RED_THREADS + (int)threadIdx.x;
    if (i >= Nz) return;
    const double *u = uz + (long long)i * Nr;
    double *out = psi + (long long)i * Nr;
    double acc = 0.0, lo = 0.0, hi = 0.0;
    for (int j = 0; j < Nr; ++j) {
        acc -= (r0 + j + 0.5) * u[j];
        out[j] = acc;
        lo = fmin(lo, acc);
        hi = fmax(hi, acc);
    }
    row_range[2 * i] = lo;
    row_range[2 * i + 1] = hi;
}

// ----------------------------------------------------------------------------
// Host-side launchers.
static dim3 grid_for(const KParams &P, int bx, int by) {
    const int gx = (P.Nr + bx - 1) / bx, gy = (P.Nz + by - 1) / by;
    return dim3(gx * gy);
}

static dim3 step_grid(const KParams &P) { return grid_for(P, TX, TY); }

// Population p = OFF + q of distribution FLD: where node n reads it and
// where it writes it in the given phase (element offsets from the buffer
// start, before the node offset n is added).
template <int FLD>
static void plane_offsets(const KParams &P, int mode, int q, long long &rd, long long &wr) {
    using L = Lat<FLD>;
    const long long dn = (long long)L::ex(q) * P.pitch + L::ey(q);
    if (mode == MODE_AA_EVEN) {
        rd = (L::OFF + q) * P.plane;
        wr = (L::OFF + L::opp(q)) * P.plane;
    } else if (mode == MODE_AA_ODD) {
        rd = (L::OFF + L::opp(q)) * P.plane - dn;
        wr = (L::OFF + q) * P.plane + dn;
    } else {
        rd = (L::OFF + q) * P.plane - dn;
        wr = (L::OFF + q) * P.plane;
    }
}

// The plane addresses of one launch (see Planes).  Computed as integers:
// a read address of the odd phase or the pull may lie before its plane
// (the node offset brings it back inside for every node that uses it).
Planes step_planes(const KParams &P, int storage, int mode, const void *src, void *dst,
                   const char *Mprev, char *Mnext) {
    Planes A{};
    const uintptr_t a = (uintptr_t)src, b = (uintptr_t)dst;
    const long long es = storage == STORE_F32 ? 4 : 2;
    auto set = [&](int p, long long rd, long long wr) {
        A.rd[p] = (const char *)(a + (uintptr_t)(rd * es));
        A.wr[p] = (char *)(b + (uintptr_t)(wr * es));
    };
    long long rd, wr;
    for (int q = 0; q < 9; ++q) {
        plane_offsets<FLOW>(P, mode, q, rd, wr);
        set(q, rd, wr);
    }
    for (int q = 0; q < 5; ++q) {
        plane_offsets<SWIRL>(P, mode, q, rd, wr);
        set(GOFF + q, rd, wr);
        plane_offsets<THERMAL>(P, mode, q, rd, wr);
        set(HOFF + q, rd, wr);
    }
    // the lagged-field planes (left null for launches without them)
    if (Mprev && Mnext) {
        const long long vb = storage == STORE_F32 ? 4 : 2;  // velocity element size
        for (int v = 0; v < NLAG; ++v) {
            A.lrd[v] = Mprev + v * P.plane * vb;
            A.lwr[v] = Mnext + v * P.plane * vb;
        }
        A.uy_up = (const char *)((uintptr_t)A.lrd[1] + (uintptr_t)(vb * P.pitch));
        A.uy_dn = (const char *)((uintptr_t)A.lrd[1] - (uintptr_t)(vb * P.pitch));
    }
    return A;
}

template <class S, int BX, int BY>
static void launch_step_tile(const KParams &P, int mode, S *a, S *b, const char *Mprev,
                             char *Mnext, hipStream_t st) {
    const int edges = split_edges<S>(mode) ? edge_blocks(P.Nr, P.Nz, EDGE_PER_BLOCK) : 0;
    const dim3 grid(grid_for(P, BX, BY).x + edges), block(BX * BY);
    const Planes A = step_planes(P, store_of<S>(), mode, a, mode == MODE_AB ? b : a, Mprev, Mnext);
    switch (mode) {
    case MODE_AB: k_step<S, MODE_AB, BX, BY><<<grid, block, 0, st>>>(P, A, a, b, Mprev, Mnext); break;
    case MODE_AA_ODD: k_step<S, MODE_AA_ODD, BX, BY><<<grid, block, 0, st>>>(P, A, a, a, Mprev, Mnext); break;
    default: k_step<S, MODE_AA_EVEN, BX, BY><<<grid, block, 0, st>>>(P, A, a, a, Mprev, Mnext); break;
    }
}

template <class S>
static hipError_t launch_step_t(const KParams &P, int tile, int mode, void *src, void *dst,
                                const char *Mprev, char *Mnext, hipStream_t st) {
    S *a = (S *)src, *b = (S *)dst;
    switch (tile) {
#define AXLB_CASE(id, bx, by) \
    case id: launch_step_tile<S, bx, by>(P, mode, a, b, Mprev, Mnext, st); break;
        AXLB_TILES(AXLB_CASE)
#undef AXLB_CASE
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

template <class S>
static hipError_t launch_fields_t(const KParams &P, int mode, const void *src, const char *Mprev,
                                  double *out, hipStream_t st) {
    const dim3 grid = step_grid(P), block(TX * TY);
    const S *a = (const S *)src;
    switch (mode) {
    case MODE_AB: k_fields<S, MODE_AB><<<grid, block, 0, st>>>(P, a, Mprev, out); break;
    case MODE_AA_ODD: k_fields<S, MODE_AA_ODD><<<grid, block, 0, st>>>(P, a, Mprev, out); break;
    default: k_fields<S, MODE_AA_EVEN><<<grid, block, 0, st>>>(P, a, Mprev, out); break;
    }
    return hipGetLastError();
}

template <class S>
static hipError_t launch_init_t(const KParams &P, bool aa, bool enc, void *pop, const double *in,
                                char *M, hipStream_t st) {
    const dim3 grid = step_grid(P), block(TX * TY);
    if (aa) k_init<S, true, kEnc<S>><<<grid, block, 0, st>>>(P, (S *)pop, in, M);
    else if (enc) k_init<S, false, kEnc<S>><<<grid, block, 0, st>>>(P, (S *)pop, in, M);
    else k_init<S, false, false><<<grid, block, 0, st>>>(P, (S *)pop, in, M);
    return hipGetLastError();
}

hipError_t launch_step(const KParams &P, int storage, int tile, int mode, void *src, void *dst,
                       const char *Mprev, char *Mnext, hipStream_t st) {
    if (storage == STORE_F16)
        return launch_step_t<__half>(P, tile, mode, src, dst, Mprev, Mnext, st);
    if (storage == STORE_BF16)
        return launch_step_t<__hip_bfloat16>(P, tile, mode, src, dst, Mprev, Mnext, st);
    return launch_step_t<float>(P, tile, mode, src, dst, Mprev, Mnext, st);
}

int tile_count() { return NTILES; }

void tile_shape(int tile, int *bx, int *by) {
    switch (tile) {
#define AXLB_CASE(id, x, y) \
    case id: *bx = x; *by = y; return;
        AXLB_TILES(AXLB_CASE)
#undef AXLB_CASE
    default: *bx = *by = 0;
    }
}

hipError_t launch_fields(const KParams &P, int storage, int mode, const void *src,
                         const char *Mprev, double *out, hipStream_t st) {
    if (storage == STORE_F16) return launch_fields_t<__half>(P, mode, src, Mprev, out, st);
    if (storage == STORE_BF16) return launch_fields_t<__hip_bfloat16>(P, mode, src, Mprev, out, st);
    return launch_fields_t<float>(P, mode, src, Mprev, out, st);
}

hipError_t launch_init(const KParams &P, int storage, bool aa, bool enc, void *pop,
                       const double *in, char *M, hipStream_t st) {
    if (storage == STORE_F16) return launch_init_t<__half>(P, aa, enc, pop, in, M, st);
    if (storage == STORE_BF16) return launch_init_t<__hip_bfloat16>(P, aa, enc, pop, in, M, st);
    return launch_init_t<float>(P, aa, enc, pop, in, M, st);
}

hipError_t launch_residual(const double *fld, const double *snap, long long N, double *part,
                           int nblocks, double *out9, hipStream_t st) {
    k_residual_partial<<<nblocks, RED_THREADS, 0, st>>>(fld, snap, N, part);
    k_sum_partials<<<1, RED_THREADS, 0, st>>>(part, nblocks, 9, out9);
    return hipGetLastError();
}

hipError_t launch_nusselt(const double *T, int Nr, int Nz, int cylinder, double r0, double Ta,
                          double Tb, double *out2, hipStream_t st) {
    k_nusselt<<<1, RED_THREADS, 0, st>>>(T, Nr, Nz, cylinder, r0, Ta, Tb, out2);
    return hipGetLastError();
}

hipError_t launch_stream(const double *uz, int Nr, int Nz, double r0, double *psi,
                         double *row_range, hipStream_t st) {
    k_stream<<<(Nz + RED_THREADS - 1) / RED_THREADS, RED_THREADS, 0, st>>>(uz, Nr, Nz, r0, psi,
                                                                          row_range);
    return hipGetLastError();
}

}  // namespace axlb
