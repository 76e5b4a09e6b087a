// Wall Nusselt numbers (Section 3.2) without any device allocation, for
// callers that cannot allocate: the temperature of the two nodes next to each
// heat-transfer wall is computed straight from the populations (the same
// per-node arithmetic as the reported fields), and the per-workgroup partial
// sums go to a fixed array in device memory instead of the lattice's field
// and reduction buffers.
#include <hip/hip_runtime.h>

#include <mutex>
#include <string>

#include "../../include/axlb.h"
#include "axlb_internal.h"
#include "axlb_launch.h"
#include "axlb_node.h"
#include "axlb_reduce.h"

namespace axlb {

// Workgroups of the wall kernel: one per RED_THREADS wall positions (rows of
// an annulus, columns of a cylinder), so at most NU_MAX_BLOCKS * RED_THREADS
// = 2^21 positions.
constexpr int NU_MAX_BLOCKS = 8192;
constexpr int NU_RESULT = 2 * NU_MAX_BLOCKS;

// The scratch array: NU_MAX_BLOCKS pairs of partial sums, then the final
// pair; 128 KiB per device, held until the process ends.  Host code must not
// use this name as an address (on the host it is only a stand-in for the
// symbol): scratch_on() looks up each device's own copy.
static __device__ __align__(256) double scratch[NU_RESULT + 2];

// Current-step output fields of a node as a field source for `differences`:
// it streams the neighbour's populations from the buffer (with the boundary
// rules) and takes their moments, as the current-step kernel does for its
// LDS tile.  A neighbour beyond a periodic face is its image.
template <class S>
struct PulledFields {
    const KParams &P;
    const S *src;
    int i, j;
    __device__ float operator()(int v, int di, int dj) const {
        int ni = i + di;
        if ((unsigned)ni >= (unsigned)P.Nz) ni += ni < 0 ? P.Nz : -P.Nz;
        float f[9], g[5], h[5];
        pull_all<false>(P, GlobalPops<S, false>{P, src, nullptr}, ni, j + dj, f, g, h);
        const Moments m = moments(f, g, h);
        const float ir = rcp(1.f + m.drho);
        return v == 0 ? m.jx * ir : v == 1 ? m.jy * ir : v == 2 ? m.psi * ir : m.dphi;
    }
};

// Temperature of node (i, j) after the pre-collision half step, as the
// reported fields give it.  MODE selects the slot convention of the state
// (AB, or the AA phase); CUR takes the current-step derivatives.
template <class S, int MODE, bool CUR>
__device__ double node_T(const KParams &P, const S *src, const char *Mprev, int i, int j) {
    float f[9], g[5], h[5], d[5];
    if (CUR) {
        pull_all<false>(P, GlobalPops<S, false>{P, src, nullptr}, i, j, f, g, h);
        differences(P, PulledFields<S>{P, src, i, j}, i, j, d);
    } else {
        const bool interior = interior_node(P, i, j);
        gather<S, MODE>(P, src, Mprev, i, j, interior, f, g, h);
        derivatives<S>(P, Mprev, i, j, interior, d);
    }
    const Moments m = moments(f, g, h);
    const float iy = rcp(P.r0 + (float)j + 0.5f);
    const Half H = half_step(P, iy, m.drho, m.jx, m.jy, m.psi, m.dphi, d);
    return (double)P.Tref + (double)H.dphi;
}

// Partial sums of the one-sided wall gradients (-8 T_w + 9 T_1 - T_2)/3
// along each wall's inward normal: annulus rows at the inner and outer wall;
// cylinder columns at the bottom and top lid, weighted by the radius.
template <class S, int MODE, bool CUR>
__global__ void __launch_bounds__(RED_THREADS) k_nusselt_walls(const KParams P, const S *src,
                                                                const char *Mprev, int cylinder,
                                                                double Ta, double Tb,
                                                                double *part) {
    __shared__ double sh[2 * (RED_THREADS / 64)];
    double v[2] = {0.0, 0.0};
    const int k = (int)blockIdx.x * RED_THREADS + (int)threadIdx.x;
    if (!cylinder && k < P.Nz) {
        const double T1 = node_T<S, MODE, CUR>(P, src, Mprev, k, 0);
        const double T2 = node_T<S, MODE, CUR>(P, src, Mprev, k, 1);
        const double U1 = node_T<S, MODE, CUR>(P, src, Mprev, k, P.Nr - 1);
        const double U2 = node_T<S, MODE, CUR>(P, src, Mprev, k, P.Nr - 2);
        v[0] = (-8.0 * Ta + 9.0 * T1 - T2) / 3.0;
        v[1] = -(-8.0 * Tb + 9.0 * U1 - U2) / 3.0;
    } else if (cylinder && k < P.Nr) {
        const double y = (double)P.r0 + k + 0.5;
        const double T1 = node_T<S, MODE, CUR>(P, src, Mprev, 0, k);
        const double T2 = node_T<S, MODE, CUR>(P, src, Mprev, 1, k);
        const double U1 = node_T<S, MODE, CUR>(P, src, Mprev, P.Nz - 1, k);
        const double U2 = node_T<S, MODE, CUR>(P, src, Mprev, P.Nz - 2, k);
        v[0] = y * (-8.0 * Ta + 9.0 * T1 - T2) / 3.0;
        v[1] = -y * (-8.0 * Tb + 9.0 * U1 - U2) / 3.0;
    }
    block_sum<2>(v, sh);
    if (threadIdx.x == 0) {
        part[2 * blockIdx.x] = v[0];
        part[2 * blockIdx.x + 1] = v[1];
    }
}

// Sum of the first nblocks partial pairs, in a fixed order, into out[0..1].
__global__ void __launch_bounds__(RED_THREADS) k_nusselt_finish(const double *part, int nblocks,
                                                                 double *out) {
    __shared__ double sh[2 * (RED_THREADS / 64)];
    double v[2] = {0.0, 0.0};
    for (int b = (int)threadIdx.x; b < nblocks; b += RED_THREADS) {
        v[0] += part[2 * b];
        v[1] += part[2 * b + 1];
    }
    block_sum<2>(v, sh);
    if (threadIdx.x == 0) {
        out[0] = v[0];
        out[1] = v[1];
    }
}

template <class S>
static hipError_t launch_walls(const axlb_lattice *L, int nblocks, double Ta, double Tb,
                               double *part) {
    const KParams &P = L->P;
    const dim3 grid(nblocks), block(RED_THREADS);
    if (L->deriv == AXLB_DERIV_CURRENT) {
        k_nusselt_walls<S, MODE_AB, true><<<grid, block, 0, L->stream>>>(
            P, (const S *)L->pop[L->cur], nullptr, L->cylinder, Ta, Tb, part);
    } else if (L->layout != AXLB_LAYOUT_AA) {
        k_nusselt_walls<S, MODE_AB, false><<<grid, block, 0, L->stream>>>(
            P, (const S *)L->pop[L->cur], L->lag[L->cur], L->cylinder, Ta, Tb, part);
    } else {
        // the state the next step reads: its phase follows the step parity
        const int par = (int)(L->steps & 1);
        if (par == 0)
            k_nusselt_walls<S, MODE_AA_ODD, false><<<grid, block, 0, L->stream>>>(
                P, (const S *)L->pop[0], L->lag[0], L->cylinder, Ta, Tb, part);
        else
            k_nusselt_walls<S, MODE_AA_EVEN, false><<<grid, block, 0, L->stream>>>(
                P, (const S *)L->pop[0], L->lag[1], L->cylinder, Ta, Tb, part);
    }
    return hipGetLastError();
}

// Device address of each device's copy of `scratch`, looked up once per
// device (with that device current) and kept for the life of the process.
constexpr int MAX_DEVICES = 64;
static std::mutex g_scratch_mu;
static double *g_scratch[MAX_DEVICES] = {};

static hipError_t scratch_on(int dev, double **out) {
    if (dev < 0 || dev >= MAX_DEVICES) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch[dev]) {
        void *p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        g_scratch[dev] = static_cast<double *>(p);
    }
    *out = g_scratch[dev];
    return hipSuccess;
}

}  // namespace axlb

using namespace axlb;

static int nu_fail(axlb_lattice *L, int code, const std::string &msg) {
    L->err = msg;
    return code;
}

extern "C" int axlb_nusselt_noalloc(axlb_lattice *L, double *nu_a, double *nu_b, double *mean) {
    if (!L) return AXLB_EINVAL;
    const int fa = L->cylinder ? AXLB_Z_LO : AXLB_R_IN, fb = L->cylinder ? AXLB_Z_HI : AXLB_R_OUT;
    if (L->kind[fa][2] != AXLB_DIRICHLET || L->kind[fb][2] != AXLB_DIRICHLET)
        return nu_fail(L, AXLB_ESTATE, "Nusselt numbers need imposed T on both heat-transfer walls");
    if (L->cylinder && (L->split[0] || L->split[1]))
        return nu_fail(L, AXLB_ESTATE, "Nusselt numbers need lids of one temperature each");
    const double Ta = L->val[fa][2], Tb = L->val[fb][2];
    const double dT = L->cylinder ? Tb - Ta : Ta - Tb;
    if (dT == 0.0) return nu_fail(L, AXLB_ESTATE, "the two wall temperatures are equal");
    if ((L->cylinder && L->Nz < 2) || L->Nr < 2)
        return nu_fail(L, AXLB_ESTATE, "too few nodes for the wall gradient");
    const int W = L->cylinder ? L->Nr : L->Nz;
    const int nblocks = (W + RED_THREADS - 1) / RED_THREADS;
    if (nblocks > NU_MAX_BLOCKS)
        return nu_fail(L, AXLB_EINVAL,
                       "axlb_nusselt_noalloc: the wall spans " + std::to_string(W) +
                           " nodes; its fixed scratch serves at most " +
                           std::to_string(NU_MAX_BLOCKS * RED_THREADS));
    hipError_t e = hipSetDevice(L->device);
    double *part = nullptr;
    if (e == hipSuccess) e = scratch_on(L->device, &part);
    if (e == hipSuccess) {
        if (L->storage == AXLB_F16) e = launch_walls<__half>(L, nblocks, Ta, Tb, part);
        else if (L->storage == AXLB_BF16) e = launch_walls<__hip_bfloat16>(L, nblocks, Ta, Tb, part);
        else e = launch_walls<float>(L, nblocks, Ta, Tb, part);
    }
    if (e == hipSuccess) {
        k_nusselt_finish<<<1, RED_THREADS, 0, L->stream>>>(part, nblocks, part + NU_RESULT);
        e = hipGetLastError();
    }
    double s[2] = {0.0, 0.0};
    if (e == hipSuccess)
        e = hipMemcpyAsync(s, part + NU_RESULT, sizeof(s), hipMemcpyDeviceToHost, L->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(L->stream);
    if (e != hipSuccess)
        return nu_fail(L, AXLB_EDEVICE, std::string("axlb_nusselt_noalloc: ") + hipGetErrorString(e));
    double a, b;
    if (!L->cylinder) {
        // Section 3.2: Nu = -R/(H dT) int d_y T dx over the wall
        const double H = L->Nz, Ri = L->r_inner, Ro = L->r_inner + L->Nr;
        a = -Ri / (H * dT) * s[0];
        b = -Ro / (H * dT) * s[1];
    } else {
        const double H = L->Nz, R = L->Nr;
        a = H / dT * 2.0 / (R * R) * s[0];
        b = H / dT * 2.0 / (R * R) * s[1];
    }
    if (nu_a) *nu_a = a;
    if (nu_b) *nu_b = b;
    if (mean) *mean = 0.5 * (a + b);
    return AXLB_OK;
}
