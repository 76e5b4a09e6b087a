// Device code of one node update of the axisymmetric cascaded LB step
// (arXiv 1806.10241, Section 2), shared by the single-lattice and the batched
// kernels so that both perform identical arithmetic.  Internal.
#pragma once

#include <type_traits>

#include "axlb_device.h"

namespace axlb {

// ----------------------------------------------------------------------------
// Lattices.  D2Q9 velocities in the order of Section 2.2, eq. (10); D2Q5 in
// the order of eq. (28).
template <int FLD> struct Lat;
template <> struct Lat<FLOW> {
    static constexpr int NQ = 9, OFF = 0;
    __host__ __device__ static constexpr int ex(int q) {
        return q == 1 || q == 5 || q == 8 ? 1 : (q == 3 || q == 6 || q == 7 ? -1 : 0);
    }
    __host__ __device__ static constexpr int ey(int q) {
        return q == 2 || q == 5 || q == 6 ? 1 : (q == 4 || q == 7 || q == 8 ? -1 : 0);
    }
    __host__ __device__ static constexpr int opp(int q) {
        return q == 0 ? 0 : (q <= 4 ? (q + 1) % 4 + 1 : (q + 1) % 4 + 5);
    }
    __host__ __device__ static constexpr int refl(int q) {  // e_y -> -e_y
        return q == 2 ? 4 : q == 4 ? 2 : q == 5 ? 8 : q == 8 ? 5 : q == 6 ? 7 : q == 7 ? 6 : q;
    }
    __host__ __device__ static constexpr int reflx(int q) {  // e_x -> -e_x
        return q == 1 ? 3 : q == 3 ? 1 : q == 5 ? 6 : q == 6 ? 5 : q == 7 ? 8 : q == 8 ? 7 : q;
    }
};
template <int OFFSET> struct Lat5 {
    static constexpr int NQ = 5, OFF = OFFSET;
    __host__ __device__ static constexpr int ex(int q) { return q == 1 ? 1 : (q == 3 ? -1 : 0); }
    __host__ __device__ static constexpr int ey(int q) { return q == 2 ? 1 : (q == 4 ? -1 : 0); }
    __host__ __device__ static constexpr int opp(int q) { return q == 0 ? 0 : (q + 1) % 4 + 1; }
    __host__ __device__ static constexpr int refl(int q) { return q == 2 ? 4 : q == 4 ? 2 : q; }
};
template <> struct Lat<SWIRL> : Lat5<GOFF> {};
template <> struct Lat<THERMAL> : Lat5<HOFF> {};

static_assert(Lat<FLOW>::opp(1) == 3 && Lat<FLOW>::opp(2) == 4 && Lat<FLOW>::opp(5) == 7 &&
                  Lat<FLOW>::opp(6) == 8 && Lat<FLOW>::opp(8) == 6,
              "D2Q9 opposite table");
static_assert(Lat<SWIRL>::opp(1) == 3 && Lat<SWIRL>::opp(4) == 2, "D2Q5 opposite table");
static_assert(Lat<FLOW>::reflx(Lat<FLOW>::refl(5)) == Lat<FLOW>::opp(5) &&
                  Lat<FLOW>::reflx(Lat<FLOW>::refl(8)) == Lat<FLOW>::opp(8) &&
                  Lat<FLOW>::ex(Lat<FLOW>::reflx(1)) == -1 && Lat<FLOW>::ey(Lat<FLOW>::reflx(8)) == -1,
              "D2Q9 reflection tables");

// Random words of the stochastic rounding of 16-bit stores (ignored by FP32
// storage).  A node update's 19 stores share one multiplicative hash of the
// node's position and of the XOR of the bit patterns of the 19 FP32 values:
// it changes whenever any value changes, and a change in a value's lowest
// bits reaches the word's top bits, which set the threshold.  Store p (plane
// 0..18) adds p + 1 steps of a Weyl sequence to it, so the slots of a node
// draw different thresholds.  One quarter-rate 32-bit multiply per node;
// the node key uses the full-rate 24-bit multiply.
template <int N>
__device__ __forceinline__ unsigned xor_bits(const float (&v)[N]) {
    unsigned x = __float_as_uint(v[0]);
#pragma unroll
    for (int k = 1; k < N; ++k) x ^= __float_as_uint(v[k]);
    return x;
}
__device__ __forceinline__ unsigned node_word(const float (&f)[9], const float (&g)[5],
                                              const float (&h)[5], int i, int j) {
    const unsigned key = __umul24((unsigned)i, 0x9E3779u) ^ __umul24((unsigned)j, 0x85EBCAu);
    return (xor_bits(f) ^ xor_bits(g) ^ xor_bits(h) ^ key) * 0x9E3779B1U;
}
__device__ __forceinline__ unsigned slot_word(unsigned w, int p) {
    return w + (unsigned)(p + 1) * 0x632BE5ABU;
}
// The key of a lone value at node (i, j), plane p (initial states).
__device__ __forceinline__ unsigned skey(int i, int j, int p) {
    return ((unsigned)i * 0x9E3779B1U) ^ ((unsigned)j * 0x85EBCA77U) ^ ((unsigned)p * 0xC2B2AE3DU);
}

__device__ __forceinline__ bool is_wall(int k) {
    return k == NOSLIP || k == DIRICHLET || k == OMEGA_R || k == ADIABATIC || k == VELOCITY;
}

// Normal velocity that a face imposes where a link crosses it at c2
// (VELOCITY for f: along +y on radial faces, +x on axial faces), 0 for
// every other kind.
__device__ __forceinline__ float face_velocity(const KParams &P, int face, int c2) {
    return kind_at(P, face, FLOW, c2) == VELOCITY ? val_at<FLOW>(P, face, c2, 0.f) : 0.f;
}

// Moving-wall bounce-back for f: the population q that comes back off a
// wall moving with u_w along the face normal gains 2 w_q rho_0 (e_q . u_w) /
// c_s^2 = 6 w_q (e_q . u_w) with rho_0 = 1 (shifted storage subtracts the
// same w_q on both sides).  Lattice weights 4/9, 1/9, 1/36.
template <int Q>
__device__ __forceinline__ float moving_wall(const KParams &P, int face, int c2) {
    using L = Lat<FLOW>;
    constexpr int ex = L::ex(Q), ey = L::ey(Q);
    constexpr float w = (ex == 0 && ey == 0) ? 4.f / 9.f : ((ex == 0 || ey == 0) ? 1.f / 9.f : 1.f / 36.f);
    const float e_n = (float)(face <= R_OUT ? ey : ex);
    return 6.f * w * e_n * val_at<FLOW>(P, face, c2, 0.f);
}

// Unshifted wall value of g or h (u_theta,w or T_w) for the advective part
// of the anti-bounce-back at a wall the fluid crosses; ym is the radius
// where the link crosses the wall, c2 twice its column.
template <int FLD>
__device__ __forceinline__ float wall_raw(const KParams &P, int face, int c2, float ym) {
    const int k = kind_at(P, face, FLD, c2);
    const float v = val_at<FLD>(P, face, c2, ym);
    return k == DIRICHLET ? v : (k == OMEGA_R ? v * ym : 0.f);
}

// Value that the advection-diffusion wall rule imposes (psi_w = u_theta,w
// with rho_0 = 1, or T_w - T_ref in shifted storage).
template <int FLD>
__device__ __forceinline__ float wall_value(const KParams &P, int face, int c2, float ym) {
    float s = wall_raw<FLD>(P, face, c2, ym);
    if (FLD == THERMAL) s -= P.Tref;
    return s;
}

// ----------------------------------------------------------------------------
// Offset encoding of bfloat16 populations.  bfloat16 keeps 8 significant
// bits, and a shifted population f - w_q is dominated by its part linear in
// the velocity, 3 w_q e_q . u (g by w_q u_theta, h - w_q T_ref by
// w_q (T - T_ref)), so the store would round away most of what the
// collision changes.  A bfloat16 slot therefore holds its population minus
// that linear equilibrium part evaluated with the lagged fields of the node
// that wrote it, exactly as stored in the lagged-field block of the step
// (the writer has them in registers, a reader loads them with its
// derivative stencils): the stored value is the small non-equilibrium
// remainder plus the change of u over one link, and the reader adds the same
// FP32 offset back.  FP32 and binary16 storage, and the current-step
// derivative form (which keeps no lagged fields), store populations as they
// are.  Which node wrote a slot, and for which direction:
//  * two buffers, and the AA odd phase reading what the even phase wrote:
//    the node that holds the slot, for the direction of the plane (AB) or
//    the opposite one (AA, whose even phase writes f*_q into plane opp q);
//  * the AA even phase reading what the odd phase pushed: the source node of
//    the pull form, for the direction of the plane, where the link stays in
//    the fluid, is reflected at the axis or the free surface, or wraps
//    periodically; after a wall the node itself, for the direction that hit
//    the wall (the odd phase applies the wall rule before it stores).
template <class S>
constexpr bool kEnc = std::is_same<S, __hip_bfloat16>::value;

// Lagged fields of a node as the lagged-field block holds them (u_x, u_y,
// u_theta, T - T_ref).
struct Lag4 {
    float ux, uy, ut, dT;
};

// Offset of population q of distribution FLD for lagged fields L: products
// with +-1 and one rounding per term, so that every path forms the same bits.
template <int FLD>
__device__ __forceinline__ float pop_off(int q, const Lag4 &L) {
    if (FLD == FLOW) {
        const int ex = Lat<FLOW>::ex(q), ey = Lat<FLOW>::ey(q);
        float e = 0.f, w3 = 1.f / 12.f;  // 3 w_q: 1/3 along an axis, 1/12 diagonally
        if (ex != 0 && ey != 0) {
            e = (ex > 0 ? L.ux : -L.ux) + (ey > 0 ? L.uy : -L.uy);
        } else if (ex != 0) {
            e = ex > 0 ? L.ux : -L.ux;
            w3 = 1.f / 3.f;
        } else if (ey != 0) {
            e = ey > 0 ? L.uy : -L.uy;
            w3 = 1.f / 3.f;
        }
        return w3 * e;
    }
    const float w = q == 0 ? 1.f / 3.f : 1.f / 6.f;
    return w * (FLD == SWIRL ? L.ut : L.dT);
}
// Offset of plane p (0..18) holding direction p (OPP: the opposite one).
template <bool OPP>
__device__ __forceinline__ float plane_off(int p, const Lag4 &L) {
    if (p < GOFF) return pop_off<FLOW>(OPP ? Lat<FLOW>::opp(p) : p, L);
    if (p < HOFF) return pop_off<SWIRL>(OPP ? Lat<SWIRL>::opp(p - GOFF) : p - GOFF, L);
    return pop_off<THERMAL>(OPP ? Lat<THERMAL>::opp(p - HOFF) : p - HOFF, L);
}

// The lagged fields at node (i, j) of block M, where i may lie one row
// beyond a periodic z face (its image) or a HALO face (the halo row's).
template <class S>
__device__ __forceinline__ Lag4 lag_at(const KParams &P, const char *M, int i, int j) {
    const char *B = M;
    long long plane = P.plane, off;
    if ((unsigned)i >= (unsigned)P.Nz) {
        const int f = i < 0 ? 0 : 1;
        if (kind_of(P, Z_LO + f, FLOW) == HALO) {
            B = P.halo_lag[f];
            plane = P.pitch;
            off = j;
            return {lag_ld<S>(B, 0, plane, off), lag_ld<S>(B, 1, plane, off),
                    lag_ld<S>(B, 2, plane, off), lag_ld<S>(B, 3, plane, off)};
        }
        i += i < 0 ? P.Nz : -P.Nz;
    }
    off = (long long)i * P.pitch + j;
    return {lag_ld<S>(B, 0, plane, off), lag_ld<S>(B, 1, plane, off), lag_ld<S>(B, 2, plane, off),
            lag_ld<S>(B, 3, plane, off)};
}

// The lagged fields at element offset m of block M (a fluid node).
template <class S>
__device__ __forceinline__ Lag4 lag_node(const KParams &P, const char *M, unsigned m) {
    return {lag_ld<S>(M, 0, P.plane, m), lag_ld<S>(M, 1, P.plane, m), lag_ld<S>(M, 2, P.plane, m),
            lag_ld<S>(M, 3, P.plane, m)};
}

// The lagged fields a node update stores, as a reader will load them.
template <class S>
__device__ __forceinline__ Lag4 lag_stored(float ux, float uy, float ut, float dT) {
    return {lag_round<S>(0, ux), lag_round<S>(1, uy), lag_round<S>(2, ut), lag_round<S>(3, dT)};
}

// Offset of population Q of distribution FLD that node (i, j) reads from its
// own slot in the AA even phase: the writer's lagged fields (see above).
template <class S, int FLD, int Q>
__device__ __forceinline__ float even_off(const KParams &P, const char *M, int i, int j) {
    using L = Lat<FLD>;
    constexpr int ex = L::ex(Q), ey = L::ey(Q);
    int si = i - ex, sj = j - ey;
    if ((unsigned)si < (unsigned)P.Nz && (unsigned)sj < (unsigned)P.Nr)
        return pop_off<FLD>(Q, lag_at<S>(P, M, si, sj));
    const int c2 = 2 * j - ey;
    const int fy = sj < 0 ? R_IN : (sj >= P.Nr ? R_OUT : -1);
    const int fx = si < 0 ? Z_LO : (si >= P.Nz ? Z_HI : -1);
    if ((fy >= 0 && is_wall(kind_of(P, fy, FLD))) || (fx >= 0 && is_wall(kind_at(P, fx, FLD, c2))))
        return pop_off<FLD>(L::opp(Q), lag_at<S>(P, M, i, j));
    if (fy >= 0) sj = j;  // the axis
    if (FLD == FLOW && fx >= 0 && kind_at(P, fx, FLOW, c2) == SLIP) si = i;
    return pop_off<FLD>(Q, lag_at<S>(P, M, si, sj));  // a row beyond a periodic face: its image
}

// ----------------------------------------------------------------------------
// Population sources for the pulls: src(p, i, j) is the value in plane p
// (0..18) at node (i, j), where i may lie one row beyond a periodic z face
// (the source then supplies the periodic image) or a HALO face.
// GlobalPops reads a population buffer in device memory.
// A row beyond a HALO z face comes from that face's halo row instead.
// ENC: offset-encoded storage whose writer is the node holding the slot,
// with the lagged fields M; AA: planes hold the opposite direction (the
// state the AA even phase leaves).
template <class S, bool ENC = kEnc<S>, bool AA = false>
struct GlobalPops {
    const KParams &P;
    const S *A;
    const char *M;
    __device__ __forceinline__ float operator()(int p, int i, int j) const {
        float v;
        const int ri = i;
        if ((unsigned)i >= (unsigned)P.Nz) {
            const int f = i < 0 ? 0 : 1;
            if (kind_of(P, Z_LO + f, FLOW) == HALO) {
                v = Conv<S>::ld(static_cast<const S *>(P.halo_pop[f]) + p * P.pitch + j);
                if constexpr (ENC) v = v + plane_off<AA>(p, lag_at<S>(P, M, ri, j));
                return v;
            }
            i += i < 0 ? P.Nz : -P.Nz;
        }
        v = Conv<S>::ld(A + p * P.plane + (long long)i * P.pitch + j);
        if constexpr (ENC) v = v + plane_off<AA>(p, lag_at<S>(P, M, i, j));
        return v;
    }
};

// Pull of population Q of distribution FLD into node (i, j) when the source
// node (i - e_x, j - e_y) lies outside the fluid.  Precedence per link: a
// solid wall (radial faces first) -> half-way bounce-back for f and for zero
// flux, anti-bounce-back -v + 2 w s_w (w = 1/6) for an imposed u_theta or T;
// then the axis -> specular reflection from the node shifted by e_x, with a
// sign change for g (u_theta is odd); then a free surface on an axial face
// (SLIP, f only) -> specular reflection from the node shifted by e_y (after
// the axis reflection where a link crosses both); then the periodic image
// along z.  An axial face split in two parts gives a link the rule of the
// part where it crosses the face, at twice the column c2 = 2 j - e_y.
// AA selects the slot convention of the odd phase of the in-place layout.
template <bool AA, int FLD, int Q, class Src>
__device__ __forceinline__ float pull_edge(const KParams &P, const Src &src, int i, int j) {
    using L = Lat<FLD>;
    constexpr int ex = L::ex(Q), ey = L::ey(Q);
    int si = i - ex;
    int sj = j - ey;
    const int c2 = 2 * j - ey;
    const int fy = sj < 0 ? R_IN : (sj >= P.Nr ? R_OUT : -1);
    const int fx = si < 0 ? Z_LO : (si >= P.Nz ? Z_HI : -1);
    int wall = -1;
    if (fy >= 0 && is_wall(kind_of(P, fy, FLD))) wall = fy;
    else if (fx >= 0 && is_wall(kind_at(P, fx, FLD, c2))) wall = fx;
    if (wall >= 0) {
        // f*_{opp Q}(i, j): AB keeps it in plane opp Q, the even AA phase put
        // it into plane Q.
        constexpr int slot = AA ? Q : L::opp(Q);
        const float v = src(L::OFF + slot, i, j);
        const bool moving = kind_at(P, wall, FLOW, c2) == VELOCITY;
        if (FLD == FLOW) return moving ? v + moving_wall<Q>(P, wall, c2) : v;
        if (kind_at(P, wall, FLD, c2) == ADIABATIC) return v;
        const float ym = P.r0 + (float)j + 0.5f - 0.5f * (float)ey;
        const float r = -v + (1.f / 3.f) * wall_value<FLD>(P, wall, c2, ym);
        if (!moving) return r;
        const float un = val_at<FLOW>(P, wall, c2, 0.f);
        return r + un * un * wall_raw<FLD>(P, wall, c2, ym);
    }
    float sign = 1.f;
    int qs = Q;
    if (fy >= 0) {  // only the axis remains on a radial face
        qs = L::refl(Q);
        sj = j;
        if (FLD == SWIRL) sign = -1.f;
    }
    if (FLD == FLOW && fx >= 0 && kind_at(P, fx, FLOW, c2) == SLIP) {
        qs = Lat<FLOW>::reflx(qs);
        si = i;
    }
    const int slot = AA ? L::opp(qs) : qs;
    return sign * src(L::OFF + slot, si, sj);  // a z row beyond a periodic face: its image
}

template <bool AA, int FLD, int Q, class Src>
__device__ __forceinline__ float pull(const KParams &P, const Src &src, int i, int j) {
    using L = Lat<FLD>;
    constexpr int ex = L::ex(Q), ey = L::ey(Q);
    const int si = i - ex, sj = j - ey;
    if ((unsigned)si < (unsigned)P.Nz && (unsigned)sj < (unsigned)P.Nr) {
        constexpr int slot = AA ? L::opp(Q) : Q;
        return src(L::OFF + slot, si, sj);
    }
    return pull_edge<AA, FLD, Q>(P, src, i, j);
}

// All 19 pulls of node (i, j) from a population source, with the boundary
// rules wherever a source node lies outside the fluid.
template <bool AA, class Src>
__device__ __forceinline__ void pull_all(const KParams &P, const Src &src, int i, int j,
                                         float (&f)[9], float (&g)[5], float (&h)[5]) {
    f[0] = pull<AA, FLOW, 0>(P, src, i, j);
    f[1] = pull<AA, FLOW, 1>(P, src, i, j);
    f[2] = pull<AA, FLOW, 2>(P, src, i, j);
    f[3] = pull<AA, FLOW, 3>(P, src, i, j);
    f[4] = pull<AA, FLOW, 4>(P, src, i, j);
    f[5] = pull<AA, FLOW, 5>(P, src, i, j);
    f[6] = pull<AA, FLOW, 6>(P, src, i, j);
    f[7] = pull<AA, FLOW, 7>(P, src, i, j);
    f[8] = pull<AA, FLOW, 8>(P, src, i, j);
    g[0] = pull<AA, SWIRL, 0>(P, src, i, j);
    g[1] = pull<AA, SWIRL, 1>(P, src, i, j);
    g[2] = pull<AA, SWIRL, 2>(P, src, i, j);
    g[3] = pull<AA, SWIRL, 3>(P, src, i, j);
    g[4] = pull<AA, SWIRL, 4>(P, src, i, j);
    h[0] = pull<AA, THERMAL, 0>(P, src, i, j);
    h[1] = pull<AA, THERMAL, 1>(P, src, i, j);
    h[2] = pull<AA, THERMAL, 2>(P, src, i, j);
    h[3] = pull<AA, THERMAL, 3>(P, src, i, j);
    h[4] = pull<AA, THERMAL, 4>(P, src, i, j);
}

// Odd AA phase: post-collision f*_Q(i, j) = v goes to the slot from which
// the next (even) phase reads it, by the same rules as pull_edge.  ENC
// subtracts the offset of the node's own stored lagged fields Ln: for the
// direction Q after a wall, for the direction of the receiving plane else.
template <class S, int FLD, int Q, bool ENC = kEnc<S>>
__device__ __forceinline__ void push_edge(const KParams &P, S *A, int i, int j, float v,
                                          unsigned w0, const Lag4 &Ln) {
    using L = Lat<FLD>;
    constexpr int ex = L::ex(Q), ey = L::ey(Q);
    int ti = i + ex;
    const int tj = j + ey;
    // the link crosses an axial face at twice the column 2 j + e_y (the
    // receiving node's 2 j' - e_y of the pull form)
    const int c2 = 2 * j + ey;
    const int fy = tj < 0 ? R_IN : (tj >= P.Nr ? R_OUT : -1);
    const int fx = ti < 0 ? Z_LO : (ti >= P.Nz ? Z_HI : -1);
    int wall = -1;
    if (fy >= 0 && is_wall(kind_of(P, fy, FLD))) wall = fy;
    else if (fx >= 0 && is_wall(kind_at(P, fx, FLD, c2))) wall = fx;
    if (wall >= 0) {
        // it comes back to (i, j) as population opp Q
        float w = v;
        const bool moving = kind_at(P, wall, FLOW, c2) == VELOCITY;
        if (FLD == FLOW) {
            if (moving) w = v + moving_wall<L::opp(Q)>(P, wall, c2);
        } else if (kind_at(P, wall, FLD, c2) != ADIABATIC) {
            const float ym = P.r0 + (float)j + 0.5f + 0.5f * (float)ey;
            w = -v + (1.f / 3.f) * wall_value<FLD>(P, wall, c2, ym);
            if (moving) {
                const float un = val_at<FLOW>(P, wall, c2, 0.f);
                w = w + un * un * wall_raw<FLD>(P, wall, c2, ym);
            }
        }
        if constexpr (ENC) w = w - pop_off<FLD>(Q, Ln);
        Conv<S>::st(A + (L::OFF + L::opp(Q)) * P.plane + (long long)i * P.pitch + j, w,
                    slot_word(w0, L::OFF + Q));
        return;
    }
    const bool slip = FLD == FLOW && fx >= 0 && kind_at(P, fx, FLOW, c2) == SLIP;
    if (fy >= 0) {  // axis: arrives at (i + e_x, j) with e_y reversed
        int q = L::refl(Q);
        if (slip) {  // and off the free surface: at (i, j), both reversed
            ti = i;
            q = Lat<FLOW>::reflx(q);
        } else if (ti < 0) {
            ti += P.Nz;
        } else if (ti >= P.Nz) {
            ti -= P.Nz;
        }
        float w = FLD == SWIRL ? -v : v;
        if constexpr (ENC) w = w - pop_off<FLD>(q, Ln);
        Conv<S>::st(A + (L::OFF + q) * P.plane + (long long)ti * P.pitch + j, w,
                    slot_word(w0, L::OFF + Q));
        return;
    }
    if (slip) {  // free surface: arrives at (i, j + e_y) with e_x reversed
        float w = v;
        if constexpr (ENC) w = w - pop_off<FLOW>(Lat<FLOW>::reflx(Q), Ln);
        Conv<S>::st(A + (L::OFF + Lat<FLOW>::reflx(Q)) * P.plane + (long long)i * P.pitch + tj, w,
                    slot_word(w0, L::OFF + Q));
        return;
    }
    ti += ti < 0 ? P.Nz : -P.Nz;  // periodic
    float w = v;
    if constexpr (ENC) w = w - pop_off<FLD>(Q, Ln);
    Conv<S>::st(A + (L::OFF + Q) * P.plane + (long long)ti * P.pitch + tj, w,
                slot_word(w0, L::OFF + Q));
}

template <class S, int FLD, int Q, bool ENC = kEnc<S>>
__device__ __forceinline__ void push(const KParams &P, S *A, int i, int j, float v, unsigned w0,
                                     const Lag4 &Ln) {
    using L = Lat<FLD>;
    constexpr int ex = L::ex(Q), ey = L::ey(Q);
    const int ti = i + ex, tj = j + ey;
    if ((unsigned)ti < (unsigned)P.Nz && (unsigned)tj < (unsigned)P.Nr) {
        float w = v;
        if constexpr (ENC) w = w - pop_off<FLD>(Q, Ln);
        Conv<S>::st(A + (L::OFF + Q) * P.plane + (long long)ti * P.pitch + tj, w,
                    slot_word(w0, L::OFF + Q));
        return;
    }
    push_edge<S, FLD, Q, ENC>(P, A, i, j, v, w0, Ln);
}

// ----------------------------------------------------------------------------
// Derivative field v (0 u_x, 1 u_y, 2 u_theta, 3 T - T_ref) at the
// neighbour (i + di, j + dj) of fluid node (i, j).  get(v, di, dj) returns
// the field at a fluid neighbour, or at the periodic image of a neighbour
// beyond a periodic face; beyond a wall or the axis the value is a ghost
// mirrored through the half-way wall: -q for u_x, u_y at a no-slip wall,
// 2 q_w - q for an imposed u_theta or T, q for zero flux; q (u_x, T) or -q
// (u_y, u_theta) at the axis; -q for u_x and q for u_y at a free surface,
// with q = get(v, 0, 0) the node's own value.
template <class Get>
__device__ __forceinline__ float field_at(const KParams &P, const Get &get, int v, int i, int j,
                                          int di, int dj) {
    const int ni = i + di, nj = j + dj;
    if ((unsigned)ni < (unsigned)P.Nz && (unsigned)nj < (unsigned)P.Nr) return get(v, di, dj);
    const int face = nj < 0 ? R_IN : (nj >= P.Nr ? R_OUT : (ni < 0 ? Z_LO : Z_HI));
    const int fld = v <= 1 ? FLOW : (v == 2 ? SWIRL : THERMAL);
    const int c2 = 2 * j;  // an axial neighbour: the node's own column
    const int k = kind_at(P, face, fld, c2);
    if (k == PERIODIC || k == HALO) return get(v, di, dj);
    const float q1 = get(v, 0, 0);
    if (k == MIRROR) return (v == 0 || v == 3) ? q1 : -q1;
    if (k == ADIABATIC) return q1;
    if (k == SLIP) return v == 0 ? -q1 : q1;  // free surface: u_x = 0, d_x u_y = 0
    if (v <= 1) {
        // the velocity component normal to a wall that imposes one: 2 u_w - q
        const int normal = face <= R_OUT ? 1 : 0;
        return v == normal ? 2.f * face_velocity(P, face, c2) - q1 : -q1;
    }
    const float yw = P.r0 + (float)j + 0.5f + 0.5f * (float)dj;
    const float s = v == 2 ? wall_value<SWIRL>(P, face, c2, yw) : wall_value<THERMAL>(P, face, c2, yw);
    return 2.f * s - q1;
}

// Central differences d = {d_x u_y, d_y u_x, d_y u_y, d_y u_theta, d_y T}
// at fluid node (i, j) from a field source as in field_at.
template <class Get>
__device__ __forceinline__ void differences(const KParams &P, const Get &get, int i, int j,
                                            float d[5]) {
    d[0] = 0.5f * (field_at(P, get, 1, i, j, +1, 0) - field_at(P, get, 1, i, j, -1, 0));
    d[1] = 0.5f * (field_at(P, get, 0, i, j, 0, +1) - field_at(P, get, 0, i, j, 0, -1));
    d[2] = 0.5f * (field_at(P, get, 1, i, j, 0, +1) - field_at(P, get, 1, i, j, 0, -1));
    d[3] = 0.5f * (field_at(P, get, 2, i, j, 0, +1) - field_at(P, get, 2, i, j, 0, -1));
    d[4] = 0.5f * (field_at(P, get, 3, i, j, 0, +1) - field_at(P, get, 3, i, j, 0, -1));
}

// An LDS tile of the four derivative fields as a field source: (ta, tb) is
// the node's cell; periodic images sit in the cells beyond the domain.
template <int H, int W>
struct TileSource {
    const float (&F)[4][H][W];
    int ta, tb;
    __device__ __forceinline__ float operator()(int v, int di, int dj) const {
        return F[v][ta + di][tb + dj];
    }
};

// The lagged fields of the previous step (format of population storage S)
// as a field source (periodic images wrap along z; beyond a HALO face, the
// halo row's fields).
template <class S>
struct LagSource {
    const KParams &P;
    const char *M;
    int i, j;
    __device__ __forceinline__ float operator()(int v, int di, int dj) const {
        int ni = i + di;
        if ((unsigned)ni >= (unsigned)P.Nz) {
            const int f = ni < 0 ? 0 : 1;
            if (kind_of(P, Z_LO + f, FLOW) == HALO)
                return lag_ld<S>(P.halo_lag[f], v, (long long)P.pitch, j + dj);
            ni += ni < 0 ? P.Nz : -P.Nz;
        }
        return lag_ld<S>(M, v, P.plane, (long long)ni * P.pitch + (j + dj));
    }
};

// ----------------------------------------------------------------------------
// The pre-collision half step (eq. 21, 38, 48) with the geometric sources of
// eq. (4), (7), (9) and the body force of eq. (5) evaluated at that same
// half-step state: the relations are solved per node, the terms linear in
// the unknowns on the left and a few fixed-point sweeps for the weak
// remainder.  Everything is carried as increments (half of each source) so
// that a source of 1e-8 is not lost against O(1) fields in FP32.
struct Half {
    float drho, irho, ux, uy, psi, dphi;  // state seen by the collision (rho = 1 + drho)
    float hMA, hFx, hFy, hSpsi, hSphi;    // half of each source
};

constexpr int HALF_SWEEPS = 3;

// Reciprocal by the hardware instruction (within 1 ulp): the half step only
// needs FP32 accuracy, and IEEE division costs ~10 instructions each.
__device__ __forceinline__ float rcp(float x) { return __builtin_amdgcn_rcpf(x); }

__device__ __forceinline__ Half half_step(const KParams &P, float iy, float drho_o, float jx_o,
                                          float jy_o, float psi_o, float dphi_o, const float d[5]) {
    const float nu = P.nu, iy2 = iy * iy;
    const float rho_o = 1.f + drho_o;
    const float nuiy2 = nu * iy2;
    const float ify = rcp(1.f + nuiy2);  // F_y terms linear in rho u_y
    const float sy2 = nu * d[2] * iy, st2 = 0.5f * nu * d[3] * iy;
    float hMA = 0.f, hFy = 0.f, hSpsi = 0.f;
    float Jy = jy_o, rho = rho_o, psi = psi_o;
#pragma unroll
    for (int it = 0; it < HALF_SWEEPS; ++it) {
        hMA = -0.5f * Jy * iy;                      // M^A/2 = -rho u_y/(2y)
        rho = rho_o + hMA;
        const float irho = rcp(rho);
        const float a = Jy * irho * iy + 0.5f * nuiy2;  // S_psi terms linear in psi
        hSpsi = (rho * st2 - psi_o * a) * rcp(1.f + a);
        psi = psi_o + hSpsi;
        hFy = (0.5f * (psi * psi - Jy * Jy) * irho * iy + rho * sy2 - nuiy2 * jy_o) * ify;
        Jy = jy_o + hFy;
    }
    hMA = -0.5f * Jy * iy;
    rho = rho_o + hMA;
    const float irho = rcp(rho);
    const float b = 0.5f * Jy * irho * iy;  // terms linear in phi and in rho u_x
    const float ib = rcp(1.f + b);
    const float phi_o = P.Tref + dphi_o;
    const float hSphi = (0.5f * P.alpha * d[4] * iy - phi_o * b) * ib;
    const float dphi = dphi_o + hSphi;
    const float Fb = P.g_axial + P.gbeta * (P.Tref - P.T0 + dphi);
    const float hFx = (0.5f * (rho * nu * (d[0] + d[1]) * iy + Fb) - jx_o * b) * ib;
    Half H;
    H.drho = drho_o + hMA;
    H.irho = irho;
    H.ux = (jx_o + hFx) * irho;
    H.uy = Jy * irho;
    H.psi = psi;
    H.dphi = dphi;
    H.hMA = hMA; H.hFx = hFx; H.hFy = hFy; H.hSpsi = hSpsi; H.hSphi = hSphi;
    return H;
}

// Cascaded D2Q9 collision, eq. (17), with the source moments of eq. (26)
// (p_0 = M^A/9, p_1 = F_x/6, p_2 = F_y/6) and f^p = f + K p (eq. 16a, 27).
// f holds shifted populations f - w_q; with rho = 1 + drho the constant parts
// of the raw moments (1/3 for xx, yy; 1/9 for xxyy) cancel against the
// equilibrium terms in closed form, leaving only small quantities.
__device__ __forceinline__ void collide_f(const KParams &P, float (&f)[9], const Half &H) {
    const float ux = H.ux, uy = H.uy, drho = H.drho, rho = 1.f + drho;
    const float ux2 = ux * ux, uy2 = uy * uy;
    const float kxx = f[1] + f[3] + f[5] + f[6] + f[7] + f[8];
    const float kyy = f[2] + f[4] + f[5] + f[6] + f[7] + f[8];
    const float kxy = f[5] - f[6] + f[7] - f[8];
    const float kxxy = f[5] + f[6] - f[7] - f[8];
    const float kxyy = f[5] - f[6] - f[7] + f[8];
    const float kxxyy = f[5] + f[6] + f[7] + f[8];
    const float p0 = (2.f / 9.f) * H.hMA;
    const float p1 = (1.f / 3.f) * H.hFx;
    const float p2 = (1.f / 3.f) * H.hFy;
    const float p3 = P.om3 * (1.f / 12.f) * ((2.f / 3.f) * drho + rho * (ux2 + uy2) - (kxx + kyy));
    const float p4 = P.om45 * 0.25f * (rho * (ux2 - uy2) - (kxx - kyy));
    const float p5 = P.om45 * 0.25f * (rho * ux * uy - kxy);
    const float p6 = P.om6 * 0.25f * (2.f * rho * ux2 * uy + kxxy - 2.f * ux * kxy -
                                      uy * ((1.f / 3.f) + kxx)) -
                     0.5f * uy * (3.f * p3 + p4) - 2.f * ux * p5;
    const float p7 = P.om7 * 0.25f * (2.f * rho * ux * uy2 + kxyy - 2.f * uy * kxy -
                                      ux * ((1.f / 3.f) + kyy)) -
                     0.5f * ux * (3.f * p3 - p4) - 2.f * uy * p5;
    const float p8 =
        P.om8 * 0.25f *
            ((1.f / 9.f) * drho + 3.f * rho * ux2 * uy2 -
             (kxxyy - 2.f * ux * kxyy - 2.f * uy * kxxy + ux2 * ((1.f / 3.f) + kyy) +
              uy2 * ((1.f / 3.f) + kxx) + 4.f * ux * uy * kxy)) -
        2.f * p3 - 0.5f * uy2 * (3.f * p3 + p4) - 0.5f * ux2 * (3.f * p3 - p4) -
        4.f * ux * uy * p5 - 2.f * uy * p6 - 2.f * ux * p7;
    // f += K p with the columns of K grouped so that shared partial sums
    // are formed once
    const float a = p0 - p3, ax = a + p4, ay = a - p4;
    const float c = p0 + 2.f * p3 + p8, cu = p1 + p2, cv = p1 - p2;
    const float s67 = p6 + p7, d67 = p7 - p6;
    f[0] += p0 - 4.f * (p3 - p8);
    f[1] += (ax + p1) + 2.f * (p7 - p8);
    f[3] += (ax - p1) - 2.f * (p7 + p8);
    f[2] += (ay + p2) + 2.f * (p6 - p8);
    f[4] += (ay - p2) - 2.f * (p6 + p8);
    f[5] += (c + cu) + (p5 - s67);
    f[7] += (c - cu) + (p5 + s67);
    f[6] += (c - cv) + (d67 - p5);
    f[8] += (c + cv) - (d67 + p5);
}

// Cascaded D2Q5 collision for an advected scalar s = s_ref + ds stored as
// g - w_q s_ref (eq. 34 for psi with s_ref = 0, eq. 49 for T with s_ref =
// T_ref): relaxation of the central moments of eq. (31)/(43) to their
// Maxwellian values gives a minus sign in front of |u|^2 s and
// (u_x^2 - u_y^2) s.  Source moment q_0 = S/5 (eq. 41, 51), g^p = g + L q
// (eq. 42, 52).
__device__ __forceinline__ void collide_adv(float (&g)[5], float ux, float uy, float s,
                                            float ds, float hS, float o12, float o3, float o4) {
    const float kx = g[1] - g[3], ky = g[2] - g[4];
    const float kxx = g[1] + g[3], kyy = g[2] + g[4];
    const float q0 = 0.4f * hS;
    const float q1 = 0.5f * o12 * (s * ux - kx);
    const float q2 = 0.5f * o12 * (s * uy - ky);
    const float q3 = 0.25f * o3 *
                         ((2.f / 3.f) * ds - (kxx + kyy) + 2.f * (ux * kx + uy * ky) -
                          (ux * ux + uy * uy) * s) +
                     ux * q1 + uy * q2;
    const float q4 = 0.25f * o4 *
                         (-(kxx - kyy) + 2.f * (ux * kx - uy * ky) - (ux * ux - uy * uy) * s) +
                     ux * q1 - uy * q2;
    const float a = q0 + q3, ax = a + q4, ay = a - q4;
    g[0] += q0 - 4.f * q3;
    g[1] += ax + q1;
    g[3] += ax - q1;
    g[2] += ay + q2;
    g[4] += ay - q2;
}

// Output moments (eq. 18, 35, 47) and central differences of the lagged
// fields for node (i, j).
struct Moments {
    float drho, jx, jy, psi, dphi;
};

__device__ __forceinline__ Moments moments(const float (&f)[9], const float (&g)[5],
                                           const float (&h)[5]) {
    Moments m;
    m.drho = ((f[0] + f[1]) + (f[2] + f[3])) + ((f[4] + f[5]) + (f[6] + f[7])) + f[8];
    m.jx = (f[1] - f[3]) + (f[5] - f[6]) + (f[8] - f[7]);
    m.jy = (f[2] - f[4]) + (f[5] - f[8]) + (f[6] - f[7]);
    m.psi = (g[0] + g[1]) + (g[2] + g[3]) + g[4];
    m.dphi = (h[0] + h[1]) + (h[2] + h[3]) + h[4];
    return m;
}

template <class S>
__device__ __forceinline__ void derivatives(const KParams &P, const char *M, int i, int j,
                                            bool interior, float d[5]) {
    if (interior) {
        // all four neighbours are fluid nodes: plain loads at 32-bit offsets
        const unsigned n = (unsigned)i * (unsigned)P.pitch + (unsigned)j, w = (unsigned)P.pitch;
        const long long pl = P.plane;
        d[0] = 0.5f * (lag_ld<S>(M, 1, pl, n + w) - lag_ld<S>(M, 1, pl, n - w));
        d[1] = 0.5f * (lag_ld<S>(M, 0, pl, n + 1) - lag_ld<S>(M, 0, pl, n - 1));
        d[2] = 0.5f * (lag_ld<S>(M, 1, pl, n + 1) - lag_ld<S>(M, 1, pl, n - 1));
        d[3] = 0.5f * (lag_ld<S>(M, 2, pl, n + 1) - lag_ld<S>(M, 2, pl, n - 1));
        d[4] = 0.5f * (lag_ld<S>(M, 3, pl, n + 1) - lag_ld<S>(M, 3, pl, n - 1));
        return;
    }
    differences(P, LagSource<S>{P, M, i, j}, i, j, d);
}

// ----------------------------------------------------------------------------
// Tile mapping: a workgroup updates TX x TY nodes (r x z), one node per
// thread; with TX >= 64 a wavefront spans 64 consecutive r, so every plane
// access is one contiguous 256-byte run in FP32.  Consecutive workgroup ids
// are dealt round-robin over the 8 XCDs; they are remapped so that each XCD
// owns one contiguous band of tiles and the neighbour rows an update touches
// stay in that XCD's L2.
constexpr int TX = 64, TY = 4;  // tile of the field, init and default step kernels

template <int BX, int BY>
__device__ __forceinline__ void tile_of(const KParams &P, int &i, int &j) {
    const int gx = (P.Nr + BX - 1) / BX;
    const int gy = (P.Nz + BY - 1) / BY;
    const int nb = gx * gy;
    const int b = blockIdx.x;
    const int xcd = b & 7, k = b >> 3;
    const int q = nb >> 3, r = nb & 7;
    const int t = xcd * q + (xcd < r ? xcd : r) + k;
    j = (t % gx) * BX + (int)threadIdx.x % BX;
    i = (t / gx) * BY + (int)threadIdx.x / BX;
}

enum Mode { MODE_AB = 0, MODE_AA_ODD = 1, MODE_AA_EVEN = 2 };

// Interior pull: the source node n - e_q is a fluid node (32-bit offsets
// against a uniform plane base).  With offset encoding the source node wrote
// the slot, for direction Q in both slot conventions.
template <class S, bool AA, int FLD, int Q, bool ENC = kEnc<S>>
__device__ __forceinline__ float pull_in(const KParams &P, const S *A, const char *M, unsigned n) {
    using L = Lat<FLD>;
    constexpr int slot = AA ? L::opp(Q) : Q;
    const unsigned dn = (unsigned)(L::ex(Q) * P.pitch + L::ey(Q));
    float v = Conv<S>::ld(A + (long long)(L::OFF + slot) * P.plane + (n - dn));
    if constexpr (ENC) v = v + pop_off<FLD>(Q, lag_node<S>(P, M, n - dn));
    return v;
}

template <class S, int FLD, int Q>
__device__ __forceinline__ void push_in(const KParams &P, S *A, unsigned n, float v, unsigned w0) {
    using L = Lat<FLD>;
    const unsigned dn = (unsigned)(L::ex(Q) * P.pitch + L::ey(Q));
    Conv<S>::st(A + (long long)(L::OFF + Q) * P.plane + (n + dn), v, slot_word(w0, L::OFF + Q));
}

// Offset decoding of the populations x of distribution FLD that node (i, j)
// read from its own slots in the AA even phase (even_off per population).
template <class S, int FLD, int N, int... Q>
__device__ __forceinline__ void even_offsets(const KParams &P, const char *M, int i, int j,
                                             float (&x)[N], std::integer_sequence<int, Q...>) {
    ((x[Q] = x[Q] + even_off<S, FLD, Q>(P, M, i, j)), ...);
}
// The same where every source node n - e_q is a fluid node (n the node's
// element offset): the writer of population q is n - e_q.
template <class S, int FLD, int N, int... Q>
__device__ __forceinline__ void link_offsets(const KParams &P, const char *M, unsigned n,
                                             float (&x)[N], std::integer_sequence<int, Q...>) {
    ((x[Q] = x[Q] + pop_off<FLD>(Q, lag_node<S>(P, M, n - (unsigned)(Lat<FLD>::ex(Q) * P.pitch +
                                                                        Lat<FLD>::ey(Q))))),
     ...);
}
template <class S>
__device__ __forceinline__ void decode_even(const KParams &P, const char *M, int i, int j,
                                            bool interior, float (&f)[9], float (&g)[5],
                                            float (&h)[5]) {
    if (interior) {
        const unsigned n = (unsigned)i * (unsigned)P.pitch + (unsigned)j;
        link_offsets<S, FLOW>(P, M, n, f, std::make_integer_sequence<int, 9>{});
        link_offsets<S, SWIRL>(P, M, n, g, std::make_integer_sequence<int, 5>{});
        link_offsets<S, THERMAL>(P, M, n, h, std::make_integer_sequence<int, 5>{});
    } else {
        even_offsets<S, FLOW>(P, M, i, j, f, std::make_integer_sequence<int, 9>{});
        even_offsets<S, SWIRL>(P, M, i, j, g, std::make_integer_sequence<int, 5>{});
        even_offsets<S, THERMAL>(P, M, i, j, h, std::make_integer_sequence<int, 5>{});
    }
}

// Post-collision populations as a node stores them: minus the offsets of
// its own stored lagged fields Ln (direction q) with offset encoding.
template <bool ENC>
__device__ __forceinline__ void encode(const float (&f)[9], const float (&g)[5],
                                       const float (&h)[5], const Lag4 &Ln, float (&ef)[9],
                                       float (&eg)[5], float (&eh)[5]) {
#pragma unroll
    for (int q = 0; q < 9; ++q) {
        ef[q] = f[q];
        if constexpr (ENC) ef[q] = f[q] - pop_off<FLOW>(q, Ln);
    }
#pragma unroll
    for (int q = 0; q < 5; ++q) {
        eg[q] = g[q];
        eh[q] = h[q];
        if constexpr (ENC) {
            eg[q] = g[q] - pop_off<SWIRL>(q, Ln);
            eh[q] = h[q] - pop_off<THERMAL>(q, Ln);
        }
    }
}

// The 19 populations node (i, j) streams in from state A (lagged fields M
// of the same step), in slot convention MODE.
template <class S, int MODE, bool ENC = kEnc<S>>
__device__ __forceinline__ void gather(const KParams &P, const S *A, const char *M, int i, int j,
                                       bool interior, float (&f)[9], float (&g)[5],
                                       float (&h)[5]) {
    const unsigned n = (unsigned)i * (unsigned)P.pitch + (unsigned)j;
    if (MODE == MODE_AA_EVEN) {
#pragma unroll
        for (int q = 0; q < 9; ++q) f[q] = Conv<S>::ld(A + (long long)q * P.plane + n);
#pragma unroll
        for (int q = 0; q < 5; ++q) {
            g[q] = Conv<S>::ld(A + (long long)(GOFF + q) * P.plane + n);
            h[q] = Conv<S>::ld(A + (long long)(HOFF + q) * P.plane + n);
        }
        if constexpr (ENC) decode_even<S>(P, M, i, j, interior, f, g, h);
        return;
    }
    constexpr bool AA = MODE == MODE_AA_ODD;
    if (interior) {
        f[0] = pull_in<S, AA, FLOW, 0, ENC>(P, A, M, n);
        f[1] = pull_in<S, AA, FLOW, 1, ENC>(P, A, M, n);
        f[2] = pull_in<S, AA, FLOW, 2, ENC>(P, A, M, n);
        f[3] = pull_in<S, AA, FLOW, 3, ENC>(P, A, M, n);
        f[4] = pull_in<S, AA, FLOW, 4, ENC>(P, A, M, n);
        f[5] = pull_in<S, AA, FLOW, 5, ENC>(P, A, M, n);
        f[6] = pull_in<S, AA, FLOW, 6, ENC>(P, A, M, n);
        f[7] = pull_in<S, AA, FLOW, 7, ENC>(P, A, M, n);
        f[8] = pull_in<S, AA, FLOW, 8, ENC>(P, A, M, n);
        g[0] = pull_in<S, AA, SWIRL, 0, ENC>(P, A, M, n);
        g[1] = pull_in<S, AA, SWIRL, 1, ENC>(P, A, M, n);
        g[2] = pull_in<S, AA, SWIRL, 2, ENC>(P, A, M, n);
        g[3] = pull_in<S, AA, SWIRL, 3, ENC>(P, A, M, n);
        g[4] = pull_in<S, AA, SWIRL, 4, ENC>(P, A, M, n);
        h[0] = pull_in<S, AA, THERMAL, 0, ENC>(P, A, M, n);
        h[1] = pull_in<S, AA, THERMAL, 1, ENC>(P, A, M, n);
        h[2] = pull_in<S, AA, THERMAL, 2, ENC>(P, A, M, n);
        h[3] = pull_in<S, AA, THERMAL, 3, ENC>(P, A, M, n);
        h[4] = pull_in<S, AA, THERMAL, 4, ENC>(P, A, M, n);
        return;
    }
    pull_all<AA>(P, GlobalPops<S, ENC, AA>{P, A, M}, i, j, f, g, h);
}

// Stores the post-collision populations of node (i, j) in slot convention
// MODE; Ln: the node's lagged fields as stored (offset encoding).
template <class S, int MODE, bool ENC = kEnc<S>>
__device__ __forceinline__ void scatter(const KParams &P, S *A, int i, int j, bool interior,
                                        const float (&f)[9], const float (&g)[5],
                                        const float (&h)[5], const Lag4 &Ln) {
    const unsigned n = (unsigned)i * (unsigned)P.pitch + (unsigned)j;
    const unsigned w0 = node_word(f, g, h, i + P.row0, j);
    if (MODE == MODE_AA_ODD && !interior) {
        push<S, FLOW, 0, ENC>(P, A, i, j, f[0], w0, Ln);
        push<S, FLOW, 1, ENC>(P, A, i, j, f[1], w0, Ln);
        push<S, FLOW, 2, ENC>(P, A, i, j, f[2], w0, Ln);
        push<S, FLOW, 3, ENC>(P, A, i, j, f[3], w0, Ln);
        push<S, FLOW, 4, ENC>(P, A, i, j, f[4], w0, Ln);
        push<S, FLOW, 5, ENC>(P, A, i, j, f[5], w0, Ln);
        push<S, FLOW, 6, ENC>(P, A, i, j, f[6], w0, Ln);
        push<S, FLOW, 7, ENC>(P, A, i, j, f[7], w0, Ln);
        push<S, FLOW, 8, ENC>(P, A, i, j, f[8], w0, Ln);
        push<S, SWIRL, 0, ENC>(P, A, i, j, g[0], w0, Ln);
        push<S, SWIRL, 1, ENC>(P, A, i, j, g[1], w0, Ln);
        push<S, SWIRL, 2, ENC>(P, A, i, j, g[2], w0, Ln);
        push<S, SWIRL, 3, ENC>(P, A, i, j, g[3], w0, Ln);
        push<S, SWIRL, 4, ENC>(P, A, i, j, g[4], w0, Ln);
        push<S, THERMAL, 0, ENC>(P, A, i, j, h[0], w0, Ln);
        push<S, THERMAL, 1, ENC>(P, A, i, j, h[1], w0, Ln);
        push<S, THERMAL, 2, ENC>(P, A, i, j, h[2], w0, Ln);
        push<S, THERMAL, 3, ENC>(P, A, i, j, h[3], w0, Ln);
        push<S, THERMAL, 4, ENC>(P, A, i, j, h[4], w0, Ln);
        return;
    }
    float ef[9], eg[5], eh[5];
    encode<ENC>(f, g, h, Ln, ef, eg, eh);
    if (MODE == MODE_AB) {
#pragma unroll
        for (int q = 0; q < 9; ++q)
            Conv<S>::st(A + (long long)q * P.plane + n, ef[q], slot_word(w0, q));
#pragma unroll
        for (int q = 0; q < 5; ++q) {
            Conv<S>::st(A + (long long)(GOFF + q) * P.plane + n, eg[q], slot_word(w0, GOFF + q));
            Conv<S>::st(A + (long long)(HOFF + q) * P.plane + n, eh[q], slot_word(w0, HOFF + q));
        }
    } else if (MODE == MODE_AA_EVEN) {
#pragma unroll
        for (int q = 0; q < 9; ++q)
            Conv<S>::st(A + (long long)Lat<FLOW>::opp(q) * P.plane + n, ef[q], slot_word(w0, q));
#pragma unroll
        for (int q = 0; q < 5; ++q) {
            Conv<S>::st(A + (long long)(GOFF + Lat<SWIRL>::opp(q)) * P.plane + n, eg[q],
                        slot_word(w0, GOFF + q));
            Conv<S>::st(A + (long long)(HOFF + Lat<THERMAL>::opp(q)) * P.plane + n, eh[q],
                        slot_word(w0, HOFF + q));
        }
    } else {
        push_in<S, FLOW, 0>(P, A, n, ef[0], w0);
        push_in<S, FLOW, 1>(P, A, n, ef[1], w0);
        push_in<S, FLOW, 2>(P, A, n, ef[2], w0);
        push_in<S, FLOW, 3>(P, A, n, ef[3], w0);
        push_in<S, FLOW, 4>(P, A, n, ef[4], w0);
        push_in<S, FLOW, 5>(P, A, n, ef[5], w0);
        push_in<S, FLOW, 6>(P, A, n, ef[6], w0);
        push_in<S, FLOW, 7>(P, A, n, ef[7], w0);
        push_in<S, FLOW, 8>(P, A, n, ef[8], w0);
        push_in<S, SWIRL, 0>(P, A, n, eg[0], w0);
        push_in<S, SWIRL, 1>(P, A, n, eg[1], w0);
        push_in<S, SWIRL, 2>(P, A, n, eg[2], w0);
        push_in<S, SWIRL, 3>(P, A, n, eg[3], w0);
        push_in<S, SWIRL, 4>(P, A, n, eg[4], w0);
        push_in<S, THERMAL, 0>(P, A, n, eh[0], w0);
        push_in<S, THERMAL, 1>(P, A, n, eh[1], w0);
        push_in<S, THERMAL, 2>(P, A, n, eh[2], w0);
        push_in<S, THERMAL, 3>(P, A, n, eh[3], w0);
        push_in<S, THERMAL, 4>(P, A, n, eh[4], w0);
    }
}

// A node whose eight neighbours are all fluid nodes: no boundary rule can
// apply to any of its links or derivative stencils.  False for every (i, j)
// outside the lattice, also when Nz or Nr is below 3 (the tile kernels of
// the odd phase rely on that to skip the ragged tail).
__device__ __forceinline__ bool interior_node(const KParams &P, int i, int j) {
    return i >= 1 && i <= P.Nz - 2 && j >= 1 && j <= P.Nr - 2;
}

// The nodes on the edge of a lattice, where boundary rules may apply:
// columns j = 0 and j = Nr - 1 (every row), then rows i = 0 and i = Nz - 1
// without their end nodes (one row when Nz = 1).  Every other node is
// interior_node.  Edge nodes run in workgroups of their own, so that the
// waves of interior tiles never diverge into the boundary code.
__host__ __device__ __forceinline__ int edge_count(int Nr, int Nz) {
    return 2 * Nz + (Nr - 2) * (Nz >= 2 ? 2 : 1);
}
// Workgroups of `threads` that the edge nodes of one lattice take in a
// single-lattice launch: a multiple of 8 (one per XCD in turn).
__host__ __device__ __forceinline__ int edge_blocks(int Nr, int Nz, int threads) {
    return ((edge_count(Nr, Nz) + threads - 1) / threads + 7) / 8 * 8;
}
__device__ __forceinline__ void edge_node(const KParams &P, int e, int &i, int &j) {
    if (e < 2 * P.Nz) {
        j = e < P.Nz ? 0 : P.Nr - 1;
        i = e < P.Nz ? e : e - P.Nz;
        return;
    }
    e -= 2 * P.Nz;
    const int w = P.Nr - 2;
    i = e < w ? 0 : P.Nz - 1;
    j = 1 + (e < w ? e : e - w);
}

// One time step of node (i, j): stream (gather), output moments, half
// source step, cascaded collisions with the source moments, store; the
// node's half-step fields go to the lagged buffer of the next step.
// `interior` must equal interior_node(P, i, j); callers pass a constant.
// Output moments, half source step and the three collisions of a node in
// row j whose pulled populations are f, g, h and whose central differences
// are d; f, g, h become the post-collision populations, and the half-step
// state (the node's lagged fields) is returned.
__device__ __forceinline__ Half relax_node(const KParams &P, int j, float (&f)[9], float (&g)[5],
                                           float (&h)[5], const float d[5]) {
    const Moments m = moments(f, g, h);
    const float iy = rcp(P.r0 + (float)j + 0.5f);
    const Half H = half_step(P, iy, m.drho, m.jx, m.jy, m.psi, m.dphi, d);
    collide_f(P, f, H);
    collide_adv(g, H.ux, H.uy, H.psi, H.psi, H.hSpsi, P.og12, P.og3, P.og4);
    collide_adv(h, H.ux, H.uy, P.Tref + H.dphi, H.dphi, H.hSphi, P.oh12, P.oh3, P.oh4);
    return H;
}

template <class S, int MODE>
__device__ __forceinline__ void update_node(const KParams &P, const S *src, S *dst,
                                            const char *__restrict__ Mprev,
                                            char *__restrict__ Mnext, int i, int j,
                                            bool interior) {
    float f[9], g[5], h[5];
    gather<S, MODE>(P, src, Mprev, i, j, interior, f, g, h);
    float d[5];
    derivatives<S>(P, Mprev, i, j, interior, d);
    const Half H = relax_node(P, j, f, g, h, d);
    scatter<S, MODE>(P, dst, i, j, interior, f, g, h,
                     lag_stored<S>(H.ux, H.uy, H.psi * H.irho, H.dphi));
    const unsigned n = (unsigned)i * (unsigned)P.pitch + (unsigned)j;
    lag_st<S>(Mnext, 0, P.plane, n, H.ux);
    lag_st<S>(Mnext, 1, P.plane, n, H.uy);
    lag_st<S>(Mnext, 2, P.plane, n, H.psi * H.irho);
    lag_st<S>(Mnext, 3, P.plane, n, H.dphi);
}

// ----------------------------------------------------------------------------
// Accesses through device-memory (address space 1) pointers: the compiler
// then emits global instructions with an SGPR base and a 32-bit VGPR
// offset, also where the base was read from memory (a plain pointer read
// from memory would give flat instructions with a 64-bit address each).
using gbyte = __attribute__((address_space(1))) char;
template <class T>
__device__ __forceinline__ T gload(const char *base, unsigned off) {
    return *(const __attribute__((address_space(1))) T *)((const gbyte *)base + off);
}
template <class T>
__device__ __forceinline__ void gstore(char *base, unsigned off, T v) {
    *(__attribute__((address_space(1))) T *)((gbyte *)base + off) = v;
}
template <class S>
using StoreBits = std::conditional_t<sizeof(S) == 4, float, unsigned short>;

template <class S>
__device__ __forceinline__ float ld_plane(const char *base, unsigned off) {
    const S v = __builtin_bit_cast(S, gload<StoreBits<S>>(base, off));
    return Conv<S>::ld(&v);
}
template <class S>
__device__ __forceinline__ void st_plane(char *base, unsigned off, float x, unsigned rnd,
                                         typename Conv<S>::Reg &r) {
    gstore(base, off, Conv<S>::bits(x, rnd, r));
}
// A lagged velocity (format of population storage S) at byte offset off.
template <class S>
__device__ __forceinline__ float lag_plane(const char *base, unsigned off) {
    using F = LagFmt<S>;
    return F::dec(gload<typename F::Bits>(base, off));
}

// The 19 populations node (i, j) reads (gather_planes) or writes
// (scatter_planes) through plane addresses; o is the node's byte offset
// n * sizeof(S).
template <class S>
__device__ __forceinline__ void gather_planes(const Planes &A, unsigned o, float (&f)[9],
                                              float (&g)[5], float (&h)[5]) {
#pragma unroll
    for (int q = 0; q < 9; ++q) f[q] = ld_plane<S>(A.rd[q], o);
#pragma unroll
    for (int q = 0; q < 5; ++q) {
        g[q] = ld_plane<S>(A.rd[GOFF + q], o);
        h[q] = ld_plane<S>(A.rd[HOFF + q], o);
    }
}
// Ln: the node's lagged fields as stored (offset encoding); gi: the node's
// global row (rounding key).
template <class S, bool ENC = kEnc<S>>
__device__ __forceinline__ void scatter_planes(const Planes &A, unsigned o, int gi, int j,
                                               const float (&f)[9], const float (&g)[5],
                                               const float (&h)[5], const Lag4 &Ln) {
    typename Conv<S>::Reg r{};
    const unsigned w0 = node_word(f, g, h, gi, j);
    float ef[9], eg[5], eh[5];
    encode<ENC>(f, g, h, Ln, ef, eg, eh);
#pragma unroll
    for (int q = 0; q < 9; ++q) st_plane<S>(A.wr[q], o, ef[q], slot_word(w0, q), r);
#pragma unroll
    for (int q = 0; q < 5; ++q) {
        st_plane<S>(A.wr[GOFF + q], o, eg[q], slot_word(w0, GOFF + q), r);
        st_plane<S>(A.wr[HOFF + q], o, eh[q], slot_word(w0, HOFF + q), r);
    }
}

// Offset decoding of populations gathered through plane addresses where
// every source node n - e_q is a fluid node (n: the node's element offset):
// the writer's lagged fields through the launch's lagged-field planes, the
// values lag_node gives.
template <class S>
__device__ __forceinline__ Lag4 lag_planes(const Planes &A, unsigned m) {
    using F = LagFmt<S>;
    return {lag_plane<S>(A.lrd[0], m * F::VB), lag_plane<S>(A.lrd[1], m * F::VB),
            lag_plane<S>(A.lrd[2], m * F::VB), gload<float>(A.lrd[3], m * 4u)};
}
template <class S, int FLD, int N, int... Q>
__device__ __forceinline__ void link_offsets_planes(const KParams &P, const Planes &A, unsigned n,
                                                    float (&x)[N],
                                                    std::integer_sequence<int, Q...>) {
    ((x[Q] = x[Q] + pop_off<FLD>(Q, lag_planes<S>(A, n - (unsigned)(Lat<FLD>::ex(Q) * P.pitch +
                                                                     Lat<FLD>::ey(Q))))),
     ...);
}
template <class S>
__device__ __forceinline__ void decode_planes(const KParams &P, const Planes &A, unsigned n,
                                              float (&f)[9], float (&g)[5], float (&h)[5]) {
    link_offsets_planes<S, FLOW>(P, A, n, f, std::make_integer_sequence<int, 9>{});
    link_offsets_planes<S, SWIRL>(P, A, n, g, std::make_integer_sequence<int, 5>{});
    link_offsets_planes<S, THERMAL>(P, A, n, h, std::make_integer_sequence<int, 5>{});
}
// A register copy of a byte offset that the compiler cannot trace back to
// an earlier basic block: it chooses the SGPR-base address form per block,
// only for an offset it sees widened from 32 bits in the same block.
__device__ __forceinline__ unsigned local_offset(unsigned o) {
    asm volatile("" : "+v"(o));
    return o;
}

// The same update through a launch's plane addresses (Planes), for the tile
// workgroups of the step kernel: valid for every node in the AA even phase
// (each node reads and writes its own slots) and for interior nodes in the
// AA odd phase and the two-buffer pull.  The arithmetic, the rounding keys
// and the derivative stencils are update_node's, so both give identical
// bits; only the address arithmetic differs (one 32-bit offset per node).
template <class S>
__device__ __forceinline__ void update_planes(const KParams &P, const Planes &A, int i, int j,
                                              bool interior) {
    using F = LagFmt<S>;
    constexpr unsigned VB = F::VB;
    const unsigned n = (unsigned)i * (unsigned)P.pitch + (unsigned)j;
    const unsigned o = n * (unsigned)sizeof(S), ov = n * VB, o4 = n * 4u;
    float f[9], g[5], h[5];
    gather_planes<S>(A, o, f, g, h);
    if constexpr (kEnc<S>) {
        // edge nodes come here in the AA even phase only
        if (interior) decode_planes<S>(P, A, n, f, g, h);
        else decode_even<S>(P, A.lrd[0], i, j, false, f, g, h);
    }
    float d[5];
    if (interior) {
        d[0] = 0.5f * (lag_plane<S>(A.uy_up, ov) - lag_plane<S>(A.uy_dn, ov));
        d[1] = 0.5f * (lag_plane<S>(A.lrd[0], ov + VB) - lag_plane<S>(A.lrd[0], ov - VB));
        d[2] = 0.5f * (lag_plane<S>(A.lrd[1], ov + VB) - lag_plane<S>(A.lrd[1], ov - VB));
        d[3] = 0.5f * (lag_plane<S>(A.lrd[2], ov + VB) - lag_plane<S>(A.lrd[2], ov - VB));
        d[4] = 0.5f * (gload<float>(A.lrd[3], o4 + 4u) - gload<float>(A.lrd[3], o4 - 4u));
    } else {
        differences(P, LagSource<S>{P, A.lrd[0], i, j}, i, j, d);
    }
    const Half H = relax_node(P, j, f, g, h, d);
    // the stores follow the branch above
    const unsigned so = local_offset(o), sov = local_offset(ov), so4 = local_offset(o4);
    scatter_planes<S>(A, so, i + P.row0, j, f, g, h,
                      lag_stored<S>(H.ux, H.uy, H.psi * H.irho, H.dphi));
    gstore(A.lwr[0], sov, F::enc(H.ux));
    gstore(A.lwr[1], sov, F::enc(H.uy));
    gstore(A.lwr[2], sov, F::enc(H.psi * H.irho));
    gstore(A.lwr[3], so4, H.dphi);
}

}  // namespace axlb
