// Device-side definitions of the axisymmetric cascaded LB step for gfx950.
// Internal to the HIP library: the public interface is include/axlb.h.
#pragma once

#include <hip/hip_runtime.h>
#include <hip/hip_fp16.h>
#include <hip/hip_bf16.h>

namespace axlb {

// Faces, distributions and boundary kinds (numbering of include/axlb.h).
enum { R_IN = 0, R_OUT = 1, Z_LO = 2, Z_HI = 3 };
enum { FLOW = 0, SWIRL = 1, THERMAL = 2 };
enum {
    NOSLIP = 0, PERIODIC = 1, MIRROR = 2, DIRICHLET = 3, OMEGA_R = 4, ADIABATIC = 5, HALO = 6,
    VELOCITY = 7, SLIP = 8
};

// Plane numbering of the population buffer: f_0..f_8, g_0..g_4, h_0..h_4.
constexpr int NPOP = 19;
constexpr int GOFF = 9;
constexpr int HOFF = 14;
// Lagged derivative fields, one block per time level: four planes of
// `plane` elements, u_x, u_y, u_theta and T - T_ref.  They are rewritten
// every step and only enter the central differences of the geometric
// sources.  The block is addressed as bytes; its element format follows the
// population storage (LagFmt):
//  * FP32 populations: all four planes FP32 (16 B per node), so that the
//    FP32 path holds FP32 state throughout.  binary16 velocities were
//    measured to cost up to 1e-5 of the speed in u_z near the axis of a
//    cylinder, where the radial differences are divided by r.
//  * 16-bit populations: u_x, u_y, u_theta in binary16 scaled by 2^10
//    (values down to ~6e-8 stay clear of subnormals, |values| up to 64 fit),
//    T - T_ref in FP32 (10 B per node): the velocity rounding stays far
//    below the 16-bit populations' own, while T keeps FP32 because its wall
//    gradient is the Nusselt number.
// Plane 3 (T) starts at byte 3 * plane * VB, 4-byte aligned since plane is
// a multiple of 64.
constexpr int NLAG = 4;
constexpr float LAG_SCALE = 1024.f;

// Scaled binary16 -> FP32 as one mixed-precision FMA (v_fma_mix_f32: the
// binary16 operand is widened inside the instruction); adding +0 instead of
// multiplying only turns a -0 result into +0.
__device__ __forceinline__ float f16_scaled(__half h, float s) {
    return __builtin_fmaf(__half2float(h), s, 0.f);
}

// Element format of the velocity planes for population storage S: Bits is
// the stored word, VB its size in bytes, enc/dec convert from/to FP32.
template <class S> struct LagFmt {
    using Bits = unsigned short;
    static constexpr int VB = 2;
    __device__ static __forceinline__ float dec(Bits b) {
        return f16_scaled(__builtin_bit_cast(__half, b), 1.f / LAG_SCALE);
    }
    __device__ static __forceinline__ Bits enc(float x) {
        return __builtin_bit_cast(unsigned short, __float2half_rn(x * LAG_SCALE));
    }
};
template <> struct LagFmt<float> {
    using Bits = float;
    static constexpr int VB = 4;
    __device__ static __forceinline__ float dec(Bits b) { return b; }
    __device__ static __forceinline__ Bits enc(float x) { return x; }
};
// Bytes per node of one block, by velocity element size.
__host__ __device__ constexpr size_t lag_node_bytes(int vb) { return 3 * (size_t)vb + 4; }

// Field v at element offset off of a block with the given plane size.
template <class S, class I>
__device__ __forceinline__ float lag_ld(const char *M, int v, long long plane, I off) {
    using F = LagFmt<S>;
    if (v == 3) return reinterpret_cast<const float *>(M + 3 * plane * F::VB)[off];
    return F::dec(reinterpret_cast<const typename F::Bits *>(M + v * plane * F::VB)[off]);
}
template <class S, class I>
__device__ __forceinline__ void lag_st(char *M, int v, long long plane, I off, float x) {
    using F = LagFmt<S>;
    if (v == 3) reinterpret_cast<float *>(M + 3 * plane * F::VB)[off] = x;
    else reinterpret_cast<typename F::Bits *>(M + v * plane * F::VB)[off] = F::enc(x);
}
// The value lag_ld returns after lag_st stored x in field v.
template <class S>
__device__ __forceinline__ float lag_round(int v, float x) {
    if (v == 3) return x;
    return LagFmt<S>::dec(LagFmt<S>::enc(x));
}

// Everything a step kernel needs, passed by value.
struct KParams {
    int Nr, Nz, pitch;     // fluid nodes along r, z; row pitch (elements)
    // Global index of row 0 (a slab of a taller lattice): the stochastic
    // rounding of 16-bit stores keys on global rows.  It sits in the
    // alignment gap before `plane`: a larger parameter block made the step
    // kernels spill scalar registers (about 6400 v_readlane in the FP32
    // two-step kernel against 700).
    int row0;
    long long plane;       // elements per population / field plane
    float r0;              // radius of node row j is r0 + j + 1/2
    float nu, alpha;
    float g_axial, gbeta, T0, Tref;
    float om3, om45, om6, om7, om8;   // D2Q9 rates (omega_4 = omega_5 from nu)
    float og12, og3, og4;             // D2Q5 rates for psi
    float oh12, oh3, oh4;             // D2Q5 rates for T
    unsigned long long kinds;         // boundary kind of (face, field) in bits
                                      // 4 (3 face + field) .. +3
    float val[4][3];                  // imposed u_theta / T, or Omega
    // Axial faces in two parts: links that cross face Z_LO + f at twice
    // the radial column c2 >= 2 split[f] - 1 take the outer rule (kinds in
    // okinds, bits 4 (3 f + field) .. +3; value oval + oslope * r); split 0
    // leaves the face whole.
    int split[2];
    unsigned okinds;
    float oval[2][3], oslope[2][3];
    // HALO z faces (index 0: Z_LO, 1: Z_HI): the neighbouring row of the
    // adjacent slab, populations as 19 planes of `pitch` elements of the
    // storage type, then its lagged fields as a block of `pitch`-element
    // planes (lag_ld layout)
    const void *halo_pop[2];
    const char *halo_lag[2];
};

// Plane addresses of one step launch, for the tile workgroups of the step
// kernel: population p (f 0..8, g 9..13, h 14..18) of node n is read at
// rd[p] + n * sizeof(S) and written at wr[p] + n * sizeof(S), the streaming
// shift and slot exchange of the launch's phase being folded into the
// addresses on the host; lagged field v of node n is read at lrd[v] and
// written at lwr[v] + n * (element size), and uy_up / uy_dn address the
// u_y plane one row above / below.  The per-node offset is a 32-bit byte
// offset added to a uniform base, which gfx950 takes directly (an SGPR
// base plus a VGPR offset) instead of a 64-bit address per access; planes
// therefore hold at most 2^30 nodes.
struct Planes {
    const char *rd[NPOP];
    char *wr[NPOP];
    const char *lrd[NLAG];
    char *lwr[NLAG];
    const char *uy_up, *uy_dn;
};

__host__ __device__ __forceinline__ int kind_of(const KParams &P, int face, int fld) {
    return (int)((P.kinds >> (4 * (3 * face + fld))) & 15ull);
}

// Face value of distribution FLD without a dynamically indexed parameter
// array (which would force the parameters into scratch memory).
template <int FLD>
__device__ __forceinline__ float val_of(const KParams &P, int face) {
    return face == 0 ? P.val[0][FLD] : face == 1 ? P.val[1][FLD] : face == 2 ? P.val[2][FLD]
                                                                             : P.val[3][FLD];
}

// Whether a link that crosses `face` at twice the radial column c2 (2 j for
// a link along x into column j, 2 j - e_y for a diagonal one) meets the
// outer part of a split axial face.
__device__ __forceinline__ bool outer_part(const KParams &P, int face, int c2) {
    if (face < Z_LO) return false;
    const int s = face == Z_LO ? P.split[0] : P.split[1];
    return s > 0 && c2 >= 2 * s - 1;
}

// Kind of the rule of distribution fld where a link crosses `face` at c2.
__device__ __forceinline__ int kind_at(const KParams &P, int face, int fld, int c2) {
    return outer_part(P, face, c2) ? (int)((P.okinds >> (4 * (3 * (face - Z_LO) + fld))) & 15u)
                                   : kind_of(P, face, fld);
}

// Value of the rule of distribution FLD where a link crosses `face` at c2,
// at radius ym (a sloped value on an outer part).
template <int FLD>
__device__ __forceinline__ float val_at(const KParams &P, int face, int c2, float ym) {
    if (!outer_part(P, face, c2)) return val_of<FLD>(P, face);
    return face == Z_LO ? P.oval[0][FLD] + P.oslope[0][FLD] * ym
                        : P.oval[1][FLD] + P.oslope[1][FLD] * ym;
}

// Storage conversions: FP32 arithmetic; FP32, binary16 or bfloat16 storage.
// The 16-bit stores round stochastically, so that increments smaller than
// half a 16-bit ulp survive in expectation instead of being rounded away
// every step (see the 16-bit specialisations below).  `rnd` is the store's
// random word (slot_word for the stores of a node update, sr_single for a
// lone value); FP32 ignores it.
template <class S> struct Conv;
// Conv<S>::bits(v, rnd, r) gives the bit pattern st stores for v; the
// 16-bit conversions write it into the low half of the register r and leave
// its high half as it was, so a sequence of stores can reuse one register
// instead of clearing a fresh one for each.
template <> struct Conv<float> {
    using Reg = int;
    __device__ static __forceinline__ float ld(const float *p) { return *p; }
    __device__ static __forceinline__ void st(float *p, float v, unsigned) { *p = v; }
    __device__ static __forceinline__ float bits(float v, unsigned, Reg &) { return v; }
};

// 16-bit stores round stochastically with the gfx950 conversions
// v_cvt_sr_f16_f32 / v_cvt_sr_bf16_f32: the result rounds away from zero
// with probability equal to the discarded fraction, the threshold coming
// from the top bits of the random operand.  The operand is derived from a
// multiplicative hash of the stored values' bits and the node's position,
// whose top bits are the well mixed ones: rounding is deterministic (a
// checkpoint replays bit for bit) and fresh whenever a value changes.  NaN
// stays NaN; values beyond the format's range become infinite.
typedef _Float16 half2_t __attribute__((ext_vector_type(2)));
typedef short short2_t __attribute__((ext_vector_type(2)));
// Random word of a lone stored value with key `key`.
__device__ __forceinline__ unsigned sr_single(float x, unsigned key) {
    return (__float_as_uint(x) ^ key) * 0x9E3779B1U;
}

// binary16 holds the shifted populations scaled by 2^8 (exact), which keeps
// values down to ~2e-7 out of the subnormal range; 2^8 * 64 still sits far
// below the binary16 maximum for any population a stable run produces.
constexpr float F16_SCALE = 256.f;
template <> struct Conv<__half> {
    using Reg = half2_t;
    __device__ static __forceinline__ float ld(const __half *p) {
        return f16_scaled(*p, 1.f / F16_SCALE);
    }
    __device__ static __forceinline__ unsigned short bits(float v, unsigned rnd, Reg &r) {
        r = __builtin_amdgcn_cvt_sr_f16_f32(r, v * F16_SCALE, rnd, false);
        return __builtin_bit_cast(unsigned short, r[0]);
    }
    __device__ static __forceinline__ void st(__half *p, float v, unsigned rnd) {
        Reg r{0, 0};
        *p = __builtin_bit_cast(__half, bits(v, rnd, r));
    }
};
template <> struct Conv<__hip_bfloat16> {
    using Reg = short2_t;
    __device__ static __forceinline__ float ld(const __hip_bfloat16 *p) {
        return __bfloat162float(*p);
    }
    __device__ static __forceinline__ unsigned short bits(float v, unsigned rnd, Reg &r) {
        r = __builtin_amdgcn_cvt_sr_bf16_f32(r, v, rnd, false);
        return __builtin_bit_cast(unsigned short, r[0]);
    }
    __device__ static __forceinline__ void st(__hip_bfloat16 *p, float v, unsigned rnd) {
        Reg r{0, 0};
        *p = __builtin_bit_cast(__hip_bfloat16, bits(v, rnd, r));
    }
};

}  // namespace axlb
