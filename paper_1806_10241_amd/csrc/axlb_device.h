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
enum { NOSLIP = 0, PERIODIC = 1, MIRROR = 2, DIRICHLET = 3, OMEGA_R = 4, ADIABATIC = 5 };

// Plane numbering of the population buffer: f_0..f_8, g_0..g_4, h_0..h_4.
constexpr int NPOP = 19;
constexpr int GOFF = 9;
constexpr int HOFF = 14;
// Lagged derivative fields: u_x, u_y, u_theta, T - T_ref.
constexpr int NLAG = 4;

// Everything a step kernel needs, passed by value.
struct KParams {
    int Nr, Nz, pitch;     // fluid nodes along r, z; row pitch (elements)
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

// Storage conversions: FP32 arithmetic, FP32 / binary16 / bfloat16 storage,
// round to nearest even on the way out.
template <class S> struct Conv;
template <> struct Conv<float> {
    __device__ static __forceinline__ float ld(const float *p) { return *p; }
    __device__ static __forceinline__ void st(float *p, float v) { *p = v; }
};
template <> struct Conv<__half> {
    __device__ static __forceinline__ float ld(const __half *p) { return __half2float(*p); }
    __device__ static __forceinline__ void st(__half *p, float v) { *p = __float2half_rn(v); }
};
template <> struct Conv<__hip_bfloat16> {
    __device__ static __forceinline__ float ld(const __hip_bfloat16 *p) { return __bfloat162float(*p); }
    __device__ static __forceinline__ void st(__hip_bfloat16 *p, float v) { *p = __float2bfloat16(v); }
};

}  // namespace axlb
