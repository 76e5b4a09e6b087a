// Host launchers of the step, field, initialisation and reduction kernels.
// Internal to the HIP library.
#pragma once

#include <hip/hip_runtime.h>

#include <type_traits>

#include "axlb_device.h"

namespace axlb {

enum { STORE_F32 = 0, STORE_F16 = 1, STORE_BF16 = 2 };
template <class S> constexpr int store_of() {
    return std::is_same<S, float>::value ? STORE_F32
                                         : (std::is_same<S, __half>::value ? STORE_F16 : STORE_BF16);
}
// Velocity element size of the lagged fields for a storage code.
inline int lag_vb(int storage) { return storage == STORE_F32 ? 4 : 2; }

// Tile shapes of the step kernel: tile_shape(t) gives r x z nodes per workgroup.
#define AXLB_TILES(X) X(0, 64, 4) X(1, 64, 2) X(2, 64, 8) X(3, 128, 2) X(4, 256, 1) \
    X(5, 64, 1) X(6, 128, 4) X(7, 32, 8)
constexpr int NTILES = 8;
int tile_count();
void tile_shape(int tile, int *bx, int *by);

// mode: 0 = AB pull (src -> dst), 1 = AA odd phase, 2 = AA even phase (src == dst).
hipError_t launch_step(const KParams &P, int storage, int tile, int mode, void *src, void *dst,
                       const char *Mprev, char *Mnext, hipStream_t st);
// The plane addresses (Planes) of one step of the given mode: populations
// read from src and written to dst (src == dst in the AA phases), lagged
// fields read from Mprev and written to Mnext.
Planes step_planes(const KParams &P, int storage, int mode, const void *src, void *dst,
                   const char *Mprev, char *Mnext);
hipError_t launch_fields(const KParams &P, int storage, int mode, const void *src,
                         const char *Mprev, double *out, hipStream_t st);
// Current-step derivatives (two buffers, pull): one step src -> dst, or the
// reported fields of the state in src.
hipError_t launch_step_current(const KParams &P, int storage, int tile, const void *src,
                               void *dst, hipStream_t st);
hipError_t launch_fields_current(const KParams &P, int storage, const void *src, double *out,
                                 hipStream_t st);
// Two steps in one launch (two buffers, lagged derivatives): src/Mprev hold
// the state before step t, dst/Mnext receive it after step t + 1.
hipError_t launch_step_two(const KParams &P, int storage, const void *src, void *dst,
                           const char *Mprev, char *Mnext, hipStream_t st);
// A member of a batch of two-buffer lattices, for the two-step launch:
// buffer pair c (0 or 1) is read when the member's current pair is c.
struct TwoDesc {
    KParams P;
    const void *src[2];    // population buffer read from pair c
    const char *lag[2];    // lagged fields read from pair c
    Planes pl[2];          // plane addresses of a two-step launch from pair c
    int cur0;              // the member's pair at batch creation
    int gx;                // tiles along r
};
// Interior tile of the batched two-step kernel (nodes along r, along z).
void two_batch_tile_shape(int *tw, int *th);
// Work-list entries (member, tile index within the member).
hipError_t launch_step_two_batch(int storage, const TwoDesc *D, const int2 *tiles, int t0,
                                 int ntiles, int phase, hipStream_t st);
// enc: offset-encode bfloat16 populations with the lagged fields (every
// form but the current-step derivatives).
hipError_t launch_init(const KParams &P, int storage, bool aa, bool enc, void *pop,
                       const double *in, char *M, hipStream_t st);
hipError_t launch_residual(const double *fld, const double *snap, long long N, double *part,
                           int nblocks, double *out9, hipStream_t st);
hipError_t launch_nusselt(const double *T, int Nr, int Nz, int cylinder, double r0, double Ta,
                          double Tb, double *out2, hipStream_t st);
hipError_t launch_stream(const double *uz, int Nr, int Nz, double r0, double *psi,
                         double *row_range, hipStream_t st);

}  // namespace axlb
