// Host-side lattice object of the HIP library.  Internal.
#pragma once

#include <hip/hip_runtime.h>

#include <map>
#include <string>
#include <utility>

#include "../../include/axlb.h"
#include "axlb_device.h"

namespace axlb {

constexpr long BUNDLE = 100;      // steps per captured HIP graph
constexpr int RED_BLOCKS = 256;   // partial sums of the FP64 reductions

struct Layout {
    int pitch;                 // row pitch in elements (multiple of 64)
    long long plane;           // elements per plane
    size_t pop_bytes, lag_bytes, fld_bytes, snap_bytes, red_bytes;
    size_t halo_pop_bytes, halo_lag_bytes;  // one z face's halo row: populations, lagged fields
    size_t total;
};

size_t storage_size(int storage);
Layout layout_for(int Nr, int Nz, int storage, int layout);

}  // namespace axlb

struct axlb_lattice {
    int Nr = 0, Nz = 0, cylinder = 0;
    double r_inner = 0, nu = 0, alpha = 0, Ra = 0, Omega = 0, gbeta = 0, g_axial = 0, T0 = 0.5;
    double T_ref = 0.5;
    axlb_relax relax{};
    int storage = 0, layout = 0, deriv = 0;
    int row0 = 0;  // global index of row 0 (slabs)
    int cur = 0;  // two-buffer layouts: the population and lagged-field pair the next step reads
    int kind[4][3]{};
    double val[4][3]{};
    // outer parts of split axial faces (index 0: Z_LO, 1: Z_HI): from radial
    // node split[f] on (0: the face is whole), rule okind / oval + oslope r
    int split[2]{};
    int okind[2][3]{};
    double oval[2][3]{}, oslope[2][3]{};
    double *psi = nullptr;  // stream function and row maxima (device, on demand)
    int device = 0;
    hipStream_t stream = nullptr;
    bool own_stream = false, own_mem = false;
    axlb::Layout lay{};
    char *base = nullptr;
    void *pop[2] = {nullptr, nullptr};
    char *lag[2] = {nullptr, nullptr};  // lagged-field blocks (byte addressed)
    double *fld = nullptr, *snap = nullptr, *red = nullptr;
    char *halo[2] = {nullptr, nullptr};  // halo rows of the z faces (HALO kind)
    // captured step sequences: (steps in the graph, graph key) -> executable
    std::map<std::pair<long, int>, hipGraphExec_t> graphs;
    bool use_graphs = true;
    int tile = 0;  // step-kernel tile shape (see tile_shape)
    bool started = false, has_snap = false;
    bool batched = false;  // member of an axlb_batch: steps through the batch
    long steps = 0, snap_step = 0;
    axlb::KParams P{};
    std::string err;
};

namespace axlb {
KParams make_params(const axlb_lattice *L);
// Checks and locks the boundary rules (as the first step does).
int lattice_start(axlb_lattice *L);
// One step as a plain kernel launch on the lattice's stream.
int lattice_step_once(axlb_lattice *L);
}
