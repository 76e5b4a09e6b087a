// C-ABI of the axisymmetric cascaded LB step (include/axlb.h): parameter
// validation, device memory, step scheduling with HIP graph bundles,
// reductions and checkpoints.  No exception crosses the interface.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "../../include/axlb.h"
#include "axlb_internal.h"
#include "axlb_launch.h"

using namespace axlb;

static thread_local std::string g_create_error;

namespace axlb {

size_t storage_size(int storage) { return storage == AXLB_F32 ? 4 : 2; }

Layout layout_for(int Nr, int Nz, int storage, int layout) {
    Layout L;
    L.pitch = ((Nr + 63) / 64) * 64;
    L.plane = (long long)Nz * L.pitch;
    const size_t a = 256;
    auto up = [&](size_t b) { return (b + a - 1) / a * a; };
    L.pop_bytes = up((size_t)NPOP * L.plane * storage_size(storage));
    const int vb = lag_vb(storage);
    L.lag_bytes = up(lag_node_bytes(vb) * L.plane);
    const size_t N = (size_t)Nr * Nz;
    L.fld_bytes = up(5 * N * sizeof(double));
    L.snap_bytes = up(4 * N * sizeof(double));
    L.red_bytes = up((RED_BLOCKS * 9 + 16) * sizeof(double));
    L.halo_pop_bytes = up((size_t)NPOP * L.pitch * storage_size(storage));
    L.halo_lag_bytes = up(lag_node_bytes(vb) * L.pitch);
    L.total = (layout == AXLB_LAYOUT_AA ? 1 : 2) * L.pop_bytes + 2 * L.lag_bytes + L.fld_bytes +
              L.snap_bytes + L.red_bytes + 2 * (L.halo_pop_bytes + L.halo_lag_bytes);
    return L;
}

}  // namespace axlb

#define HIP_TRY(lat, expr)                                                        \
    do {                                                                          \
        hipError_t e_ = (expr);                                                   \
        if (e_ != hipSuccess) return fail(lat, AXLB_EDEVICE, std::string(#expr) + \
                                                                 ": " + hipGetErrorString(e_)); \
    } while (0)

static int fail(axlb_lattice *lat, int code, const std::string &msg) {
    if (lat) lat->err = msg;
    else g_create_error = msg;
    return code;
}

static bool is_wall(int k) {
    return k == AXLB_NOSLIP || k == AXLB_DIRICHLET || k == AXLB_OMEGA_R || k == AXLB_ADIABATIC ||
           k == AXLB_VELOCITY;
}

static bool rate_ok(double w) { return std::isfinite(w) && w > 0.0 && w < 2.0; }

// Device parameters of a lattice.
KParams axlb::make_params(const axlb_lattice *L) {
    KParams P;
    std::memset(&P, 0, sizeof(P));
    P.Nr = L->Nr;
    P.Nz = L->Nz;
    P.pitch = L->lay.pitch;
    P.plane = L->lay.plane;
    P.r0 = (float)(L->cylinder ? 0.0 : L->r_inner);
    P.nu = (float)L->nu;
    P.alpha = (float)L->alpha;
    P.g_axial = (float)L->g_axial;
    P.gbeta = (float)L->gbeta;
    P.T0 = (float)L->T0;
    P.Tref = (float)L->T_ref;
    // nu = c_s^2 (1/omega - 1/2), c_s^2 = 1/3 (text after eq. 17, 34, 49)
    P.om3 = (float)L->relax.omega3;
    P.om45 = (float)(1.0 / (3.0 * L->nu + 0.5));
    P.om6 = (float)L->relax.omega6;
    P.om7 = (float)L->relax.omega7;
    P.om8 = (float)L->relax.omega8;
    P.og12 = (float)(1.0 / (3.0 * L->nu + 0.5));
    P.og3 = (float)L->relax.omega_psi3;
    P.og4 = (float)L->relax.omega_psi4;
    P.oh12 = (float)(1.0 / (3.0 * L->alpha + 0.5));
    P.oh3 = (float)L->relax.omega_phi3;
    P.oh4 = (float)L->relax.omega_phi4;
    P.kinds = 0;
    for (int f = 0; f < 4; ++f)
        for (int d = 0; d < 3; ++d) {
            P.kinds |= (unsigned long long)(L->kind[f][d] & 15) << (4 * (3 * f + d));
            double v = L->val[f][d];
            if (L->kind[f][d] == AXLB_OMEGA_R && std::isnan(v)) v = L->Omega;
            P.val[f][d] = (float)v;
        }
    for (int f = 0; f < 2; ++f) {
        P.halo_pop[f] = L->halo[f];
        P.halo_lag[f] = L->halo[f] + L->lay.halo_pop_bytes;
    }
    P.row0 = L->row0;
    P.okinds = 0;
    for (int f = 0; f < 2; ++f) {
        P.split[f] = L->split[f];
        for (int d = 0; d < 3; ++d) {
            P.okinds |= (unsigned)(L->okind[f][d] & 15) << (4 * (3 * f + d));
            P.oval[f][d] = (float)L->oval[f][d];
            P.oslope[f][d] = (float)L->oslope[f][d];
        }
    }
    return P;
}

// Boundary settings that the step kernels can execute.
static int check_bcs(axlb_lattice *L) {
    for (int d = 0; d < 3; ++d) {
        const bool plo = L->kind[AXLB_Z_LO][d] == AXLB_PERIODIC;
        const bool phi = L->kind[AXLB_Z_HI][d] == AXLB_PERIODIC;
        if (plo != phi) return fail(L, AXLB_EINVAL, "periodic z must be set on both z faces");
        const bool wall = is_wall(L->kind[AXLB_Z_LO][d]) || is_wall(L->kind[AXLB_Z_HI][d]);
        if (wall && L->Nz < 2) return fail(L, AXLB_EINVAL, "Nz >= 2 needed with walls along z");
    }
    bool halo = false;
    for (int f = 0; f < 4; ++f) {
        const bool w = is_wall(L->kind[f][0]) || L->kind[f][0] == AXLB_SLIP;
        const bool p = L->kind[f][0] == AXLB_PERIODIC;
        const bool h = L->kind[f][0] == AXLB_HALO;
        halo = halo || h;
        for (int d = 1; d < 3; ++d) {
            if (is_wall(L->kind[f][d]) != w || (L->kind[f][d] == AXLB_PERIODIC) != p ||
                (L->kind[f][d] == AXLB_HALO) != h)
                return fail(L, AXLB_EINVAL,
                            "a face must be a wall, periodic, a halo or the axis for all three fields");
        }
    }
    for (int f = 0; f < 4; ++f)
        if (L->kind[f][0] == AXLB_VELOCITY &&
            (L->kind[f][1] == AXLB_ADIABATIC || L->kind[f][2] != AXLB_DIRICHLET))
            return fail(L, AXLB_EINVAL,
                        "a VELOCITY face needs imposed u_theta (g) and imposed T (h)");
    // a free surface carries wall rules for g and h
    for (int f = AXLB_Z_LO; f <= AXLB_Z_HI; ++f)
        if (L->kind[f][0] == AXLB_SLIP && (!is_wall(L->kind[f][1]) || !is_wall(L->kind[f][2])))
            return fail(L, AXLB_EINVAL, "a SLIP face needs wall rules for g and h");
    // split axial faces: both parts solid or free surface, no fluid crossing
    for (int f = 0; f < 2; ++f) {
        if (L->split[f] == 0) continue;
        if (L->split[f] >= L->Nr)
            return fail(L, AXLB_EINVAL, "the outer part of an axial face starts beyond the lattice");
        const int face = AXLB_Z_LO + f;
        for (int d = 0; d < 3; ++d) {
            const int a = L->kind[face][d], b = L->okind[f][d];
            const bool fa = d == 0 ? (a == AXLB_NOSLIP || a == AXLB_SLIP) : is_wall(a);
            const bool fb = d == 0 ? (b == AXLB_NOSLIP || b == AXLB_SLIP) : is_wall(b);
            if (!fa || !fb)
                return fail(L, AXLB_EINVAL,
                            "a split axial face is NOSLIP or SLIP for f and a wall for g and h "
                            "in both parts");
        }
    }
    if (halo && (L->layout != AXLB_LAYOUT_AB || L->deriv != AXLB_DERIV_LAGGED))
        return fail(L, AXLB_EINVAL, "HALO faces need the two-buffer, one-step layout");
    return AXLB_OK;
}

static bool two_buffers(const axlb_lattice *L) { return L->layout != AXLB_LAYOUT_AA; }

// Launches step t (counted from the lattice's creation), or steps t and
// t + 1 when `two` (the two-step layout only).  The AA phase follows the
// parity of t; the two-buffer layouts read buffer `cur` (populations and
// lagged fields) and write the other one.
static int launch_steps(axlb_lattice *L, long t, int cur, bool two) {
    const KParams &P = L->P;
    hipError_t e;
    if (L->layout == AXLB_LAYOUT_AA) {
        const int par = (int)(t & 1);
        e = launch_step(P, L->storage, L->tile, par == 0 ? 1 : 2, L->pop[0], L->pop[0], L->lag[par],
                        L->lag[par ^ 1], L->stream);
    } else if (L->deriv == AXLB_DERIV_CURRENT) {
        e = launch_step_current(P, L->storage, L->tile, L->pop[cur], L->pop[cur ^ 1], L->stream);
    } else if (two) {
        e = launch_step_two(P, L->storage, L->pop[cur], L->pop[cur ^ 1], L->lag[cur],
                            L->lag[cur ^ 1], L->stream);
    } else {
        e = launch_step(P, L->storage, L->tile, 0, L->pop[cur], L->pop[cur ^ 1], L->lag[cur],
                        L->lag[cur ^ 1], L->stream);
    }
    if (e != hipSuccess) return fail(L, AXLB_EDEVICE, std::string("step launch: ") + hipGetErrorString(e));
    return AXLB_OK;
}

// One step as a plain launch, advancing the step count and the buffer.
static int launch_one(axlb_lattice *L) {
    const int rc = launch_steps(L, L->steps, L->cur, false);
    if (rc) return rc;
    L->steps += 1;
    if (two_buffers(L)) L->cur ^= 1;
    return AXLB_OK;
}

// Key of the graph that runs the next steps: the AA phase, or the buffer
// the two-buffer layouts read.  A BUNDLE of steps flips either an even
// number of times (BUNDLE is a multiple of 4), so every bundle of a call
// shares the key of the call's first step.
static int graph_key(const axlb_lattice *L) {
    return two_buffers(L) ? L->cur : (int)(L->steps & 1);
}

// Graphs of other lengths than BUNDLE (the tail of an axlb_step call) kept
// per lattice; beyond this many the cached tails are dropped first.
constexpr size_t MAX_TAIL_GRAPHS = 8;

static void drop_graphs(axlb_lattice *L, bool tails_only = false) {
    for (auto it = L->graphs.begin(); it != L->graphs.end();) {
        if (tails_only && it->first.first == BUNDLE) {
            ++it;
            continue;
        }
        (void)hipGraphExecDestroy(it->second);
        it = L->graphs.erase(it);
    }
}

// HIP graph of `len` consecutive steps for graph key k (see graph_key):
// the launches a plain run would make, two steps per launch in the
// two-step layout (an odd length ends with one single step).
static int ensure_graph(axlb_lattice *L, long len, int k) {
    const auto key = std::make_pair(len, k);
    if (L->graphs.count(key)) return AXLB_OK;
    if (len != BUNDLE && L->graphs.size() >= MAX_TAIL_GRAPHS) drop_graphs(L, true);
    HIP_TRY(L, hipStreamBeginCapture(L->stream, hipStreamCaptureModeThreadLocal));
    int rc = AXLB_OK;
    const bool two = L->layout == AXLB_LAYOUT_AB2;
    int cur = k;
    for (long s = 0; s < len && rc == AXLB_OK;) {
        const bool pair = two && s + 1 < len;
        rc = launch_steps(L, k + s, cur, pair);  // for AA, k + s has the parity of the step
        cur ^= 1;
        s += pair ? 2 : 1;
    }
    hipGraph_t g = nullptr;
    hipError_t e = hipStreamEndCapture(L->stream, &g);
    if (rc != AXLB_OK) {
        if (g) (void)hipGraphDestroy(g);
        return rc;
    }
    if (e != hipSuccess) return fail(L, AXLB_EDEVICE, std::string("graph capture: ") + hipGetErrorString(e));
    hipGraphExec_t x = nullptr;
    e = hipGraphInstantiate(&x, g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    if (e != hipSuccess)
        return fail(L, AXLB_EDEVICE, std::string("graph instantiate: ") + hipGetErrorString(e));
    // upload it now, so that its first replay costs no more than the others
    e = hipGraphUpload(x, L->stream);
    if (e != hipSuccess) {
        (void)hipGraphExecDestroy(x);
        return fail(L, AXLB_EDEVICE, std::string("graph upload: ") + hipGetErrorString(e));
    }
    L->graphs[key] = x;
    return AXLB_OK;
}

static int set_device(axlb_lattice *L) {
    HIP_TRY(L, hipSetDevice(L->device));
    return AXLB_OK;
}

// Fields of the current state into L->fld (device, FP64 planes rho, u_r,
// u_z, u_theta, T).
static int compute_fields(axlb_lattice *L) {
    const int par = (int)(L->steps & 1), cur = L->cur;
    hipError_t e;
    if (L->deriv == AXLB_DERIV_CURRENT)
        e = launch_fields_current(L->P, L->storage, L->pop[cur], L->fld, L->stream);
    else if (L->layout == AXLB_LAYOUT_AA)
        e = launch_fields(L->P, L->storage, par == 0 ? 1 : 2, L->pop[0], L->lag[par], L->fld,
                          L->stream);
    else
        e = launch_fields(L->P, L->storage, 0, L->pop[cur], L->lag[cur], L->fld, L->stream);
    if (e != hipSuccess) return fail(L, AXLB_EDEVICE, std::string("fields launch: ") + hipGetErrorString(e));
    return AXLB_OK;
}

int axlb::lattice_start(axlb_lattice *L) {
    int rc = set_device(L);
    if (rc) return rc;
    if (!L->started) {
        rc = check_bcs(L);
        if (rc) return rc;
        L->P = make_params(L);
        L->started = true;
    }
    return AXLB_OK;
}

int axlb::lattice_step_once(axlb_lattice *L) {
    const int rc = lattice_start(L);
    if (rc) return rc;
    return launch_one(L);
}

extern "C" {

int axlb_state_bytes(int Nr, int Nz, int storage, int layout, size_t *bytes) {
    if (!bytes || Nr < 2 || Nz < 1 || storage < 0 || storage > 2 || layout < 0 || layout > 2)
        return fail(nullptr, AXLB_EINVAL, "axlb_state_bytes: bad arguments");
    *bytes = layout_for(Nr, Nz, storage, layout).total;
    return AXLB_OK;
}

int axlb_lattice_create(int Nr, int Nz, const axlb_geometry *geo, double nu, double alpha,
                        double Pr, double Ra, double Omega, const axlb_relax *w,
                        const axlb_options *opt, axlb_lattice **out) {
    if (!out) return fail(nullptr, AXLB_EINVAL, "out is NULL");
    *out = nullptr;
    if (!geo) return fail(nullptr, AXLB_EINVAL, "geometry is NULL");
    // the step kernel addresses a plane with 32-bit byte offsets (4 bytes per node)
    if (Nr < 2 || Nz < 1 || (long long)Nz * (((long long)Nr + 63) / 64 * 64) > (1LL << 30))
        return fail(nullptr, AXLB_EINVAL,
                    "Nr >= 2, Nz >= 1 and Nz * (Nr rounded up to 64) <= 2^30 required");
    if (geo->kind != AXLB_ANNULUS && geo->kind != AXLB_CYLINDER)
        return fail(nullptr, AXLB_EINVAL, "unknown geometry kind");
    if (geo->kind == AXLB_ANNULUS && !(geo->r_inner > 0.0 && std::isfinite(geo->r_inner)))
        return fail(nullptr, AXLB_EINVAL, "annulus needs r_inner > 0");
    if (!(nu > 0.0 && std::isfinite(nu)) || !(alpha > 0.0 && std::isfinite(alpha)))
        return fail(nullptr, AXLB_EINVAL, "nu > 0 and alpha > 0 required (relaxation time > 1/2)");
    if (Pr != 0.0 && !(std::fabs(Pr - nu / alpha) <= 1e-9 * std::fabs(Pr)))
        return fail(nullptr, AXLB_EINVAL, "Pr differs from nu/alpha");
    if (!(Ra >= 0.0 && std::isfinite(Ra))) return fail(nullptr, AXLB_EINVAL, "Ra must be >= 0");
    axlb_relax R = {1.0, 1.0, 1.0, 1.0, 1.0, 1.0, 1.0, 1.0};
    if (w) R = *w;
    for (double x : {R.omega3, R.omega6, R.omega7, R.omega8, R.omega_psi3, R.omega_psi4,
                     R.omega_phi3, R.omega_phi4})
        if (!rate_ok(x)) return fail(nullptr, AXLB_EINVAL, "relaxation rates must lie in (0, 2)");
    axlb_options O;
    std::memset(&O, 0, sizeof(O));
    O.storage = AXLB_F32;
    O.layout = AXLB_LAYOUT_AA;
    O.T_ref = 0.5;
    O.device = -1;
    if (opt) O = *opt;
    if (O.storage < 0 || O.storage > 2) return fail(nullptr, AXLB_EINVAL, "unknown storage");
    if (O.layout < 0 || O.layout > 2) return fail(nullptr, AXLB_EINVAL, "unknown layout");
    if (O.deriv != AXLB_DERIV_LAGGED && O.deriv != AXLB_DERIV_CURRENT)
        return fail(nullptr, AXLB_EINVAL, "unknown derivative time level");
    if (O.deriv == AXLB_DERIV_CURRENT && O.layout != AXLB_LAYOUT_AB)
        return fail(nullptr, AXLB_EINVAL,
                    "current-step derivatives need the two-buffer, one-step layout");
    if (O.deriv == AXLB_DERIV_CURRENT && O.storage == AXLB_BF16)
        return fail(nullptr, AXLB_EINVAL,
                    "bfloat16 storage needs the lagged derivatives: its offset encoding takes "
                    "the lagged fields, and plain bfloat16 misses the 16-bit accuracy bar");
    if (!std::isfinite(O.T_ref)) return fail(nullptr, AXLB_EINVAL, "T_ref must be finite");
    if (O.row0 < 0 || (long long)O.row0 + Nz > INT32_MAX)
        return fail(nullptr, AXLB_EINVAL, "row0 must be >= 0 and row0 + Nz below 2^31");

    axlb_lattice *L = new (std::nothrow) axlb_lattice();
    if (!L) return fail(nullptr, AXLB_ENOMEM, "host allocation failed");
    L->Nr = Nr;
    L->Nz = Nz;
    L->cylinder = geo->kind == AXLB_CYLINDER;
    L->r_inner = L->cylinder ? 0.0 : geo->r_inner;
    L->nu = nu;
    L->alpha = alpha;
    L->Ra = Ra;
    L->Omega = Omega;
    L->gbeta = Ra * nu * alpha / ((double)Nr * Nr * Nr);
    L->T0 = 0.5;
    L->relax = R;
    L->storage = O.storage;
    L->layout = O.layout;
    L->deriv = O.deriv;
    L->row0 = O.row0;
    L->T_ref = O.T_ref;
    for (int f = 0; f < 4; ++f) {
        L->kind[f][0] = AXLB_NOSLIP;
        L->kind[f][1] = AXLB_NOSLIP;
        L->kind[f][2] = AXLB_ADIABATIC;
        for (int d = 0; d < 3; ++d) L->val[f][d] = 0.0;
    }
    if (L->cylinder)
        for (int d = 0; d < 3; ++d) L->kind[AXLB_R_IN][d] = AXLB_MIRROR;

    auto bad = [&](int code, const std::string &m) {
        g_create_error = m;
        axlb_destroy(L);
        return code;
    };
    int dev = O.device;
    if (dev < 0 && hipGetDevice(&dev) != hipSuccess) return bad(AXLB_EDEVICE, "hipGetDevice failed");
    L->device = dev;
    if (hipSetDevice(dev) != hipSuccess) return bad(AXLB_EDEVICE, "hipSetDevice failed");
    L->lay = layout_for(Nr, Nz, L->storage, L->layout);
    if (O.device_buf) {
        if (O.device_bytes < L->lay.total || ((uintptr_t)O.device_buf & 255))
            return bad(AXLB_EINVAL, "device_buf too small or not 256-byte aligned");
        L->base = (char *)O.device_buf;
        L->own_mem = false;
    } else {
        if (hipMalloc((void **)&L->base, L->lay.total) != hipSuccess) {
            L->base = nullptr;
            return bad(AXLB_ENOMEM, "hipMalloc of the lattice state failed");
        }
        L->own_mem = true;
    }
    char *p = L->base;
    L->pop[0] = p;
    p += L->lay.pop_bytes;
    if (two_buffers(L)) {
        L->pop[1] = p;
        p += L->lay.pop_bytes;
    } else {
        L->pop[1] = L->pop[0];
    }
    L->lag[0] = p;
    p += L->lay.lag_bytes;
    L->lag[1] = p;
    p += L->lay.lag_bytes;
    L->fld = (double *)p;
    p += L->lay.fld_bytes;
    L->snap = (double *)p;
    p += L->lay.snap_bytes;
    L->red = (double *)p;
    p += L->lay.red_bytes;
    for (int f = 0; f < 2; ++f) {
        L->halo[f] = p;
        p += L->lay.halo_pop_bytes + L->lay.halo_lag_bytes;
    }
    if (O.stream) {
        L->stream = (hipStream_t)O.stream;
        L->own_stream = false;
    } else {
        if (hipStreamCreateWithFlags(&L->stream, hipStreamNonBlocking) != hipSuccess)
            return bad(AXLB_EDEVICE, "hipStreamCreate failed");
        L->own_stream = true;
    }
    // zero everything once so that padding never holds garbage
    if (hipMemsetAsync(L->base, 0, L->lay.total, L->stream) != hipSuccess)
        return bad(AXLB_EDEVICE, "hipMemsetAsync failed");
    L->P = make_params(L);
    int rc = axlb_set_fields(L, nullptr, nullptr, nullptr, nullptr, nullptr);
    if (rc != AXLB_OK) return bad(rc, L->err);
    *out = L;
    return AXLB_OK;
}

int axlb_set_bc(axlb_lattice *L, int face, int field, int kind, double value) {
    if (!L) return fail(nullptr, AXLB_EINVAL, "lattice is NULL");
    if (L->started) return fail(L, AXLB_ESTATE, "boundary rules are fixed once stepping started");
    if (face < 0 || face > 3 || field < 0 || field > 2 || kind < 0 || kind > 8)
        return fail(L, AXLB_EINVAL, "face, field or kind out of range");
    if (kind == AXLB_SLIP && (field != AXLB_FLOW || face < AXLB_Z_LO))
        return fail(L, AXLB_EINVAL, "SLIP is a rule for f (FLOW) on z faces");
    if (L->cylinder && face == AXLB_R_IN && kind != AXLB_MIRROR)
        return fail(L, AXLB_EINVAL, "the inner face of a cylinder is the axis");
    if (kind == AXLB_MIRROR && !(L->cylinder && face == AXLB_R_IN))
        return fail(L, AXLB_EINVAL, "MIRROR is only the axis of a cylinder");
    if ((kind == AXLB_PERIODIC || kind == AXLB_HALO) && face != AXLB_Z_LO && face != AXLB_Z_HI)
        return fail(L, AXLB_EINVAL, "PERIODIC and HALO are only for z faces");
    if (field == AXLB_FLOW && (kind == AXLB_DIRICHLET || kind == AXLB_OMEGA_R || kind == AXLB_ADIABATIC))
        return fail(L, AXLB_EINVAL, "FLOW walls are NOSLIP or VELOCITY");
    if (field != AXLB_FLOW && kind == AXLB_VELOCITY)
        return fail(L, AXLB_EINVAL, "VELOCITY is a rule for f (FLOW) only");
    if (kind == AXLB_VELOCITY && !std::isfinite(value))
        return fail(L, AXLB_EINVAL, "VELOCITY value must be finite");
    if (field == AXLB_THERMAL && (kind == AXLB_NOSLIP || kind == AXLB_OMEGA_R))
        return fail(L, AXLB_EINVAL, "THERMAL walls are DIRICHLET or ADIABATIC");
    if (kind == AXLB_DIRICHLET && !std::isfinite(value))
        return fail(L, AXLB_EINVAL, "DIRICHLET value must be finite");
    if (kind == AXLB_OMEGA_R && std::isinf(value))
        return fail(L, AXLB_EINVAL, "OMEGA_R value must be finite or NaN");
    L->kind[face][field] = kind;
    L->val[face][field] = value;
    L->P = make_params(L);
    return AXLB_OK;
}

int axlb_set_bc_outer(axlb_lattice *L, int face, int from, int field, int kind, double value,
                      double slope) {
    if (!L) return fail(nullptr, AXLB_EINVAL, "lattice is NULL");
    if (L->started) return fail(L, AXLB_ESTATE, "boundary rules are fixed once stepping started");
    if (face != AXLB_Z_LO && face != AXLB_Z_HI)
        return fail(L, AXLB_EINVAL, "only z faces have an outer part");
    if (field < 0 || field > 2) return fail(L, AXLB_EINVAL, "field out of range");
    const int f = face - AXLB_Z_LO;
    if (from < 1 || from >= L->Nr)
        return fail(L, AXLB_EINVAL, "the outer part must start at radial node 1 .. Nr - 1");
    if (L->split[f] != 0 && L->split[f] != from)
        return fail(L, AXLB_EINVAL, "an axial face splits at one radial node for all fields");
    const bool ok = field == AXLB_FLOW ? (kind == AXLB_NOSLIP || kind == AXLB_SLIP)
                  : field == AXLB_SWIRL
                        ? (kind == AXLB_NOSLIP || kind == AXLB_DIRICHLET || kind == AXLB_OMEGA_R ||
                           kind == AXLB_ADIABATIC)
                        : (kind == AXLB_DIRICHLET || kind == AXLB_ADIABATIC);
    if (!ok) return fail(L, AXLB_EINVAL, "kind not allowed on the outer part for this field");
    if (!std::isfinite(value) || !std::isfinite(slope))
        return fail(L, AXLB_EINVAL, "value and slope must be finite");
    if (slope != 0.0 && kind != AXLB_DIRICHLET)
        return fail(L, AXLB_EINVAL, "a slope is only for DIRICHLET");
    // parts of a split face not yet given a rule are NOSLIP / NOSLIP /
    // ADIABATIC, as a wall is by default
    if (L->split[f] == 0) {
        L->okind[f][0] = AXLB_NOSLIP;
        L->okind[f][1] = AXLB_NOSLIP;
        L->okind[f][2] = AXLB_ADIABATIC;
        for (int d = 0; d < 3; ++d) L->oval[f][d] = L->oslope[f][d] = 0.0;
    }
    L->split[f] = from;
    L->okind[f][field] = kind;
    L->oval[f][field] = value;
    L->oslope[f][field] = slope;
    L->P = make_params(L);
    return AXLB_OK;
}

int axlb_set_body_force(axlb_lattice *L, double g_axial, double T0) {
    if (!L) return fail(nullptr, AXLB_EINVAL, "lattice is NULL");
    if (L->started) return fail(L, AXLB_ESTATE, "body force is fixed once stepping started");
    if (!std::isfinite(g_axial) || !std::isfinite(T0)) return fail(L, AXLB_EINVAL, "non-finite force");
    L->g_axial = g_axial;
    L->T0 = T0;
    L->P = make_params(L);
    return AXLB_OK;
}

int axlb_set_fields(axlb_lattice *L, const double *rho, const double *ur, const double *uz,
                    const double *uth, const double *T) {
    if (!L) return fail(nullptr, AXLB_EINVAL, "lattice is NULL");
    if (L->batched) return fail(L, AXLB_ESTATE, "the lattice is in a batch");
    int rc = set_device(L);
    if (rc) return rc;
    const size_t N = (size_t)L->Nr * L->Nz;
    std::vector<double> h(5 * N);
    for (size_t k = 0; k < N; ++k) {
        h[k] = rho ? rho[k] : 1.0;
        h[N + k] = ur ? ur[k] : 0.0;
        h[2 * N + k] = uz ? uz[k] : 0.0;
        h[3 * N + k] = uth ? uth[k] : 0.0;
        h[4 * N + k] = T ? T[k] : L->T_ref;
        for (int c = 0; c < 5; ++c)
            if (!std::isfinite(h[c * N + k])) return fail(L, AXLB_EINVAL, "non-finite initial field");
        if (!(h[k] > 0.0)) return fail(L, AXLB_EINVAL, "initial density must be positive");
    }
    HIP_TRY(L, hipMemcpyAsync(L->fld, h.data(), 5 * N * sizeof(double), hipMemcpyHostToDevice,
                              L->stream));
    hipError_t e = launch_init(L->P, L->storage, L->layout == AXLB_LAYOUT_AA,
                               L->deriv == AXLB_DERIV_LAGGED, L->pop[0], L->fld, L->lag[0],
                               L->stream);
    if (e != hipSuccess) return fail(L, AXLB_EDEVICE, std::string("init launch: ") + hipGetErrorString(e));
    HIP_TRY(L, hipStreamSynchronize(L->stream));
    L->steps = 0;
    L->cur = 0;
    L->has_snap = false;
    return AXLB_OK;
}

int axlb_step(axlb_lattice *L, long n) {
    if (!L) return fail(nullptr, AXLB_EINVAL, "lattice is NULL");
    if (n < 0) return fail(L, AXLB_EINVAL, "negative step count");
    if (L->batched) return fail(L, AXLB_ESTATE, "the lattice steps through its batch");
    if (n == 0) return AXLB_OK;
    int rc = lattice_start(L);
    if (rc) return rc;
    while (n > 0) {
        if (L->use_graphs && n >= 2) {
            // a bundle, or the whole tail of the call, as one graph replay
            const long len = n >= BUNDLE ? BUNDLE : n;
            const int k = graph_key(L);
            rc = ensure_graph(L, len, k);
            if (rc) return rc;
            HIP_TRY(L, hipGraphLaunch(L->graphs[std::make_pair(len, k)], L->stream));
            L->steps += len;
            if (two_buffers(L)) {
                // buffers swap once per launch
                const long launches = L->layout == AXLB_LAYOUT_AB2 ? (len + 1) / 2 : len;
                if (launches & 1) L->cur ^= 1;
            }
            n -= len;
        } else if (n >= 2 && L->layout == AXLB_LAYOUT_AB2) {
            rc = launch_steps(L, L->steps, L->cur, true);
            if (rc) return rc;
            L->steps += 2;
            L->cur ^= 1;
            n -= 2;
        } else {
            rc = launch_one(L);
            if (rc) return rc;
            n -= 1;
        }
    }
    return AXLB_OK;
}

int axlb_set_graphs(axlb_lattice *L, int enable) {
    if (!L) return fail(nullptr, AXLB_EINVAL, "lattice is NULL");
    L->use_graphs = enable != 0;
    return AXLB_OK;
}

int axlb_prepare_steps(axlb_lattice *L, long n) {
    if (!L) return fail(nullptr, AXLB_EINVAL, "lattice is NULL");
    if (n < 0) return fail(L, AXLB_EINVAL, "negative step count");
    if (L->batched) return fail(L, AXLB_ESTATE, "the lattice steps through its batch");
    int rc = lattice_start(L);
    if (rc || !L->use_graphs) return rc;
    // the graphs axlb_step(n) replays from the current state: its bundles
    // and its tail share the key of the first step
    const int k = graph_key(L);
    if (n >= BUNDLE) rc = ensure_graph(L, BUNDLE, k);
    if (rc == AXLB_OK && n % BUNDLE >= 2) rc = ensure_graph(L, n % BUNDLE, k);
    return rc;
}

long axlb_steps_done(const axlb_lattice *L) { return L ? L->steps : -1; }

int axlb_sync(axlb_lattice *L) {
    if (!L) return fail(nullptr, AXLB_EINVAL, "lattice is NULL");
    int rc = set_device(L);
    if (rc) return rc;
    HIP_TRY(L, hipStreamSynchronize(L->stream));
    return AXLB_OK;
}

int axlb_get_moments(axlb_lattice *L, double *rho, double *ur, double *uz, double *uth,
                     double *T) {
    if (!L) return fail(nullptr, AXLB_EINVAL, "lattice is NULL");
    int rc = set_device(L);
    if (rc) return rc;
    rc = compute_fields(L);
    if (rc) return rc;
    const size_t N = (size_t)L->Nr * L->Nz;
    double *dst[5] = {rho, ur, uz, uth, T};
    for (int c = 0; c < 5; ++c)
        if (dst[c])
            HIP_TRY(L, hipMemcpyAsync(dst[c], L->fld + c * N, N * sizeof(double),
                                      hipMemcpyDeviceToHost, L->stream));
    HIP_TRY(L, hipStreamSynchronize(L->stream));
    return AXLB_OK;
}

int axlb_nusselt(axlb_lattice *L, double *nu_a, double *nu_b, double *mean) {
    if (!L) return fail(nullptr, AXLB_EINVAL, "lattice is NULL");
    const int fa = L->cylinder ? AXLB_Z_LO : AXLB_R_IN, fb = L->cylinder ? AXLB_Z_HI : AXLB_R_OUT;
    if (L->kind[fa][2] != AXLB_DIRICHLET || L->kind[fb][2] != AXLB_DIRICHLET)
        return fail(L, AXLB_ESTATE, "Nusselt numbers need imposed T on both heat-transfer walls");
    if (L->cylinder && (L->split[0] || L->split[1]))
        return fail(L, AXLB_ESTATE, "Nusselt numbers need lids of one temperature each");
    const double Ta = L->val[fa][2], Tb = L->val[fb][2];
    const double dT = L->cylinder ? Tb - Ta : Ta - Tb;
    if (dT == 0.0) return fail(L, AXLB_ESTATE, "the two wall temperatures are equal");
    if ((L->cylinder && L->Nz < 2) || L->Nr < 2)
        return fail(L, AXLB_ESTATE, "too few nodes for the wall gradient");
    int rc = set_device(L);
    if (rc) return rc;
    rc = compute_fields(L);
    if (rc) return rc;
    const size_t N = (size_t)L->Nr * L->Nz;
    double *out = L->red + RED_BLOCKS * 9;
    hipError_t e = launch_nusselt(L->fld + 4 * N, L->Nr, L->Nz, L->cylinder, L->r_inner, Ta, Tb,
                                  out, L->stream);
    if (e != hipSuccess) return fail(L, AXLB_EDEVICE, std::string("nusselt launch: ") + hipGetErrorString(e));
    double s[2];
    HIP_TRY(L, hipMemcpyAsync(s, out, sizeof(s), hipMemcpyDeviceToHost, L->stream));
    HIP_TRY(L, hipStreamSynchronize(L->stream));
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

int axlb_stream_function(axlb_lattice *L, double *psi, double *psi_min, double *psi_max) {
    if (!L) return fail(nullptr, AXLB_EINVAL, "lattice is NULL");
    int rc = set_device(L);
    if (rc) return rc;
    const size_t N = (size_t)L->Nr * L->Nz;
    if (!L->psi) HIP_TRY(L, hipMalloc((void **)&L->psi, (N + 2 * (size_t)L->Nz) * sizeof(double)));
    rc = compute_fields(L);
    if (rc) return rc;
    const double r0 = L->cylinder ? 0.0 : L->r_inner;
    hipError_t e = launch_stream(L->fld + 2 * N, L->Nr, L->Nz, r0, L->psi, L->psi + N, L->stream);
    if (e != hipSuccess) return fail(L, AXLB_EDEVICE, std::string("stream function launch: ") + hipGetErrorString(e));
    std::vector<double> rows(2 * (size_t)L->Nz);
    HIP_TRY(L, hipMemcpyAsync(rows.data(), L->psi + N, rows.size() * sizeof(double),
                              hipMemcpyDeviceToHost, L->stream));
    if (psi)
        HIP_TRY(L, hipMemcpyAsync(psi, L->psi, N * sizeof(double), hipMemcpyDeviceToHost, L->stream));
    HIP_TRY(L, hipStreamSynchronize(L->stream));
    double lo = 0.0, hi = 0.0;
    for (int i = 0; i < L->Nz; ++i) {
        lo = std::fmin(lo, rows[2 * (size_t)i]);
        hi = std::fmax(hi, rows[2 * (size_t)i + 1]);
    }
    if (psi_min) *psi_min = lo;
    if (psi_max) *psi_max = hi;
    return AXLB_OK;
}

int axlb_residual(axlb_lattice *L, double *r) {
    if (!L || !r) return fail(L, AXLB_EINVAL, "NULL argument");
    int rc = set_device(L);
    if (rc) return rc;
    rc = compute_fields(L);
    if (rc) return rc;
    const size_t N = (size_t)L->Nr * L->Nz;
    double *out = L->red + RED_BLOCKS * 9;
    hipError_t e = launch_residual(L->fld, L->snap, (long long)N, L->red, RED_BLOCKS, out, L->stream);
    if (e != hipSuccess) return fail(L, AXLB_EDEVICE, std::string("residual launch: ") + hipGetErrorString(e));
    double s[9];
    HIP_TRY(L, hipMemcpyAsync(s, out, sizeof(s), hipMemcpyDeviceToHost, L->stream));
    HIP_TRY(L, hipMemcpyAsync(L->snap, L->fld + N, 4 * N * sizeof(double),
                              hipMemcpyDeviceToDevice, L->stream));
    HIP_TRY(L, hipStreamSynchronize(L->stream));
    const bool had = L->has_snap;
    const long K = L->steps - L->snap_step;
    L->has_snap = true;
    L->snap_step = L->steps;
    if (s[8] != 0.0) {
        *r = NAN;
        return fail(L, AXLB_EUNSTABLE, "non-finite value in the fields");
    }
    if (!had || K <= 0) {
        *r = INFINITY;
        return AXLB_OK;
    }
    // velocity components against the speed field (a component may be zero
    // up to round-off), T against itself
    double m = 0.0;
    const double speed2 = s[1] + s[3] + s[5];
    if (speed2 > 0.0)
        for (int c = 0; c < 3; ++c)
            m = std::fmax(m, std::sqrt(s[2 * c]) / ((double)K * std::sqrt(speed2)));
    if (s[7] > 0.0) m = std::fmax(m, std::sqrt(s[6]) / ((double)K * std::sqrt(s[7])));
    *r = m;
    return AXLB_OK;
}

// Checkpoint image: header, then the population buffer the next step reads,
// then the lagged fields it reads.
struct Header {
    uint64_t magic;
    int32_t Nr, Nz, storage, layout;
    int64_t steps;
    uint64_t pop_bytes, lag_bytes;
};
static const uint64_t MAGIC = 0x31424c584131ULL;  // "1AXLB1"
// An image of offset-encoded bfloat16 populations (every form with lagged
// derivatives) carries its own magic: such populations mean something only
// with the lagged fields, so a lattice with current-step derivatives (plain
// bfloat16) must not load them, nor the other way round.
static const uint64_t MAGIC_ENC = 0x32424c584131ULL;  // "1AXLB2"
static uint64_t image_magic(const axlb_lattice *L) {
    return L->storage == AXLB_BF16 && L->deriv == AXLB_DERIV_LAGGED ? MAGIC_ENC : MAGIC;
}

int axlb_state_size(const axlb_lattice *L, size_t *bytes) {
    if (!L || !bytes) return fail(nullptr, AXLB_EINVAL, "NULL argument");
    *bytes = sizeof(Header) + L->lay.pop_bytes + L->lay.lag_bytes;
    return AXLB_OK;
}

int axlb_save(axlb_lattice *L, void *host, size_t bytes) {
    if (!L || !host) return fail(L, AXLB_EINVAL, "NULL argument");
    size_t need;
    axlb_state_size(L, &need);
    if (bytes < need) return fail(L, AXLB_EINVAL, "buffer too small");
    int rc = set_device(L);
    if (rc) return rc;
    // the buffers the next step reads: AA's one population buffer and the
    // lagged block of the step parity; the two-buffer layouts' current pair
    const int k = two_buffers(L) ? L->cur : (int)(L->steps & 1);
    Header h = {image_magic(L), L->Nr, L->Nz, L->storage, L->layout, L->steps, L->lay.pop_bytes,
                L->lay.lag_bytes};
    char *p = (char *)host;
    std::memcpy(p, &h, sizeof(h));
    void *pop = two_buffers(L) ? L->pop[k] : L->pop[0];
    HIP_TRY(L, hipMemcpyAsync(p + sizeof(h), pop, L->lay.pop_bytes, hipMemcpyDeviceToHost, L->stream));
    HIP_TRY(L, hipMemcpyAsync(p + sizeof(h) + L->lay.pop_bytes, L->lag[k], L->lay.lag_bytes,
                              hipMemcpyDeviceToHost, L->stream));
    HIP_TRY(L, hipStreamSynchronize(L->stream));
    return AXLB_OK;
}

int axlb_load(axlb_lattice *L, const void *host, size_t bytes) {
    if (!L || !host) return fail(L, AXLB_EINVAL, "NULL argument");
    if (L->batched) return fail(L, AXLB_ESTATE, "the lattice is in a batch");
    size_t need;
    axlb_state_size(L, &need);
    Header h;
    if (bytes < need) return fail(L, AXLB_EINVAL, "image too small");
    std::memcpy(&h, host, sizeof(h));
    if (h.magic != image_magic(L) || h.Nr != L->Nr || h.Nz != L->Nz || h.storage != L->storage ||
        h.layout != L->layout || h.pop_bytes != L->lay.pop_bytes || h.lag_bytes != L->lay.lag_bytes ||
        h.steps < 0)
        return fail(L, AXLB_EINVAL, "image does not match this lattice");
    int rc = set_device(L);
    if (rc) return rc;
    const int k = two_buffers(L) ? L->cur : (int)(h.steps & 1);
    const char *p = (const char *)host;
    void *pop = two_buffers(L) ? L->pop[k] : L->pop[0];
    HIP_TRY(L, hipMemcpyAsync(pop, p + sizeof(h), L->lay.pop_bytes, hipMemcpyHostToDevice, L->stream));
    HIP_TRY(L, hipMemcpyAsync(L->lag[k], p + sizeof(h) + L->lay.pop_bytes, L->lay.lag_bytes,
                              hipMemcpyHostToDevice, L->stream));
    HIP_TRY(L, hipStreamSynchronize(L->stream));
    L->steps = h.steps;
    L->has_snap = false;
    return AXLB_OK;
}

int axlb_destroy(axlb_lattice *L) {
    if (!L) return AXLB_OK;
    // a batch keeps stepping its members' memory: refuse until it is gone
    if (L->batched)
        return fail(L, AXLB_ESTATE, "the lattice is in a batch: destroy the batch first");
    (void)hipSetDevice(L->device);
    if (L->stream) (void)hipStreamSynchronize(L->stream);
    drop_graphs(L);
    if (L->psi) (void)hipFree(L->psi);
    if (L->own_mem && L->base) (void)hipFree(L->base);
    if (L->own_stream && L->stream) (void)hipStreamDestroy(L->stream);
    delete L;
    return AXLB_OK;
}

int axlb_set_tile(axlb_lattice *L, int tile) {
    if (!L) return fail(nullptr, AXLB_EINVAL, "lattice is NULL");
    if (L->batched) return fail(L, AXLB_ESTATE, "the lattice is in a batch");
    if (tile < 0 || tile >= tile_count()) return fail(L, AXLB_EINVAL, "tile out of range");
    if (tile != L->tile) {
        int rc = set_device(L);
        if (rc) return rc;
        HIP_TRY(L, hipStreamSynchronize(L->stream));
        drop_graphs(L);
        L->tile = tile;
    }
    return AXLB_OK;
}

int axlb_get_tile(const axlb_lattice *L, int *tile, int *tile_r, int *tile_z) {
    if (!L) return fail(nullptr, AXLB_EINVAL, "lattice is NULL");
    int bx, by;
    tile_shape(L->tile, &bx, &by);
    if (tile) *tile = L->tile;
    if (tile_r) *tile_r = bx;
    if (tile_z) *tile_z = by;
    return AXLB_OK;
}

int axlb_tile_shape(int tile, int *tile_r, int *tile_z) {
    if (tile < 0 || tile >= tile_count()) return fail(nullptr, AXLB_EINVAL, "tile out of range");
    tile_shape(tile, tile_r, tile_z);
    return AXLB_OK;
}

int axlb_autotune(axlb_lattice *L, int steps_per_trial, double *ms_per_step, int *best) {
    if (!L) return fail(nullptr, AXLB_EINVAL, "lattice is NULL");
    if (L->batched) return fail(L, AXLB_ESTATE, "the lattice is in a batch");
    if (steps_per_trial < 2) return fail(L, AXLB_EINVAL, "steps_per_trial must be >= 2");
    int rc = lattice_start(L);
    if (rc) return rc;
    // the trials step the lattice: keep the state and restore it afterwards
    const size_t pops = (two_buffers(L) ? 2 : 1) * L->lay.pop_bytes;
    const size_t bytes = pops + 2 * L->lay.lag_bytes;
    char *keep = nullptr;
    if (hipMalloc((void **)&keep, bytes) != hipSuccess) return fail(L, AXLB_ENOMEM, "autotune snapshot");
    const long steps0 = L->steps;
    const int cur0 = L->cur;
    const int tile0 = L->tile;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    auto cleanup = [&]() {
        if (e0) (void)hipEventDestroy(e0);
        if (e1) (void)hipEventDestroy(e1);
        (void)hipFree(keep);
    };
    // pop[0], (pop[1]), lag[0], lag[1] are consecutive in the lattice block
    if (hipMemcpyAsync(keep, L->pop[0], bytes, hipMemcpyDeviceToDevice, L->stream) != hipSuccess ||
        hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) {
        cleanup();
        return fail(L, AXLB_EDEVICE, "autotune setup");
    }
    double best_ms = 1e300;
    int best_tile = tile0;
    for (int t = 0; t < tile_count(); ++t) {
        L->tile = t;
        int r2 = AXLB_OK;
        for (int s = 0; s < 2 && r2 == AXLB_OK; ++s) r2 = launch_one(L);
        (void)hipEventRecord(e0, L->stream);
        for (int s = 0; s < steps_per_trial && r2 == AXLB_OK; ++s) r2 = launch_one(L);
        (void)hipEventRecord(e1, L->stream);
        float ms = 0.f;
        if (r2 != AXLB_OK || hipEventSynchronize(e1) != hipSuccess ||
            hipEventElapsedTime(&ms, e0, e1) != hipSuccess) {
            L->tile = tile0;
            cleanup();
            return r2 != AXLB_OK ? r2 : fail(L, AXLB_EDEVICE, "autotune timing");
        }
        const double per = ms / steps_per_trial;
        if (ms_per_step) ms_per_step[t] = per;
        if (per < best_ms) {
            best_ms = per;
            best_tile = t;
        }
    }
    hipError_t e = hipMemcpyAsync(L->pop[0], keep, bytes, hipMemcpyDeviceToDevice, L->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(L->stream);
    cleanup();
    if (e != hipSuccess) return fail(L, AXLB_EDEVICE, "autotune restore");
    L->steps = steps0;
    L->cur = cur0;
    L->has_snap = false;
    if (best_tile != L->tile || L->tile != tile0) drop_graphs(L);
    L->tile = best_tile;
    if (best) *best = best_tile;
    return AXLB_OK;
}

int axlb_halo_bytes(const axlb_lattice *L, size_t *bytes) {
    if (!L || !bytes) return fail(nullptr, AXLB_EINVAL, "NULL argument");
    *bytes = L->lay.halo_pop_bytes + L->lay.halo_lag_bytes;
    return AXLB_OK;
}

int axlb_halo_export(axlb_lattice *L, int face, void *device_dst) {
    if (!L || !device_dst) return fail(L, AXLB_EINVAL, "NULL argument");
    if (face != AXLB_Z_LO && face != AXLB_Z_HI) return fail(L, AXLB_EINVAL, "halo faces are z faces");
    if (L->layout != AXLB_LAYOUT_AB) return fail(L, AXLB_EINVAL, "halos need the AB layout");
    int rc = set_device(L);
    if (rc) return rc;
    // the row next to the face, of the state the next step reads
    const long long row = face == AXLB_Z_LO ? 0 : L->Nz - 1;
    const size_t es = storage_size(L->storage);
    const size_t pitch = (size_t)L->lay.pitch, plane = (size_t)L->lay.plane;
    char *dst = (char *)device_dst;
    const char *pop = (const char *)L->pop[L->cur] + row * pitch * es;
    HIP_TRY(L, hipMemcpy2DAsync(dst, pitch * es, pop, plane * es, L->Nr * es, NPOP,
                                hipMemcpyDeviceToDevice, L->stream));
    // the halo row's lagged fields use the block layout with pitch-element
    // planes: three velocity planes of vb-byte elements, then T in FP32
    const char *lag = L->lag[L->cur];
    char *hl = dst + L->lay.halo_pop_bytes;
    const size_t vb = lag_vb(L->storage);
    HIP_TRY(L, hipMemcpy2DAsync(hl, pitch * vb, lag + row * pitch * vb, plane * vb, L->Nr * vb, 3,
                                hipMemcpyDeviceToDevice, L->stream));
    HIP_TRY(L, hipMemcpyAsync(hl + 3 * pitch * vb, lag + 3 * plane * vb + row * pitch * sizeof(float),
                              L->Nr * sizeof(float), hipMemcpyDeviceToDevice, L->stream));
    return AXLB_OK;
}

int axlb_halo_import(axlb_lattice *L, int face, const void *device_src) {
    if (!L || !device_src) return fail(L, AXLB_EINVAL, "NULL argument");
    if (face != AXLB_Z_LO && face != AXLB_Z_HI) return fail(L, AXLB_EINVAL, "halo faces are z faces");
    int rc = set_device(L);
    if (rc) return rc;
    HIP_TRY(L, hipMemcpyAsync(L->halo[face - AXLB_Z_LO], device_src,
                              L->lay.halo_pop_bytes + L->lay.halo_lag_bytes,
                              hipMemcpyDeviceToDevice, L->stream));
    return AXLB_OK;
}

const char *axlb_last_error(const axlb_lattice *L) {
    return L ? L->err.c_str() : g_create_error.c_str();
}

}  // extern "C"
