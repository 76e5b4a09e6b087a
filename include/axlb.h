/*
 * axlb: the time step of the axisymmetric cascaded central-moment lattice
 * Boltzmann method for thermal flows with swirl (Hajabdollahi, Premnath &
 * Welch, arXiv 1806.10241, Section 2) on AMD Instinct MI355X (gfx950).
 *
 * One lattice is the meridian plane of an annulus (R_i <= r <= R_i + Nr) or
 * of a solid cylinder (0 <= r <= Nr) with Nz nodes along the axis, in
 * lattice units (dx = dt = 1).  Each node carries the three distribution
 * functions of the paper: a D2Q9 f for rho, u_z, u_r (Section 2.2), a D2Q5 g
 * for psi = rho u_theta (Section 2.3) and a D2Q5 h for T (Section 2.4).
 * One call of axlb_step advances all of them by the symmetric split scheme
 * of eq. (20), (37) and (45): streaming, pre-collision half source step
 * (eq. 21, 38, 48), cascaded collision (eq. 17, 34, 49), post-collision
 * source moments (eq. 26, 41, 51), with the geometric sources of eq. (4),
 * (7), (9) and the body force of eq. (5).
 *
 * Conventions shared by every call:
 *  - Status: functions return AXLB_OK (0) or a negative AXLB_E* code; no
 *    exception crosses this interface; axlb_last_error() gives the message.
 *  - Host field arrays are FP64, length Nz*Nr, layout [iz][ir] (r fastest),
 *    owned by the caller.  Device state is owned by the library.
 *  - Coordinates: z (axial, index iz) is the paper's x, r (radial, index ir)
 *    its y.  Nodes sit half a spacing from walls and from the axis:
 *    r = r0 + ir + 1/2 with r0 = R_i (annulus) or 0 (cylinder).
 *  - Ordering: axlb_step is asynchronous on the lattice's HIP stream; calls
 *    that return host data (get_moments, nusselt, residual, save) wait for
 *    that stream.  One lattice must not be used from two threads at once;
 *    different lattices are independent.
 */
#ifndef AXLB_H
#define AXLB_H

#include <stddef.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- status codes ---- */
#define AXLB_OK 0
#define AXLB_EINVAL (-1)    /* bad argument: sizes, tau <= 1/2, Pr != nu/alpha, BC mix */
#define AXLB_ENOMEM (-2)    /* device memory or the pool's memory budget exhausted     */
#define AXLB_EUNSTABLE (-3) /* a non-finite value was found in the state               */
#define AXLB_EDEVICE (-4)   /* a HIP runtime call failed                               */
#define AXLB_ESTATE (-5)    /* call not valid in the current state                     */

/* ---- population storage (Section 2; FP32 arithmetic in every case) ---- */
#define AXLB_F32 0   /* 4 bytes per population, 152 B per node update         */
#define AXLB_F16 1   /* IEEE binary16 of the value times 2^8, stochastic
                        rounding, 76 B per node update                         */
#define AXLB_BF16 2  /* bfloat16, stochastic rounding, 76 B per node update    */
/* Stochastic rounding draws its random bits from a hash of the value and
 * the slot, so that a run (and a checkpoint replay) is deterministic.
 * bfloat16 with lagged derivatives stores each population minus its linear
 * equilibrium part (3 w_q e_q.u for f, w_q u_theta for g, w_q (T - T_ref)
 * for h) taken at the lagged fields of the node that wrote it, so bfloat16
 * takes the lagged derivatives only (AXLB_DERIV_LAGGED); its checkpoint
 * images carry a magic of their own. */

/* ---- streaming layouts ---- */
#define AXLB_LAYOUT_AA 0 /* one population buffer, in place, alternating phases */
#define AXLB_LAYOUT_AB 1 /* two population buffers, pull streaming              */
#define AXLB_LAYOUT_AB2 2 /* two buffers, two time steps per launch (below)     */
/* AXLB_LAYOUT_AB2 holds the same two buffers as AB.  One launch advances two
 * time steps: a workgroup takes a 30 x 22 tile and the one-node ring around
 * it through the first step, keeping the populations and lagged fields in
 * LDS, then takes its tile through the second step.  The results are
 * bit-identical to AB; each pair of steps reads and writes the state once.
 * An odd step count ends with one AB step.  Choosing a layout: AB2 moves
 * half the bytes per step and wins wherever the step is bound by memory
 * (measured with FP32 storage: 1024 x 2048 AB2 41k against AA 35k MLUPS,
 * 2048 x 4096 AB2 42k against AA 25k); with 16-bit storage, where the step
 * is bound by arithmetic, AA is faster at 1024 x 2048 (53k against 48k).
 * AA needs one population buffer instead of two. */

/* ---- time level of the central differences in the geometric sources ----
 * (eq. 4b, 4c, 7, 9; Section 3.2 only says "central difference").
 * LAGGED: the previous step's pre-collision fields u_z, u_r, u_theta, T,
 *   kept in a side buffer (either layout; the only form the single-buffer
 *   layout allows, since in-place streaming overwrites a neighbour's
 *   current populations).
 * CURRENT: this step's output fields (after streaming, before the source
 *   half step) of the neighbours; needs AXLB_LAYOUT_AB and FP32 or binary16
 *   storage (bfloat16 meets the 16-bit accuracy only through its offset
 *   encoding, which takes the lagged fields: AXLB_EINVAL).
 * The two share every steady state. */
#define AXLB_DERIV_LAGGED 0
#define AXLB_DERIV_CURRENT 1

/* ---- geometry ---- */
#define AXLB_ANNULUS 0  /* fluid between r = R_i and r = R_i + Nr            */
#define AXLB_CYLINDER 1 /* fluid between the axis r = 0 and r = Nr           */

/* ---- faces, distribution functions and boundary kinds ---- */
#define AXLB_R_IN 0  /* inner cylinder wall, or the axis of a cylinder */
#define AXLB_R_OUT 1
#define AXLB_Z_LO 2
#define AXLB_Z_HI 3

#define AXLB_FLOW 0    /* f: rho, u_z, u_r   */
#define AXLB_SWIRL 1   /* g: psi = rho u_theta */
#define AXLB_THERMAL 2 /* h: T               */

#define AXLB_NOSLIP 0    /* wall at rest for f (half-way bounce-back); for g: u_theta = 0 */
#define AXLB_PERIODIC 1  /* z faces only, set for all fields on both z faces           */
#define AXLB_MIRROR 2    /* the axis of a cylinder (set automatically, all fields)      */
#define AXLB_DIRICHLET 3 /* g: imposed u_theta = value; h: imposed T = value            */
#define AXLB_OMEGA_R 4   /* g: u_theta = Omega * r at the wall, Omega = value (NaN: the
                            lattice's Omega)                                            */
#define AXLB_ADIABATIC 5 /* h (or g): zero normal flux                                  */
#define AXLB_HALO 6      /* z faces only, all fields, AXLB_LAYOUT_AB with lagged derivatives:
                            the neighbours beyond the face are the boundary row of an
                            adjacent slab, imported with axlb_halo_import (below)        */
#define AXLB_VELOCITY 7  /* f only: a wall through which the fluid crosses with the imposed
                            normal velocity `value` (along +r on r faces, +z on z faces):
                            an inlet or outlet; tangential velocity 0.  Moving-wall
                            bounce-back with rho_0 = 1, so the wall carries the mass flux
                            `value` per unit area.  g on such a face must impose u_theta
                            (NOSLIP, DIRICHLET, OMEGA_R) and h must impose T (DIRICHLET);
                            their anti-bounce-back adds the advective part u_n^2 s_w.  No
                            case of the paper uses one                                  */
#define AXLB_SLIP 8      /* f only, z faces: a flat free surface half-way between the last
                            row and the next (Section 3.6, the melt surface beside the
                            crystal): u_z = 0 and no shear stress, by specular reflection
                            of the populations (the pull takes the post-collision
                            population of the neighbour along r, with e_z reversed).  g and
                            h on the face take wall rules (ADIABATIC for d u_theta/dz = 0) */

typedef struct axlb_lattice axlb_lattice;

typedef struct {
    int kind;       /* AXLB_ANNULUS or AXLB_CYLINDER                      */
    double r_inner; /* annulus inner radius R_i > 0 (ignored for cylinder) */
} axlb_geometry;

/* Relaxation rates the transport coefficients leave free (text after
 * eq. 17, 34, 49).  omega_4 = omega_5 and omega^psi_{1,2} follow from nu,
 * omega^phi_{1,2} from alpha.  NULL selects omega3 = 1 and all others 1. */
typedef struct {
    double omega3;                 /* bulk viscosity xi = (1/omega3 - 1/2)/3 */
    double omega6, omega7, omega8; /* third and fourth order, D2Q9           */
    double omega_psi3, omega_psi4; /* second order, D2Q5 for psi             */
    double omega_phi3, omega_phi4; /* second order, D2Q5 for T               */
} axlb_relax;

typedef struct {
    int storage;  /* AXLB_F32 | AXLB_F16 | AXLB_BF16                         */
    int layout;   /* AXLB_LAYOUT_AA (default) | AXLB_LAYOUT_AB | AXLB_LAYOUT_AB2 */
    double T_ref; /* temperature about which h is stored (shifted storage)   */
    void *stream; /* hipStream_t to run on; NULL: the library makes its own  */
    int device;   /* HIP device ordinal; -1: the current device              */
    void *device_buf;    /* optional caller-owned device memory of at least
                            axlb_state_bytes() bytes, 256-byte aligned, that
                            must outlive the lattice; NULL: the library
                            allocates (and frees) its own                   */
    size_t device_bytes; /* size of device_buf                              */
    int deriv;           /* AXLB_DERIV_LAGGED (default) | AXLB_DERIV_CURRENT */
    int row0;            /* global index of row 0 when the lattice is a slab of
                            a taller one (HALO faces), >= 0, default 0: the
                            stochastic rounding of 16-bit stores keys on
                            global rows, so slabs reproduce the uncut lattice
                            bit for bit in every storage                    */
} axlb_options;

/* Bytes of device memory a lattice of this size holds (populations, lagged
 * derivative fields and reduction scratch). */
int axlb_state_bytes(int Nr, int Nz, int storage, int layout, size_t *bytes);

/* Creates a lattice at rest (rho = 1, u = 0, T = T_ref).
 *  Nr, Nz  fluid nodes along r and z (Nr >= 2, Nz >= 1; Nz >= 2 unless z is
 *          periodic; Nz times Nr rounded up to a multiple of 64 at most 2^30,
 *          about 10^9 nodes).
 *  nu      kinematic viscosity; omega_4,5 = omega^psi_1,2 = 1/(3 nu + 1/2)
 *          (text after eq. 17 and eq. 34); nu > 0 (tau > 1/2).
 *  alpha   thermal diffusivity; omega^phi_1,2 = 1/(3 alpha + 1/2) (after
 *          eq. 49); alpha > 0.
 *  Pr      Prandtl number, checked against nu/alpha to 1e-9 relative
 *          (0: not checked).
 *  Ra      Rayleigh number (Section 3.2) with L = Nr and dT = 1:
 *          g beta = Ra nu alpha / Nr^3; the buoyancy force is
 *          g beta (T - T0) along +z (eq. 5, F^b_x).
 *  Omega   angular velocity of OMEGA_R faces set with value NaN.
 *  w       relaxation rates (NULL: defaults); opt: storage/layout/stream/
 *          derivative time level (NULL: FP32, AA, T_ref = 0.5, own stream,
 *          current device, lagged); AXLB_EINVAL for CURRENT with any
 *          layout but AXLB_LAYOUT_AB.
 * Defaults: every face a no-slip wall with u_theta = 0 and zero heat flux;
 * a cylinder's inner face is the axis.  *out receives the handle. */
int axlb_lattice_create(int Nr, int Nz, const axlb_geometry *geo, double nu, double alpha,
                        double Pr, double Ra, double Omega, const axlb_relax *w,
                        const axlb_options *opt, axlb_lattice **out);

/* Boundary rule of one distribution function on one face (Section 3.1 to
 * 3.4: half-way bounce-back for no-slip, the advection-diffusion wall
 * rule for imposed u_theta or T and zero flux, the axis mirror, periodic
 * z).  Only before the first step; AXLB_ESTATE afterwards. */
int axlb_set_bc(axlb_lattice *lat, int face, int field, int kind, double value);

/* Outer part of a z face (Section 3.6: the crystal covers the top for
 * r < R_x, the free surface the rest).  From radial node `from` on
 * (1 <= from < Nr, the same for all three fields), face AXLB_Z_LO or
 * AXLB_Z_HI takes the rule (kind, value) for distribution `field` instead
 * of the one axlb_set_bc gave it: f NOSLIP or SLIP; g NOSLIP, DIRICHLET,
 * OMEGA_R or ADIABATIC; h DIRICHLET or ADIABATIC.  A DIRICHLET value may
 * vary linearly with the radius, value + slope * r (r of the link's
 * crossing, r0 + j + 1/2 along z); slope must be 0 for every other kind.
 * A link crosses the face at radial position j - e_r/2 for a population
 * that arrives at node column j with radial velocity e_r; it takes the
 * outer rule when that position is >= from - 1/2, so that each link has
 * one rule and mass is conserved where the parts meet.  Fields of the part
 * not yet given are NOSLIP, NOSLIP, ADIABATIC.  Both parts of a split face
 * must be walls or free surface (no PERIODIC, HALO or VELOCITY); a
 * cylinder with a split lid has no Nusselt numbers (axlb_nusselt returns
 * AXLB_ESTATE).  Only before the first step; AXLB_EINVAL for any other
 * argument. */
int axlb_set_bc_outer(axlb_lattice *lat, int face, int from, int field, int kind, double value,
                      double slope);

/* Axial body force per unit mass g_axial and Boussinesq reference T0
 * (eq. 5: F^b_x = g_axial + g beta (T - T0)).  Only before the first step. */
int axlb_set_body_force(axlb_lattice *lat, double g_axial, double T0);

/* Resets the state to the equilibria of the given host fields (any may be
 * NULL: rho = 1, velocities 0, T = T_ref); step count returns to 0. */
int axlb_set_fields(axlb_lattice *lat, const double *rho, const double *ur, const double *uz,
                    const double *uth, const double *T);

/* Enqueues n time steps on the lattice's stream (asynchronous).  The steps
 * run as replays of captured HIP graphs: bundles of 100 steps, then one
 * graph of the remaining steps (a single remaining step is a plain launch).
 * A graph is captured the first time its length and starting phase occur
 * and is kept with the lattice (the 100-step bundles always, at most 8
 * other lengths).  Results are identical to one launch per step. */
int axlb_step(axlb_lattice *lat, long n);
/* Graph replay on (1, the default) or off (0): off, axlb_step makes one
 * plain kernel launch per step (per pair of steps in AXLB_LAYOUT_AB2), for
 * profilers that attribute counters to single dispatches.  Same results. */
int axlb_set_graphs(axlb_lattice *lat, int enable);
/* Captures, without running them, the graphs that axlb_step(lat, n) would
 * replay from the current state, so that a timed or latency-bound call
 * does not pay for the capture.  AXLB_ESTATE for a batch member. */
int axlb_prepare_steps(axlb_lattice *lat, long n);
long axlb_steps_done(const axlb_lattice *lat);
/* Waits for the lattice's stream. */
int axlb_sync(axlb_lattice *lat);

/* Fields the next step's collision sees (after the pre-collision half
 * source step, eq. 21, 38, 48): rho, u_r, u_z, u_theta = psi/rho, T.
 * Any pointer may be NULL.  Synchronous. */
int axlb_get_moments(axlb_lattice *lat, double *rho, double *ur, double *uz, double *uth,
                     double *T);

/* Wall Nusselt numbers (Section 3.2), FP64 reduction on the device.
 * Annulus: a = Nu_i at R_i, b = Nu_o at R_o (both r walls must impose T).
 * Cylinder: a, b = bottom and top lid (both z walls must impose T).
 * mean = (a + b)/2.  Synchronous. */
int axlb_nusselt(axlb_lattice *lat, double *nu_a, double *nu_b, double *mean);

/* Stream function of the meridian flow (Section 3.6, Table 4): psi with
 * d psi / d r = -r u_z (and d psi / d z = r u_r), 0 on the inner face (the
 * axis, or R_i), integrated outward over the node cells by the midpoint
 * rule on the fields of axlb_get_moments: psi[iz][ir] = -sum_{k <= ir}
 * r_k u_z(iz, k), its value at r0 + ir + 1, the outer edge of the node's
 * cell.  FP64 on the device, one thread per row.  psi (host, Nr * Nz
 * doubles) receives the field, *psi_min and *psi_max its smallest and
 * largest value (cells turning one way and the other); any pointer may be
 * NULL.  The device buffer (Nr * Nz + 2 Nz doubles) is allocated on the
 * first call and kept with the lattice.  Synchronous. */
int axlb_stream_function(axlb_lattice *lat, double *psi, double *psi_min, double *psi_max);

/* Convergence residual, FP64 on the device: the largest of
 * ||c_now - c_then||_2 / (K ||speed_now||_2) over the velocity components
 * c = u_r, u_z, u_theta (speed = |u|) and ||T_now - T_then||_2 /
 * (K ||T_now||_2), "then" being the fields at the previous call and K the
 * steps in between (terms with zero norm are skipped).  The first call only
 * records the fields and returns +inf.  AXLB_EUNSTABLE if a non-finite value
 * is found.  Synchronous. */
int axlb_residual(axlb_lattice *lat, double *r);

/* Checkpoint: the whole state (populations, lagged fields, phase, step
 * count) as an opaque byte image in caller memory.  Synchronous. */
int axlb_state_size(const axlb_lattice *lat, size_t *bytes);
int axlb_save(axlb_lattice *lat, void *host, size_t bytes);
int axlb_load(axlb_lattice *lat, const void *host, size_t bytes);

/* Step-kernel tile shapes: AXLB_NTILES workgroup shapes of tile_r x tile_z
 * nodes.  axlb_set_tile selects one for a lattice (results do not depend on
 * it); axlb_autotune times every shape for steps_per_trial steps on the
 * lattice itself, restores the state it found, selects the fastest, and
 * returns the per-step times in ms_per_step[AXLB_NTILES] (may be NULL).
 * The two-step launches of AXLB_LAYOUT_AB2 use a fixed 30 x 22 tile; the
 * selected shape applies to its single steps. */
#define AXLB_NTILES 8
int axlb_tile_shape(int tile, int *tile_r, int *tile_z);
int axlb_set_tile(axlb_lattice *lat, int tile);
int axlb_get_tile(const axlb_lattice *lat, int *tile, int *tile_r, int *tile_z);
int axlb_autotune(axlb_lattice *lat, int steps_per_trial, double *ms_per_step, int *best);

/* Releases the lattice and the device memory the library allocated for it
 * (memory lent through device_buf stays the caller's).  AXLB_ESTATE, with
 * nothing released, while the lattice is a member of a batch: the batch
 * would go on stepping its memory.  NULL is a no-op. */
int axlb_destroy(axlb_lattice *lat);

/* Wall Nusselt numbers as axlb_nusselt computes them (same per-node
 * arithmetic; the FP64 sums run in another order, so results agree to
 * rounding), for callers that cannot allocate device memory: tight serving
 * or monitoring loops, harnesses that forbid hipMalloc, processes whose
 * device memory is fully reserved.  It calls no allocating routine (only a
 * fixed device-to-host copy of the two sums) and leaves the lattice's own
 * field and reduction buffers untouched.  Its partial sums live in a fixed
 * per-device array of 128 KiB inside the library (held until the process
 * ends) that serves walls of up to 2^21 nodes (Nz for an annulus, Nr for a
 * cylinder); longer walls give AXLB_EINVAL.  Every call on one device
 * shares that array: calls that overlap on one device (from several host
 * threads, or on streams that run concurrently) race and must be ordered
 * by the caller.  Synchronous on the lattice's stream; other errors as
 * axlb_nusselt. */
int axlb_nusselt_noalloc(axlb_lattice *lat, double *nu_a, double *nu_b, double *mean);

/* ---- slabs of one lattice (a lattice cut along z, one piece per GPU) ----
 * A slab's cut faces have kind AXLB_HALO.  Before each step, the row of
 * each neighbouring slab next to the cut (its populations and lagged
 * fields, as they stand before that step) must sit in the slab's halo of
 * that face: axlb_halo_export packs a slab's boundary row next to `face`
 * into axlb_halo_bytes bytes of device memory, the caller moves them (a
 * copy on one device, a send and receive between devices) and
 * axlb_halo_import copies them into the neighbour's halo of the facing
 * face.  Steps then reproduce the uncut lattice bit for bit.  Both calls
 * are asynchronous on the lattice's stream; the caller orders the copies
 * between lattices (synchronise, or wait on events).  AXLB_EINVAL for a
 * face other than Z_LO/Z_HI, NULL pointers or a layout other than AB. */
int axlb_halo_bytes(const axlb_lattice *lat, size_t *bytes);
int axlb_halo_export(axlb_lattice *lat, int face, void *device_dst);
int axlb_halo_import(axlb_lattice *lat, int face, const void *device_src);

/* ---- batches of independent lattices (uneven sizes) ----
 * A batch advances all its member lattices together: a step of many members
 * is one fused launch over a work-list of (member, tile) entries, and
 * 100-step bundles are captured as HIP graphs.  Within a bundle, runs of
 * consecutive members whose states total at most 80 MB take all 100 steps
 * before the next run starts, two runs at a time on two streams (together
 * below the 256 MB Infinity Cache); after axlb_batch_step every member has
 * advanced by the same count either way.
 * A batch of AXLB_LAYOUT_AB2 members instead advances every member by two
 * steps per launch (the two-step kernel over a work-list of (member, tile)
 * entries, all members in one launch, 100-step bundles as graphs of 50
 * launches): the state crosses HBM once per two steps, which is what a
 * batch whose states exceed the Infinity Cache gains most from.  An odd
 * step count ends with one single step of each member.
 * Members must share device, storage and layout (AA or AB2) and belong to
 * no other batch; their boundary rules are locked.  While batched, a member runs on the batch's
 * stream: axlb_get_moments, axlb_nusselt, axlb_residual and axlb_save work
 * on it as usual, whereas axlb_step, axlb_set_fields, axlb_load,
 * axlb_set_tile, axlb_autotune and axlb_destroy refuse (AXLB_ESTATE).  A
 * member's results are bit-identical to stepping it alone.  The batch does
 * not own its members: destroy the batch first, then the lattices. */
typedef struct axlb_batch axlb_batch;
#define AXLB_NSCHEDULES 4 /* launch schedules the batch autotuner tries */

int axlb_batch_create(axlb_lattice *const *lats, int n, axlb_batch **out);
int axlb_batch_size(const axlb_batch *b, int *members, long long *nodes);
/* Enqueues n steps of every member (asynchronous on the batch stream). */
int axlb_batch_step(axlb_batch *b, long n);
int axlb_batch_sync(axlb_batch *b);
/* Tile shape (as axlb_tile_shape) and schedule: blocks = 0 launches one
 * workgroup per work-list entry, blocks > 0 that many persistent workgroups
 * that loop over the entries.  AA members only (AXLB_EINVAL for AB2, whose
 * batch has one schedule). */
int axlb_batch_set_schedule(axlb_batch *b, int tile, int blocks);
int axlb_batch_get_schedule(const axlb_batch *b, int *tile, int *blocks);
/* Whole members (AA members only): a member of at most max_nodes nodes
 * (0 <= max_nodes <= AXLB_WHOLE_MAX_NODES; 0, the default, turns the mode
 * off) runs in one workgroup of its own, which takes it through all the
 * steps of a launch (a bundle's 100 in one kernel) with a workgroup barrier
 * between steps; the other members keep the work-list.  During a bundle the
 * whole members run on a chain of their own beside the work-list's.
 * Results are bitwise those of the work-list.  AXLB_EINVAL for AB2 batches
 * or max_nodes out of range.  axlb_batch_get_whole reports the limit and
 * how many members run whole. */
#define AXLB_WHOLE_MAX_NODES 65536
int axlb_batch_set_whole(axlb_batch *b, long long max_nodes);
int axlb_batch_get_whole(const axlb_batch *b, long long *max_nodes, int *members);
/* Times every tile shape with each of the AXLB_NSCHEDULES schedules (one
 * workgroup per entry, 4, 8 and 16 persistent workgroups per compute unit)
 * for steps_per_trial steps (group by group, as the bundles of
 * axlb_batch_step run); then, when some member has at most
 * AXLB_WHOLE_MAX_NODES nodes, the best of them without and with whole
 * members (each timed as a bundle runs); restores the members' state and
 * keeps the fastest (axlb_batch_get_whole tells whether members run whole).
 * ms_per_step[AXLB_NTILES * AXLB_NSCHEDULES] may be NULL.  A batch of AB2
 * members has nothing to choose: it returns at once (times 0). */
int axlb_batch_autotune(axlb_batch *b, int steps_per_trial, double *ms_per_step,
                        int *best_tile, int *best_blocks);
void axlb_batch_destroy(axlb_batch *b);
const char *axlb_batch_last_error(const axlb_batch *b);

/* The unbatched form, for comparison: advances each of n lattices by
 * `steps` steps with one kernel launch per lattice per step. */
int axlb_step_each(axlb_lattice *const *lats, int n, long steps);

/* ---- continuous-batching request pool ----
 * Solve requests (any size, parameters and storage) wait in a queue and are
 * admitted, in the pool's order (first come first served unless
 * axlb_pool_set_policy says otherwise), while their state fits a fixed
 * device-memory budget (and at most max_members run at once).  Admitted
 * requests stay resident and advance together: each axlb_pool_tick runs one
 * 100-step bundle of every resident request as fused batched launches (one
 * batch per storage type, overlapping on the device), then retires every
 * request whose residual (axlb_residual, checked once per bundle) is below
 * its tol or whose step count reached max_steps.  Requests submitted
 * between ticks join at the next tick.  FP32 requests run in the two-step
 * layout (AXLB_LAYOUT_AB2), 16-bit ones in the single-buffer layout
 * (AXLB_LAYOUT_AA); the budget counts axlb_state_bytes of that layout.  A
 * request's result is bit-identical to running the same case alone in that
 * layout for the same number of steps. */
typedef struct axlb_pool axlb_pool;
#define AXLB_REQ_QUEUED 0
#define AXLB_REQ_RUNNING 1
#define AXLB_REQ_DONE 2
#define AXLB_REQ_FAILED 3

typedef struct {
    int Nr, Nz;
    axlb_geometry geo;
    double nu, alpha, Pr, Ra, Omega; /* as axlb_lattice_create           */
    double g_axial, T0;              /* as axlb_set_body_force           */
    int bc_kind[4][3];               /* [face][field], as axlb_set_bc    */
    double bc_value[4][3];
    int storage;                     /* AXLB_F32 | AXLB_F16 | AXLB_BF16  */
    double T_ref;
    const double *init[5];           /* optional host fields rho, u_r, u_z,
                                        u_theta, T ([iz][ir]); copied at
                                        submission                       */
    double tol;                      /* retire when the residual < tol   */
    long max_steps;                  /* ... or at this many steps         */
} axlb_request;

int axlb_pool_create(size_t budget_bytes, int device, int max_members, axlb_pool **out);
/* Admission order and concurrency.  order: AXLB_POOL_FIFO (arrival order,
 * the default) or AXLB_POOL_SMALLEST_FIRST (least Nr*Nz*max_steps first,
 * ties in arrival order: shortest job first on the only work estimate known
 * at admission; a steady stream of small requests can delay a large one
 * indefinitely).  node_window > 0 caps the fluid nodes resident at once, so
 * that the device stays busy without time-slicing every waiting request (a
 * request larger than the window still runs when nothing else does); 0
 * lifts the cap (the default).  In either order the request next in line
 * that does not fit blocks those behind it.  Takes effect at the next tick.
 * AXLB_EINVAL for an unknown order or a negative window. */
#define AXLB_POOL_FIFO 0
#define AXLB_POOL_SMALLEST_FIRST 1
int axlb_pool_set_policy(axlb_pool *p, int order, long long node_window);
/* Queues a request (copies it); *id identifies it.  AXLB_ENOMEM if its
 * state alone exceeds the budget. */
int axlb_pool_submit(axlb_pool *p, const axlb_request *r, long *id);
/* Admission, one bundle for all resident requests, retirement.
 * Synchronous; reports how many requests run and wait afterwards. */
int axlb_pool_tick(axlb_pool *p, int *running, int *queued);
int axlb_pool_status(const axlb_pool *p, long id, int *state, long *steps, double *residual);
/* Final fields (host arrays of Nz*Nr, any may be NULL) and wall Nusselt
 * numbers (NaN when the case has no imposed wall temperatures) of a DONE
 * request, which is then forgotten; a FAILED request returns its error. */
int axlb_pool_result(axlb_pool *p, long id, double *rho, double *ur, double *uz, double *uth,
                     double *T, double *nusselt3);
int axlb_pool_usage(const axlb_pool *p, size_t *used_bytes, long long *node_updates);
void axlb_pool_destroy(axlb_pool *p);
const char *axlb_pool_last_error(const axlb_pool *p);
/* Message of the last failed call on lat (or of the last failed create when
 * lat is NULL).  Valid until the next call on lat. */
const char *axlb_last_error(const axlb_lattice *lat);

#ifdef __cplusplus
}
#endif
#endif
