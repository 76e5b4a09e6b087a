/*
 * Reference oracle for the axisymmetric cascaded central-moment lattice
 * Boltzmann time step of Hajabdollahi, Premnath & Welch, "Cascaded lattice
 * Boltzmann method based on central moments for axisymmetric thermal flows
 * including swirling effects" (arXiv 1806.10241), Section 2.
 *
 * TEST INFRASTRUCTURE ONLY.  This is a plain, slow FP64 CPU implementation
 * written from the paper's equations.  It exists so that tests, the smoke
 * check and the CPU baseline of the benchmark can check the HIP library
 * against it.  It shares no code, header, table or helper with the HIP path,
 * and the HIP path never calls it.
 *
 * Conventions (Section 2.1, eq. 2): x is the axial coordinate z, y the radial
 * coordinate r, u_x = u_z, u_y = u_r, psi = rho*u_theta, phi = T.
 * A lattice has Nz nodes along x (index i) and Nr nodes along y (index j);
 * host field arrays are laid out [i][j] (j fastest), length Nz*Nr.
 */
#ifndef AXLB_ORACLE_H
#define AXLB_ORACLE_H

#ifdef __cplusplus
extern "C" {
#endif

/* Faces of the meridian-plane rectangle. */
enum { ORC_R_IN = 0, ORC_R_OUT = 1, ORC_Z_LO = 2, ORC_Z_HI = 3 };
/* The three distribution functions: f (D2Q9), g (D2Q5, psi), h (D2Q5, T). */
enum { ORC_FLOW = 0, ORC_SWIRL = 1, ORC_THERMAL = 2 };
/* Boundary kinds.  NOSLIP, DIRICHLET, OMEGA_R and ADIABATIC are solid walls
 * (half-way between the last fluid node and the first solid node); VELOCITY
 * (f only) is a wall of the same kind through which the fluid crosses with
 * the imposed normal velocity `value` (along +y on radial faces, +x on axial
 * faces: an inlet or outlet), with g and h imposed there; SLIP (f only, on
 * axial faces) is a flat free surface, half-way like a wall: no flow
 * through it and no shear stress on it (the melt surface of Section 3.6),
 * with g and h wall rules; MIRROR is the symmetry axis; PERIODIC wraps the
 * axial direction.  (6 is left unused so that the numbering matches the HIP
 * library's.) */
enum {
    ORC_NOSLIP = 0, ORC_PERIODIC = 1, ORC_MIRROR = 2,
    ORC_DIRICHLET = 3, ORC_OMEGA_R = 4, ORC_ADIABATIC = 5, ORC_VELOCITY = 7,
    ORC_SLIP = 8
};
/* Fields inside the central differences of the sources:
 * 1 = output fields of the current step (after streaming, eq. 18, 35, 47),
 * 2 = pre-collision fields of the previous step (after eq. 21, 38, 48). */
enum { ORC_DERIV_CURRENT = 1, ORC_DERIV_PREVIOUS = 2 };

/* A boundary rule.  DIRICHLET on an axial face imposes value + slope * y
 * (y the radius where a link crosses the face); slope is 0 elsewhere. */
typedef struct { int kind; double value; double slope; } orc_bc;

typedef struct {
    int Nr, Nz;
    int cylinder;      /* 1: solid cylinder, axis at y = 0; 0: annulus   */
    double r_inner;    /* annulus: radius of the inner wall               */
    double nu, alpha;  /* kinematic viscosity, thermal diffusivity        */
    double omega3;     /* bulk-viscosity rate of the D2Q9 collision       */
    double omega6, omega7, omega8;
    double omega_psi3, omega_psi4, omega_phi3, omega_phi4;
    double g_axial;    /* uniform axial body force per unit mass          */
    double gbeta;      /* buoyancy coefficient g*beta                     */
    double T0;         /* Boussinesq reference temperature                */
    int deriv_mode;    /* ORC_DERIV_CURRENT or ORC_DERIV_PREVIOUS         */
    orc_bc bc[4][3];   /* [face][field]                                   */
    /* Axial faces in two parts (Section 3.6: crystal and free surface on
     * the top).  split[f] (f = 0: z_lo, 1: z_hi) = s in 1..Nr-1: a link
     * that crosses the face at radial column c >= s - 1/2 (c = j for a
     * link along x into node column j, j - e_y/2 for a diagonal one, so
     * each link has one rule) takes outer[f][field], the others
     * bc[face][field]; 0 leaves the face whole.  The derivative ghost of
     * node column j takes the rule of column j. */
    int split[2];
    orc_bc outer[2][3];
} orc_params;

typedef struct orc_state orc_state;

/* Creates a lattice in the equilibrium state of the given fields (any
 * pointer may be NULL: rho=1, velocities 0, T=0).  Returns NULL on invalid
 * parameters. */
orc_state *orc_create(const orc_params *p, const double *rho, const double *ur,
                      const double *uz, const double *uth, const double *T);
void orc_destroy(orc_state *s);
void orc_step(orc_state *s, long n);
long orc_steps_done(const orc_state *s);

/* Macroscopic fields that the next step's collision sees: the half-step
 * density, velocities, u_theta = psi/rho and T.  Any pointer may be NULL. */
void orc_fields(const orc_state *s, double *rho, double *ur, double *uz,
                double *uth, double *T);
/* Wall heat-transfer numbers.  Annulus: inner and outer cylinder.
 * Cylinder: bottom (z_lo) and top (z_hi) lids.  mean = (a + b) / 2. */
void orc_nusselt(const orc_state *s, double *nu_a, double *nu_b, double *mean);
/* Stream function of the meridian flow (Section 3.6, Table 4), defined by
 * d psi / d y = -y u_x (and d psi / d x = y u_y) with psi = 0 on the inner
 * face: psi[i][j] is its value at radius y_j + 1/2, the outer edge of node
 * j's cell, -sum_{k <= j} y_k u_x(i, k) (midpoint rule over the cells, on
 * the fields of orc_fields).  *lo, *hi = its smallest and largest value.
 * Any pointer may be NULL. */
void orc_stream_function(const orc_state *s, double *psi, double *lo, double *hi);
/* 1 when every stored population is finite. */
int orc_all_finite(const orc_state *s);

/* State transfer: 19*Nz*Nr post-collision populations (f then g then h,
 * each [node][q]) followed by 4*Nz*Nr lagged derivative fields. */
long orc_state_len(const orc_state *s);
void orc_get_state(const orc_state *s, double *out);
void orc_set_state(orc_state *s, const double *in, long steps_done);
/* Raw populations as [field][q][i][j], one lattice at a time. */
void orc_get_populations(const orc_state *s, double *f9, double *g5, double *h5);

/* ---- node-level operators, exposed so that tests can pin them ---- */

/* Maxwellian-central-moment equilibria (D2Q9 and D2Q5). */
void orc_equilibrium_f(double rho, double ux, double uy, double feq[9]);
void orc_equilibrium_adv(double s, double ux, double uy, double geq[5]);

/* D2Q9 cascaded collision with the split mass and momentum sources:
 * eq. (17) with the pre-collision (rho, ux, uy) of eq. (21), source moments
 * of eq. (26), post-collision populations f + K p (eq. 16a).  om[3..8] are
 * omega_3..omega_8 (om[0..2] unused). */
void orc_collide_f(const double f[9], double rho, double ux, double uy,
                   double MA, double Fx, double Fy, const double om[9],
                   double fp[9]);
/* D2Q5 cascaded collision for an advected scalar s (psi or phi) with its
 * split source S: eq. (34)/(49) with the sign reading documented in the
 * implementation, eq. (41)/(51), and g + L q (eq. 33a/46a).  om[1..4]. */
void orc_collide_adv(const double g[5], double s, double ux, double uy,
                     double S, const double om[5], double gp[5]);

/* Pre-collision half source step of one node at radius y (eq. 21, 38, 48
 * with the sources of eq. 4, 5, 7, 9 evaluated at the half-step state):
 * mom = {rho^o, j_x^o, j_y^o, psi^o, phi^o}, d = {d_x u_y, d_y u_x, d_y u_y,
 * d_y u_theta, d_y phi}; out = {M^A, F_x, F_y, S_psi, S_phi, rho, u_x, u_y,
 * psi, phi}. */
void orc_half_step(const orc_params *p, double y, const double mom[5], const double d[5],
                   double out[10]);

/* Convergence residual between two snapshots of n nodes taken K steps
 * apart (the definition is at the function). */
double orc_residual(long n, const double *ur1, const double *uz1, const double *uth1,
                    const double *T1, const double *ur0, const double *uz0,
                    const double *uth0, const double *T0, long K);

/* Threads of the per-node loops (OpenMP build); results do not depend on
 * the count, since every node is computed on its own. */
void orc_set_threads(int n);
int orc_threads(void);

#ifdef __cplusplus
}
#endif
#endif
