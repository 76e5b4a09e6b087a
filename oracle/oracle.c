/*
 * Reference oracle for the axisymmetric cascaded LB time step (arXiv
 * 1806.10241, Section 2).  TEST INFRASTRUCTURE ONLY: used by the tests, the
 * smoke check and the CPU-baseline leg of the benchmark, never by the HIP
 * library.  Plain FP64, two A/B population arrays, pull streaming, and two
 * passes per step: (1) stream and take the output moments of every node,
 * (2) sources, pre-collision half step, cascaded collision with the source
 * moments, store.  Nothing is fused or reordered beyond what the equations
 * state, so that each function can be checked against the paper by eye.
 *
 * Readings of passages the paper leaves open are marked "Reading:" below;
 * every one is also listed with the design notes of the repository.
 */
#include "oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

/* Section 2.2, eq. (10): D2Q9 particle velocities in the order of the paper. */
static const int EX9[9] = {0, 1, 0, -1, 0, 1, -1, -1, 1};
static const int EY9[9] = {0, 0, 1, 0, -1, 1, 1, -1, -1};
/* Section 2.3, eq. (28): D2Q5 particle velocities. */
static const int EX5[5] = {0, 1, 0, -1, 0};
static const int EY5[5] = {0, 0, 1, 0, -1};

/* Lattice units, Delta x = Delta t = 1, c_s^2 = 1/3 (text after eq. 17);
 * the D2Q5 schemes use c_s^2 = 1/3 as well (text after eq. 34 and eq. 49). */
static const double CS2 = 1.0 / 3.0;

/* Derivative variables: u_x, u_y, u_theta, phi. */
enum { VX = 0, VY = 1, VT = 2, VP = 3 };

struct orc_state {
    orc_params p;
    long steps;
    double *f, *g, *h;   /* post-collision populations, [node][q]            */
    double *lag;         /* previous step's pre-collision fields u_x, u_y,
                            u_theta, phi, [node][4]                        */
};

static int node(const orc_state *s, int i, int j) { return i * s->p.Nr + j; }

static double ipow(int base, int e)
{
    double r = 1.0;
    for (int k = 0; k < e; ++k) r *= base;
    return r;
}

/* Index of the direction opposite to q, found from the velocity table. */
static int opposite(const int *ex, const int *ey, int nq, int q)
{
    for (int b = 0; b < nq; ++b)
        if (ex[b] == -ex[q] && ey[b] == -ey[q]) return b;
    return -1;
}

/* Index of the direction that is q reflected across a line y = const. */
static int reflect_y(const int *ex, const int *ey, int nq, int q)
{
    for (int b = 0; b < nq; ++b)
        if (ex[b] == ex[q] && ey[b] == -ey[q]) return b;
    return -1;
}

static int is_wall(int kind)
{
    return kind == ORC_NOSLIP || kind == ORC_DIRICHLET || kind == ORC_OMEGA_R ||
           kind == ORC_ADIABATIC || kind == ORC_VELOCITY;
}

/* Index of the direction that is q reflected across a line x = const. */
static int reflect_x(const int *ex, const int *ey, int nq, int q)
{
    for (int b = 0; b < nq; ++b)
        if (ex[b] == -ex[q] && ey[b] == ey[q]) return b;
    return -1;
}

/* Rule of distribution fld on a face where a link crosses it at twice the
 * radial column c2 (2j for a link along x into column j, 2j - e_y for a
 * diagonal one): an axial face split at column s gives its outer rule to
 * c2 >= 2s - 1. */
static const orc_bc *rule(const orc_params *p, int face, int fld, int c2)
{
    if (face >= ORC_Z_LO) {
        const int f = face - ORC_Z_LO;
        if (p->split[f] > 0 && c2 >= 2 * p->split[f] - 1) return &p->outer[f][fld];
    }
    return &p->bc[face][fld];
}

/* Velocity normal to a face that imposes one (VELOCITY for f), as the
 * component along +y (radial faces) or +x (axial faces); 0 for walls at
 * rest and free surfaces.  bcf is the f rule where the link crosses. */
static double normal_velocity(const orc_bc *bcf)
{
    return bcf->kind == ORC_VELOCITY ? bcf->value : 0.0;
}

/* Radial coordinate of node row j: nodes sit half a spacing off the wall
 * (annulus) or off the axis (cylinder). */
static double y_of(const orc_state *s, int j)
{
    return (s->p.cylinder ? 0.0 : s->p.r_inner) + j + 0.5;
}

/* Relaxation rate for a transport coefficient D with c_s^2 = 1/3:
 * D = c_s^2 (1/omega - 1/2) (text after eq. 17, eq. 34 and eq. 49). */
static double rate_for(double D) { return 1.0 / (D / CS2 + 0.5); }

/* ------------------------------------------------------------------------ */
/* Equilibria.  Their central moments equal those of the Maxwellian (text
 * after eq. 15 and after eq. 32): for D2Q9 the nine central moments
 * {1, x, y, xx, yy, xy, xxy, xyy, xxyy} are {rho, 0, 0, cs2 rho, cs2 rho, 0,
 * 0, 0, cs2^2 rho}; this set factorises into a product of the 1-D sets
 * {1, u, cs2 + u^2} per axis, which is what is written below. */
static double phi1d(int e, double u)
{
    /* 1-D weights whose zeroth, first and second raw moments are 1, u,
     * cs2 + u^2 on the velocities {-1, 0, 1}. */
    if (e == 0) return 1.0 - (CS2 + u * u);
    return 0.5 * (CS2 + u * u + e * u);
}

void orc_equilibrium_f(double rho, double ux, double uy, double feq[9])
{
    for (int a = 0; a < 9; ++a) feq[a] = rho * phi1d(EX9[a], ux) * phi1d(EY9[a], uy);
}

/* D2Q5: the five moments {1, x, y, xx, yy} of the scalar s equal
 * {s, s ux, s uy, s (cs2 + ux^2), s (cs2 + uy^2)} (Maxwellian central
 * moments with rho replaced by s). */
void orc_equilibrium_adv(double s, double ux, double uy, double geq[5])
{
    geq[1] = 0.5 * s * (CS2 + ux * ux + ux);
    geq[3] = 0.5 * s * (CS2 + ux * ux - ux);
    geq[2] = 0.5 * s * (CS2 + uy * uy + uy);
    geq[4] = 0.5 * s * (CS2 + uy * uy - uy);
    geq[0] = s - (geq[1] + geq[2] + geq[3] + geq[4]);
}

/* ------------------------------------------------------------------------ */
/* Raw moments, eq. (15) and eq. (32)/(44). */
static double raw9(const double f[9], int m, int n)
{
    double r = 0.0;
    for (int a = 0; a < 9; ++a) r += f[a] * ipow(EX9[a], m) * ipow(EY9[a], n);
    return r;
}

static double raw5(const double g[5], int m, int n)
{
    double r = 0.0;
    for (int a = 0; a < 5; ++a) r += g[a] * ipow(EX5[a], m) * ipow(EY5[a], n);
    return r;
}

/* Orthogonal basis vectors K_0..K_8 of eq. (12), component a. */
static double K9(int beta, int a)
{
    const double ex = EX9[a], ey = EY9[a];
    switch (beta) {
    case 0: return 1.0;
    case 1: return ex;
    case 2: return ey;
    case 3: return 3.0 * (ex * ex + ey * ey) - 4.0;
    case 4: return ex * ex - ey * ey;
    case 5: return ex * ey;
    case 6: return -3.0 * ex * ex * ey + 2.0 * ey;
    case 7: return -3.0 * ex * ey * ey + 2.0 * ex;
    default: return 9.0 * ex * ex * ey * ey - 6.0 * (ex * ex + ey * ey) + 4.0;
    }
}

/* Orthogonal basis vectors L_0..L_4 of eq. (29), component a. */
static double L5(int beta, int a)
{
    const double ex = EX5[a], ey = EY5[a];
    switch (beta) {
    case 0: return 1.0;
    case 1: return ex;
    case 2: return ey;
    case 3: return 5.0 * (ex * ex + ey * ey) - 4.0;
    default: return ex * ex - ey * ey;
    }
}

void orc_collide_f(const double f[9], double rho, double ux, double uy,
                   double MA, double Fx, double Fy, const double om[9],
                   double fp[9])
{
    const double kxx = raw9(f, 2, 0), kyy = raw9(f, 0, 2), kxy = raw9(f, 1, 1);
    const double kxxy = raw9(f, 2, 1), kxyy = raw9(f, 1, 2), kxxyy = raw9(f, 2, 2);
    const double ux2 = ux * ux, uy2 = uy * uy;
    double p[9];
    /* eq. (26): zeroth and first moment changes carry the whole source. */
    p[0] = MA / 9.0;
    p[1] = Fx / 6.0;
    p[2] = Fy / 6.0;
    /* eq. (17): cascaded changes of the non-conserved moments. */
    p[3] = om[3] / 12.0 * (2.0 * CS2 * rho + rho * (ux2 + uy2) - (kxx + kyy));
    p[4] = om[4] / 4.0 * (rho * (ux2 - uy2) - (kxx - kyy));
    p[5] = om[5] / 4.0 * (rho * ux * uy - kxy);
    p[6] = om[6] / 4.0 * (2.0 * rho * ux2 * uy + kxxy - 2.0 * ux * kxy - uy * kxx)
           - 0.5 * uy * (3.0 * p[3] + p[4]) - 2.0 * ux * p[5];
    p[7] = om[7] / 4.0 * (2.0 * rho * ux * uy2 + kxyy - 2.0 * uy * kxy - ux * kyy)
           - 0.5 * ux * (3.0 * p[3] - p[4]) - 2.0 * uy * p[5];
    p[8] = om[8] / 4.0 * (CS2 * CS2 * rho + 3.0 * rho * ux2 * uy2
                          - (kxxyy - 2.0 * ux * kxyy - 2.0 * uy * kxxy + ux2 * kyy
                             + uy2 * kxx + 4.0 * ux * uy * kxy))
           - 2.0 * p[3] - 0.5 * uy2 * (3.0 * p[3] + p[4]) - 0.5 * ux2 * (3.0 * p[3] - p[4])
           - 4.0 * ux * uy * p[5] - 2.0 * uy * p[6] - 2.0 * ux * p[7];
    /* eq. (16a): f^p = f + K p. */
    for (int a = 0; a < 9; ++a) {
        double d = 0.0;
        for (int beta = 0; beta < 9; ++beta) d += K9(beta, a) * p[beta];
        fp[a] = f[a] + d;
    }
}

void orc_collide_adv(const double g[5], double s, double ux, double uy,
                     double S, const double om[5], double gp[5])
{
    const double kx = raw5(g, 1, 0), ky = raw5(g, 0, 1);
    const double kxx = raw5(g, 2, 0), kyy = raw5(g, 0, 2);
    double q[5];
    /* eq. (41)/(51): the zeroth moment change carries the whole source. */
    q[0] = S / 5.0;
    /* eq. (34)/(49), first-order moments. */
    q[1] = om[1] / 2.0 * (s * ux - kx);
    q[2] = om[2] / 2.0 * (s * uy - ky);
    /* eq. (34)/(49), second-order moments.  Reading: relaxing the central
     * moments of eq. (31)/(43) to their Maxwellian values (trace 2 cs2 s,
     * deviator 0) yields a MINUS sign in front of (ux^2 + uy^2) s and
     * (ux^2 - uy^2) s and a factor s on 2 cs2; the printed plus signs would
     * not keep the equilibrium fixed. */
    q[3] = om[3] / 4.0 * (2.0 * CS2 * s - (kxx + kyy) + 2.0 * (ux * kx + uy * ky)
                          - (ux * ux + uy * uy) * s)
           + ux * q[1] + uy * q[2];
    q[4] = om[4] / 4.0 * (-(kxx - kyy) + 2.0 * (ux * kx - uy * ky)
                          - (ux * ux - uy * uy) * s)
           + ux * q[1] - uy * q[2];
    /* eq. (33a)/(46a): g^p = g + L q. */
    for (int a = 0; a < 5; ++a) {
        double d = 0.0;
        for (int beta = 0; beta < 5; ++beta) d += L5(beta, a) * q[beta];
        gp[a] = g[a] + d;
    }
}

/* ------------------------------------------------------------------------ */
/* Boundary values of the wall scalar for g (psi_w = rho_0 u_theta,w with
 * rho_0 = 1) and h (T_w).  ym is the radius of the point where the link
 * crosses the wall. */
static double wall_scalar(const orc_bc *bc, double ym)
{
    if (bc->kind == ORC_DIRICHLET) return bc->value + bc->slope * ym;
    if (bc->kind == ORC_OMEGA_R) return bc->value * ym;
    return 0.0; /* NOSLIP: a wall at rest */
}

/* Post-stream population q of distribution fld at node (i, j): the pull
 * form of eq. (16b), (33b), (46b).  Where the source node x - e_q is not a
 * fluid node, the boundary rules apply, in this precedence per link:
 *   1. a wall (radial faces first, then axial faces):
 *      f: half-way bounce-back (no-slip, Section 3.2).  Reading for a wall
 *      that imposes a normal velocity u_w (an inlet or outlet, which the
 *      paper's cases do not use): the moving-wall form of bounce-back,
 *      post[opp] + 2 w_q rho_0 (e_q . u_w) / c_s^2 with rho_0 = 1, which
 *      carries the mass flux rho_0 u_w through the wall;
 *      g, h: Reading of the cited advection-diffusion wall scheme: half-way
 *      anti-bounce-back for an imposed value, -post[opp] + 2 g^eq+_q(s_w,
 *      u_w), twice the even part of the D2Q5 equilibrium at the wall value,
 *      s_w (c_s^2 + u_n^2) for the one link that crosses the wall (u_n the
 *      normal velocity, 0 at a wall at rest, where this is 2 w s_w with
 *      w = 1/6), and bounce-back for zero flux (ADIABATIC);
 *   2. the symmetry axis (Section 3.3, "mirror"): specular reflection, the
 *      population comes from the node shifted by e_x along the axis with
 *      its radial velocity reversed; g is odd there (u_theta = 0 on the
 *      axis) and takes a minus sign;
 *   3. a free surface on an axial face (SLIP, Section 3.6: u_z = 0 and no
 *      shear): specular reflection, from the node shifted by e_y along the
 *      surface with the axial velocity reversed;
 *   4. periodic wrap along the axis.
 * On an axial face split into two parts, a link takes the rule of the part
 * where it crosses the face. */
static double pulled(const orc_state *s, int fld, int q, int i, int j)
{
    const orc_params *p = &s->p;
    const int nq = fld == ORC_FLOW ? 9 : 5;
    const int *ex = fld == ORC_FLOW ? EX9 : EX5;
    const int *ey = fld == ORC_FLOW ? EY9 : EY5;
    const double *post = fld == ORC_FLOW ? s->f : (fld == ORC_SWIRL ? s->g : s->h);

    int si = i - ex[q], sj = j - ey[q], qs = q;
    double sign = 1.0;
    const int fy = sj < 0 ? ORC_R_IN : (sj >= p->Nr ? ORC_R_OUT : -1);
    const int fx = si < 0 ? ORC_Z_LO : (si >= p->Nz ? ORC_Z_HI : -1);

    /* an axial face's rule is the one of the column where the link crosses */
    const int c2 = 2 * j - ey[q];
    int wall = -1;
    if (fy >= 0 && is_wall(p->bc[fy][fld].kind)) wall = fy;
    else if (fx >= 0 && is_wall(rule(p, fx, fld, c2)->kind)) wall = fx;
    if (wall >= 0) {
        const orc_bc *bc = rule(p, wall, fld, c2);
        const double own = post[node(s, i, j) * nq + opposite(ex, ey, nq, q)];
        const double un = normal_velocity(rule(p, wall, ORC_FLOW, c2));
        if (fld == ORC_FLOW) {
            const double w = phi1d(ex[q], 0.0) * phi1d(ey[q], 0.0); /* lattice weight */
            const double eu = wall <= ORC_R_OUT ? ey[q] * un : ex[q] * un;
            return own + 2.0 * w * eu / CS2;
        }
        if (bc->kind == ORC_ADIABATIC) return own;
        const double ym = y_of(s, j) - 0.5 * ey[q];
        return -own + (CS2 + un * un) * wall_scalar(bc, ym);
    }
    if (fy == ORC_R_IN && p->bc[ORC_R_IN][fld].kind == ORC_MIRROR) {
        qs = reflect_y(ex, ey, nq, q);
        sj = j;
        if (fld == ORC_SWIRL) sign = -1.0;
    }
    if (fx >= 0 && rule(p, fx, fld, c2)->kind == ORC_SLIP) {
        /* free surface: specular reflection, the population comes from the
         * node shifted by e_y along the surface with its axial velocity
         * reversed (after the axis reflection, if the link crosses both) */
        qs = reflect_x(ex, ey, nq, qs);
        si = i;
    }
    if (fx >= 0) si = (si + p->Nz) % p->Nz; /* periodic (walls handled above) */
    return sign * post[node(s, si, sj) * nq + qs];
}

/* ------------------------------------------------------------------------ */
/* Neighbour value of a derivative variable for the central differences of
 * the source terms (Section 3.2: central differences).  Reading: outside
 * the fluid the value comes from a ghost point mirrored through the wall,
 * q_g = 2 q_w - q_1 (q_1 = value at the boundary node), i.e. -q_1 for the
 * meridian velocities at a no-slip wall, 2 q_w - q_1 for an imposed u_theta
 * or T, q_1 for zero flux, and 2 u_w - q_1 for the normal velocity at a wall
 * that imposes one; at the axis even variables (u_x, T) take q_1 and odd
 * ones (u_y, u_theta) take -q_1; at a free surface u_x takes -q_1 and u_y
 * q_1; a periodic face wraps. */
static double neighbour(const orc_state *s, const double *F, int v, int i, int j,
                        int di, int dj)
{
    const orc_params *p = &s->p;
    const int ni = i + di, nj = j + dj;
    const double q1 = F[node(s, i, j) * 4 + v];
    int face = -1;
    if (nj < 0) face = ORC_R_IN;
    else if (nj >= p->Nr) face = ORC_R_OUT;
    else if (ni < 0) face = ORC_Z_LO;
    else if (ni >= p->Nz) face = ORC_Z_HI;
    if (face < 0) return F[node(s, ni, nj) * 4 + v];

    const int fld = (v == VX || v == VY) ? ORC_FLOW : (v == VT ? ORC_SWIRL : ORC_THERMAL);
    const orc_bc *bc = rule(p, face, fld, 2 * j);
    if (bc->kind == ORC_PERIODIC) return F[node(s, (ni + p->Nz) % p->Nz, nj) * 4 + v];
    if (bc->kind == ORC_MIRROR) return (v == VX || v == VP) ? q1 : -q1;
    if (bc->kind == ORC_ADIABATIC) return q1;
    if (bc->kind == ORC_SLIP) return v == VX ? -q1 : q1; /* u_x = 0, d_x u_y = 0 */
    if (v == VX || v == VY) {
        const int normal = face <= ORC_R_OUT ? VY : VX;
        return v == normal ? 2.0 * normal_velocity(bc) - q1 : -q1;
    }
    const double yw = y_of(s, j) + 0.5 * dj; /* wall radius, or y_j on an axial face */
    return 2.0 * wall_scalar(bc, yw) - q1;
}

/* ------------------------------------------------------------------------ */
/* Pass 1 for every node: post-stream populations (fs, gs, hs) and the
 * output moments rho^o, j^o (eq. 18), psi^o (eq. 35), phi^o (eq. 47).
 * mom[node][5] = rho^o, jx^o, jy^o, psi^o, phi^o; cur[node][4] = u_x^o,
 * u_y^o, u_theta^o = psi^o/rho^o, phi^o (the differentiated fields). */
static void stream_and_moments(const orc_state *s, double *fs, double *gs, double *hs,
                               double *mom, double *cur)
{
    const int Nr = s->p.Nr, Nz = s->p.Nz;
    /* every node writes only its own entries: rows may run on any thread */
#pragma omp parallel for schedule(static)
    for (int i = 0; i < Nz; ++i)
        for (int j = 0; j < Nr; ++j) {
            const int n = node(s, i, j);
            double rho = 0, jx = 0, jy = 0, psi = 0, phi = 0;
            for (int a = 0; a < 9; ++a) {
                const double v = pulled(s, ORC_FLOW, a, i, j);
                fs[n * 9 + a] = v;
                rho += v;
                jx += v * EX9[a];
                jy += v * EY9[a];
            }
            for (int a = 0; a < 5; ++a) {
                const double vg = pulled(s, ORC_SWIRL, a, i, j);
                const double vh = pulled(s, ORC_THERMAL, a, i, j);
                gs[n * 5 + a] = vg;
                hs[n * 5 + a] = vh;
                psi += vg;
                phi += vh;
            }
            double *m = mom + n * 5;
            m[0] = rho; m[1] = jx; m[2] = jy; m[3] = psi; m[4] = phi;
            double *c = cur + n * 4;
            c[VX] = jx / rho; c[VY] = jy / rho; c[VT] = psi / rho; c[VP] = phi;
        }
}

typedef struct {
    double MA, Fx, Fy, Spsi, Sphi;   /* geometric sources + body force      */
    double rho, ux, uy, psi, phi;    /* fields after the pre-collision half  */
} half_step;

/* Geometric sources and body force (eq. 4a-4c, 5, 7, 9) at the state
 * (rho, Jx = rho u_x, Jy = rho u_y, psi, phi) of a node at radius y, with
 * mu = rho nu and the central differences d[] = {d_x u_y, d_y u_x, d_y u_y,
 * d_y u_theta, d_y phi}.  Body force (Section 3.2, Boussinesq):
 * F^b_x = rho_0 [g + g beta (phi - T0)] with rho_0 = 1, F^b_y = 0. */
static void sources_at(const orc_params *p, double y, double rho, double Jx, double Jy,
                       double psi, double phi, const double d[5], half_step *o)
{
    const double ux = Jx / rho, uy = Jy / rho, nu = p->nu, mu = rho * nu;
    o->MA = -rho * uy / y;                                           /* (4a) */
    const double FAx = -rho * ux * uy / y + mu * (d[0] + d[1]) / y;  /* (4b) */
    const double FAy = psi * psi / (rho * y) - rho * uy * uy / y     /* (4c) */
                       + 2.0 * mu * d[2] / y - 2.0 * mu * uy / (y * y);
    o->Fx = FAx + (p->g_axial + p->gbeta * (phi - p->T0));          /* (5)  */
    o->Fy = FAy;
    o->Spsi = -2.0 * uy * psi / y + mu * d[3] / y - nu * psi / (y * y); /* (7) */
    o->Sphi = -uy * phi / y + p->alpha * d[4] / y;                   /* (9)  */
}

/* Pre-collision half source step (eq. 21a-21c, 38, 48) for node (i, j):
 *   rho = rho^o + M^A/2, rho u = j^o + F/2, psi = psi^o + S_psi/2,
 *   phi = phi^o + S_phi/2,
 * with the central differences of the fields in D (Section 3.2).
 * Reading: the sources are functions of the state they act on, evaluated
 * at that pre-collision (half-step) state, so the five relations above are
 * solved together (the implicit midpoint of each half step; it keeps the
 * split second order and lets a steady swirling flow conserve mass).  The
 * solve moves the terms that are linear in the unknowns to the left and
 * iterates on the rest, which couple only through u/y and u_theta/y; it
 * stops when the update is at round-off, and the returned state is then
 * re-formed from the sources evaluated at it, so that eq. (21), (38), (48)
 * hold with exactly the sources that the collision receives. */
static void half_step_solve(const orc_params *p, double y, const double m[5], const double d[5],
                            half_step *o)
{
    const double ro = m[0], jxo = m[1], jyo = m[2], pso = m[3], pho = m[4];
    const double nu = p->nu;

    double rho = ro, Jy = jyo, psi = pso;
    for (int it = 0; it < 200; ++it) {
        const double rho1 = ro - 0.5 * Jy / y;
        const double psi1 = (pso + 0.5 * rho1 * nu * d[3] / y)
                            / (1.0 + Jy / (rho1 * y) + 0.5 * nu / (y * y));
        const double Jy1 = (jyo + 0.5 * (psi1 * psi1 / (rho1 * y) - Jy * Jy / (rho1 * y)
                                         + 2.0 * rho1 * nu * d[2] / y))
                           / (1.0 + nu / (y * y));
        const double change = fabs(rho1 - rho) + fabs(psi1 - psi) + fabs(Jy1 - Jy);
        rho = rho1; psi = psi1; Jy = Jy1;
        if (change <= 1e-17 * (fabs(rho) + fabs(psi) + fabs(Jy))) break;
    }
    const double phi = (pho + 0.5 * p->alpha * d[4] / y) / (1.0 + 0.5 * Jy / (rho * y));
    const double Jx = (jxo + 0.5 * (rho * nu * (d[0] + d[1]) / y + p->g_axial
                                    + p->gbeta * (phi - p->T0)))
                      / (1.0 + 0.5 * Jy / (rho * y));

    sources_at(p, y, rho, Jx, Jy, psi, phi, d, o);
    o->rho = ro + 0.5 * o->MA;
    o->ux = (jxo + 0.5 * o->Fx) / o->rho;
    o->uy = (jyo + 0.5 * o->Fy) / o->rho;
    o->psi = pso + 0.5 * o->Spsi;
    o->phi = pho + 0.5 * o->Sphi;
}

/* The half step of node (i, j): its output moments and the central
 * differences (Section 3.2) of the fields in D. */
static void sources_half_step(const orc_state *s, int i, int j, const double *mom,
                              const double *D, half_step *o)
{
    double d[5];
    d[0] = 0.5 * (neighbour(s, D, VY, i, j, +1, 0) - neighbour(s, D, VY, i, j, -1, 0));
    d[1] = 0.5 * (neighbour(s, D, VX, i, j, 0, +1) - neighbour(s, D, VX, i, j, 0, -1));
    d[2] = 0.5 * (neighbour(s, D, VY, i, j, 0, +1) - neighbour(s, D, VY, i, j, 0, -1));
    d[3] = 0.5 * (neighbour(s, D, VT, i, j, 0, +1) - neighbour(s, D, VT, i, j, 0, -1));
    d[4] = 0.5 * (neighbour(s, D, VP, i, j, 0, +1) - neighbour(s, D, VP, i, j, 0, -1));
    half_step_solve(&s->p, y_of(s, j), mom + node(s, i, j) * 5, d, o);
}

void orc_half_step(const orc_params *p, double y, const double mom[5], const double d[5],
                   double out[10])
{
    half_step o;
    half_step_solve(p, y, mom, d, &o);
    out[0] = o.MA; out[1] = o.Fx; out[2] = o.Fy; out[3] = o.Spsi; out[4] = o.Sphi;
    out[5] = o.rho; out[6] = o.ux; out[7] = o.uy; out[8] = o.psi; out[9] = o.phi;
}

static void omegas(const orc_params *p, double om9[9], double omg[5], double omh[5])
{
    for (int k = 0; k < 9; ++k) om9[k] = 0.0;
    om9[3] = p->omega3;
    om9[4] = om9[5] = rate_for(p->nu);
    om9[6] = p->omega6; om9[7] = p->omega7; om9[8] = p->omega8;
    omg[0] = 0.0;
    omg[1] = omg[2] = rate_for(p->nu);  /* D_psi = nu */
    omg[3] = p->omega_psi3; omg[4] = p->omega_psi4;
    omh[0] = 0.0;
    omh[1] = omh[2] = rate_for(p->alpha);
    omh[3] = p->omega_phi3; omh[4] = p->omega_phi4;
}

void orc_step(orc_state *s, long n)
{
    const int Nr = s->p.Nr, Nz = s->p.Nz, N = Nr * Nz;
    double *fs = malloc(sizeof(double) * 9 * N), *gs = malloc(sizeof(double) * 5 * N);
    double *hs = malloc(sizeof(double) * 5 * N), *mom = malloc(sizeof(double) * 5 * N);
    double *cur = malloc(sizeof(double) * 4 * N);
    double *fn = malloc(sizeof(double) * 9 * N), *gn = malloc(sizeof(double) * 5 * N);
    double *hn = malloc(sizeof(double) * 5 * N), *nlag = malloc(sizeof(double) * 4 * N);
    double om9[9], omg[5], omh[5];
    omegas(&s->p, om9, omg, omh);

    for (long t = 0; t < n; ++t) {
        /* pass 1: the streaming step S and the output moments */
        stream_and_moments(s, fs, gs, hs, mom, cur);
        const double *D = s->p.deriv_mode == ORC_DERIV_CURRENT ? cur : s->lag;
        /* pass 2: M^1/2 F^1/2 C F^1/2 M^1/2 (eq. 20) and R^1/2 C R^1/2
         * (eq. 37, 45), written as pre-half step + collision with the full
         * source moment (eq. 23, 40); nodes are independent */
#pragma omp parallel for schedule(static)
        for (int i = 0; i < Nz; ++i)
            for (int j = 0; j < Nr; ++j) {
                const int k = node(s, i, j);
                half_step hs1;
                sources_half_step(s, i, j, mom, D, &hs1);
                nlag[4 * k + VX] = hs1.ux;
                nlag[4 * k + VY] = hs1.uy;
                nlag[4 * k + VT] = hs1.psi / hs1.rho;
                nlag[4 * k + VP] = hs1.phi;
                orc_collide_f(fs + 9 * k, hs1.rho, hs1.ux, hs1.uy, hs1.MA, hs1.Fx, hs1.Fy,
                              om9, fn + 9 * k);
                orc_collide_adv(gs + 5 * k, hs1.psi, hs1.ux, hs1.uy, hs1.Spsi, omg, gn + 5 * k);
                orc_collide_adv(hs + 5 * k, hs1.phi, hs1.ux, hs1.uy, hs1.Sphi, omh, hn + 5 * k);
            }
        double *tmp;
        tmp = s->f; s->f = fn; fn = tmp;
        tmp = s->g; s->g = gn; gn = tmp;
        tmp = s->h; s->h = hn; hn = tmp;
        tmp = s->lag; s->lag = nlag; nlag = tmp;
        s->steps += 1;
    }
    free(fs); free(gs); free(hs); free(mom); free(cur); free(fn); free(gn); free(hn);
    free(nlag);
}

void orc_fields(const orc_state *s, double *rho, double *ur, double *uz, double *uth,
                double *T)
{
    const int Nr = s->p.Nr, Nz = s->p.Nz, N = Nr * Nz;
    double *fs = malloc(sizeof(double) * 9 * N), *gs = malloc(sizeof(double) * 5 * N);
    double *hs = malloc(sizeof(double) * 5 * N), *mom = malloc(sizeof(double) * 5 * N);
    double *cur = malloc(sizeof(double) * 4 * N);
    stream_and_moments(s, fs, gs, hs, mom, cur);
    const double *D = s->p.deriv_mode == ORC_DERIV_CURRENT ? cur : s->lag;
#pragma omp parallel for schedule(static)
    for (int i = 0; i < Nz; ++i)
        for (int j = 0; j < Nr; ++j) {
            const int k = node(s, i, j);
            half_step o;
            sources_half_step(s, i, j, mom, D, &o);
            if (rho) rho[k] = o.rho;
            if (ur) ur[k] = o.uy;
            if (uz) uz[k] = o.ux;
            if (uth) uth[k] = o.psi / o.rho;
            if (T) T[k] = o.phi;
        }
    free(fs); free(gs); free(hs); free(mom); free(cur);
}

/* Wall heat-transfer numbers (Section 3.2): Nu_i = -R_i/(H dT) int d_yT dx at
 * the inner wall, Nu_o likewise at R_o.  Reading: the wall gradient of a
 * half-way wall is the second-order one-sided value (-8 T_w + 9 T_1 - T_2)/3
 * along the inward normal, and the integral is the midpoint sum over the Nz
 * rows (H = Nz).  For a cylinder the same construction on the lids gives the
 * area-weighted mean axial gradient, Nu = (H/dT) (2/R^2) sum_j y_j dT/dn. */
void orc_nusselt(const orc_state *s, double *nu_a, double *nu_b, double *mean)
{
    const orc_params *p = &s->p;
    const int Nr = p->Nr, Nz = p->Nz;
    double *T = malloc(sizeof(double) * Nr * Nz);
    orc_fields(s, NULL, NULL, NULL, NULL, T);
    double a = 0.0, b = 0.0;
    if (!p->cylinder) {
        const double Ta = p->bc[ORC_R_IN][ORC_THERMAL].value;
        const double Tb = p->bc[ORC_R_OUT][ORC_THERMAL].value;
        const double dT = Ta - Tb;
        const double Ri = p->r_inner, Ro = p->r_inner + Nr;
        double sa = 0.0, sb = 0.0;
        for (int i = 0; i < Nz; ++i) {
            /* d_y T at y = R_i (inward normal = +y) */
            sa += (-8.0 * Ta + 9.0 * T[node(s, i, 0)] - T[node(s, i, 1)]) / 3.0;
            /* d_y T at y = R_o (inward normal = -y) */
            sb += -(-8.0 * Tb + 9.0 * T[node(s, i, Nr - 1)] - T[node(s, i, Nr - 2)]) / 3.0;
        }
        a = -Ri / (Nz * dT) * sa;
        b = -Ro / (Nz * dT) * sb;
    } else if (p->split[0] || p->split[1] || p->bc[ORC_Z_LO][ORC_THERMAL].slope != 0.0 ||
               p->bc[ORC_Z_HI][ORC_THERMAL].slope != 0.0) {
        /* lids of more than one temperature: no Nusselt number is defined */
        a = b = NAN;
    } else {
        const double Ta = p->bc[ORC_Z_LO][ORC_THERMAL].value;
        const double Tb = p->bc[ORC_Z_HI][ORC_THERMAL].value;
        const double dT = Tb - Ta, R = Nr, H = Nz;
        double sa = 0.0, sb = 0.0;
        for (int j = 0; j < Nr; ++j) {
            const double y = y_of(s, j);
            /* d_x T at the bottom lid (inward normal = +x) */
            sa += y * (-8.0 * Ta + 9.0 * T[node(s, 0, j)] - T[node(s, 1, j)]) / 3.0;
            /* d_x T at the top lid (inward normal = -x) */
            sb += y * -(-8.0 * Tb + 9.0 * T[node(s, Nz - 1, j)] - T[node(s, Nz - 2, j)]) / 3.0;
        }
        a = H / dT * 2.0 / (R * R) * sa;
        b = H / dT * 2.0 / (R * R) * sb;
    }
    free(T);
    if (nu_a) *nu_a = a;
    if (nu_b) *nu_b = b;
    if (mean) *mean = 0.5 * (a + b);
}

/* Stream function of the meridian flow (Section 3.6): d psi / d y = -y u_x,
 * integrated outward from the inner face by the midpoint rule over the node
 * cells. */
void orc_stream_function(const orc_state *s, double *psi, double *lo, double *hi)
{
    const int Nr = s->p.Nr, Nz = s->p.Nz;
    double *ux = malloc(sizeof(double) * Nr * Nz);
    orc_fields(s, NULL, NULL, ux, NULL, NULL);
    double a = 0.0, b = 0.0;
    for (int i = 0; i < Nz; ++i) {
        double acc = 0.0;
        for (int j = 0; j < Nr; ++j) {
            acc -= y_of(s, j) * ux[node(s, i, j)];
            if (psi) psi[node(s, i, j)] = acc;
            if (acc < a) a = acc;
            if (acc > b) b = acc;
        }
    }
    free(ux);
    if (lo) *lo = a;
    if (hi) *hi = b;
}

/* ------------------------------------------------------------------------ */
/* A rule that the distribution may take on the face. */
static int rule_ok(const orc_bc *bc, int face, int fld)
{
    const int k = bc->kind;
    if (face >= ORC_Z_LO && k == ORC_MIRROR) return 0;
    if (fld == ORC_FLOW && is_wall(k) && k != ORC_NOSLIP && k != ORC_VELOCITY) return 0;
    if (fld != ORC_FLOW && (k == ORC_VELOCITY || k == ORC_SLIP)) return 0;
    if (k == ORC_SLIP && face < ORC_Z_LO) return 0;
    if (fld == ORC_THERMAL && (k == ORC_NOSLIP || k == ORC_OMEGA_R)) return 0;
    if (k < 0 || k > ORC_SLIP || k == 6) return 0;
    if (!isfinite(bc->slope)) return 0;
    if (bc->slope != 0.0 && !(k == ORC_DIRICHLET && face >= ORC_Z_LO)) return 0;
    return 1;
}

/* The three rules of one face (or face part) agree on what the face is. */
static int face_ok(const orc_bc b[3])
{
    const int w = is_wall(b[0].kind) || b[0].kind == ORC_SLIP;
    if (is_wall(b[1].kind) != w || is_wall(b[2].kind) != w) return 0;
    if (b[0].kind == ORC_VELOCITY &&
        (b[1].kind == ORC_ADIABATIC || b[2].kind != ORC_DIRICHLET || !isfinite(b[0].value)))
        return 0;
    return 1;
}

static int valid(const orc_params *p)
{
    if (p->Nr < 2 || p->Nz < 1) return 0;
    if (!(p->nu > 0) || !(p->alpha > 0)) return 0;
    if (!p->cylinder && !(p->r_inner > 0)) return 0;
    for (int fld = 0; fld < 3; ++fld) {
        const int zp_lo = p->bc[ORC_Z_LO][fld].kind == ORC_PERIODIC;
        const int zp_hi = p->bc[ORC_Z_HI][fld].kind == ORC_PERIODIC;
        if (zp_lo != zp_hi) return 0;
        if (!zp_lo && p->Nz < 2) return 0;
        /* a cylinder has the axis at its inner face; an annulus may carry a
         * mirror (symmetry plane) there as well */
        const int ax = p->bc[ORC_R_IN][fld].kind == ORC_MIRROR;
        if (p->cylinder && !ax) return 0;
        if (p->bc[ORC_R_OUT][fld].kind == ORC_MIRROR || p->bc[ORC_R_OUT][fld].kind == ORC_PERIODIC ||
            p->bc[ORC_R_IN][fld].kind == ORC_PERIODIC)
            return 0;
        for (int face = 0; face < 4; ++face) {
            if (!rule_ok(&p->bc[face][fld], face, fld)) return 0;
            if (face >= ORC_Z_LO && p->split[face - ORC_Z_LO] != 0 &&
                !rule_ok(&p->outer[face - ORC_Z_LO][fld], face, fld))
                return 0;
        }
    }
    /* a face is a wall (or a free surface) for all three distributions or
     * for none; where fluid crosses it (VELOCITY), g and h carry imposed
     * values */
    for (int face = 0; face < 4; ++face) {
        if (!face_ok(p->bc[face])) return 0;
        if (face < ORC_Z_LO) continue;
        const int sp = p->split[face - ORC_Z_LO];
        if (sp == 0) continue;
        /* a split face is solid or free surface in both parts, with no
         * fluid crossing it */
        if (sp < 1 || sp > p->Nr - 1 || !face_ok(p->outer[face - ORC_Z_LO])) return 0;
        for (int fld = 0; fld < 3; ++fld) {
            const int a = p->bc[face][fld].kind, b = p->outer[face - ORC_Z_LO][fld].kind;
            if (!(is_wall(a) || a == ORC_SLIP) || !(is_wall(b) || b == ORC_SLIP)) return 0;
            if (a == ORC_VELOCITY || b == ORC_VELOCITY) return 0;
        }
    }
    return 1;
}

orc_state *orc_create(const orc_params *p, const double *rho, const double *ur,
                      const double *uz, const double *uth, const double *T)
{
    if (!valid(p)) return NULL;
    orc_state *s = calloc(1, sizeof(orc_state));
    s->p = *p;
    const int N = p->Nr * p->Nz;
    s->f = malloc(sizeof(double) * 9 * N);
    s->g = malloc(sizeof(double) * 5 * N);
    s->h = malloc(sizeof(double) * 5 * N);
    s->lag = malloc(sizeof(double) * 4 * N);
    for (int k = 0; k < N; ++k) {
        const double r = rho ? rho[k] : 1.0;
        const double vx = uz ? uz[k] : 0.0, vy = ur ? ur[k] : 0.0;
        const double vt = uth ? uth[k] : 0.0, t = T ? T[k] : 0.0;
        orc_equilibrium_f(r, vx, vy, s->f + 9 * k);
        orc_equilibrium_adv(r * vt, vx, vy, s->g + 5 * k);
        orc_equilibrium_adv(t, vx, vy, s->h + 5 * k);
        /* the lagged fields start as the initial fields */
        s->lag[4 * k + VX] = vx;
        s->lag[4 * k + VY] = vy;
        s->lag[4 * k + VT] = vt;
        s->lag[4 * k + VP] = t;
    }
    return s;
}

void orc_destroy(orc_state *s)
{
    if (!s) return;
    free(s->f); free(s->g); free(s->h); free(s->lag); free(s);
}

long orc_steps_done(const orc_state *s) { return s->steps; }

int orc_all_finite(const orc_state *s)
{
    const long N = (long)s->p.Nr * s->p.Nz;
    for (long k = 0; k < 9 * N; ++k) if (!isfinite(s->f[k])) return 0;
    for (long k = 0; k < 5 * N; ++k) if (!isfinite(s->g[k]) || !isfinite(s->h[k])) return 0;
    return 1;
}

long orc_state_len(const orc_state *s) { return 23L * s->p.Nr * s->p.Nz; }

void orc_get_state(const orc_state *s, double *out)
{
    const long N = (long)s->p.Nr * s->p.Nz;
    memcpy(out, s->f, sizeof(double) * 9 * N);
    memcpy(out + 9 * N, s->g, sizeof(double) * 5 * N);
    memcpy(out + 14 * N, s->h, sizeof(double) * 5 * N);
    memcpy(out + 19 * N, s->lag, sizeof(double) * 4 * N);
}

void orc_set_state(orc_state *s, const double *in, long steps_done)
{
    const long N = (long)s->p.Nr * s->p.Nz;
    memcpy(s->f, in, sizeof(double) * 9 * N);
    memcpy(s->g, in + 9 * N, sizeof(double) * 5 * N);
    memcpy(s->h, in + 14 * N, sizeof(double) * 5 * N);
    memcpy(s->lag, in + 19 * N, sizeof(double) * 4 * N);
    s->steps = steps_done;
}

void orc_get_populations(const orc_state *s, double *f9, double *g5, double *h5)
{
    const long N = (long)s->p.Nr * s->p.Nz;
    for (long k = 0; k < N; ++k) {
        for (int a = 0; a < 9; ++a) if (f9) f9[a * N + k] = s->f[9 * k + a];
        for (int a = 0; a < 5; ++a) {
            if (g5) g5[a * N + k] = s->g[5 * k + a];
            if (h5) h5[a * N + k] = s->h[5 * k + a];
        }
    }
}

/* ------------------------------------------------------------------------ */
/* Convergence residual.  Reading: the paper runs its cases "to steady state"
 * without defining the test, so the residual is the largest relative change
 * per step between two snapshots K steps apart,
 *   max over c in {u_r, u_z, u_theta} of ||c_now - c_then|| / (K ||speed_now||)
 *   and ||T_now - T_then|| / (K ||T_now||),
 * with ||.|| the Euclidean norm over the nodes and speed = |(u_r, u_z,
 * u_theta)|.  The velocity components share the speed norm because one of
 * them can be pure round-off (u_r of a parallel flow).  A term whose norm is
 * zero is skipped; K <= 0 gives +inf. */
double orc_residual(long n, const double *ur1, const double *uz1, const double *uth1,
                    const double *T1, const double *ur0, const double *uz0,
                    const double *uth0, const double *T0, long K)
{
    if (K <= 0) return INFINITY;
    const double *now[3] = {ur1, uz1, uth1}, *then[3] = {ur0, uz0, uth0};
    double speed2 = 0.0, d2[3] = {0.0, 0.0, 0.0}, t2 = 0.0, dt2 = 0.0;
    for (long k = 0; k < n; ++k) {
        for (int c = 0; c < 3; ++c) {
            speed2 += now[c][k] * now[c][k];
            d2[c] += (now[c][k] - then[c][k]) * (now[c][k] - then[c][k]);
        }
        t2 += T1[k] * T1[k];
        dt2 += (T1[k] - T0[k]) * (T1[k] - T0[k]);
    }
    double r = 0.0;
    if (speed2 > 0.0)
        for (int c = 0; c < 3; ++c) r = fmax(r, sqrt(d2[c]) / ((double)K * sqrt(speed2)));
    if (t2 > 0.0) r = fmax(r, sqrt(dt2) / ((double)K * sqrt(t2)));
    return r;
}

void orc_set_threads(int n)
{
#ifdef _OPENMP
    if (n > 0) omp_set_num_threads(n);
#else
    (void)n;
#endif
}

int orc_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}
