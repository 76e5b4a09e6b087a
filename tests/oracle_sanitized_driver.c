/*
 * Drives the oracle through every boundary kind and every entry point on
 * small lattices, for a build with the address and undefined-behaviour
 * sanitizers (tests/test_oracle_sanitized.py compiles and runs it; a
 * sanitizer report makes the run fail).  Exit status 0 when every lattice
 * stays finite.
 */
#include <math.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include "../oracle/oracle.h"

static void wall(orc_params *p, int face, int swirl_kind, double swirl, int t_kind, double t)
{
    p->bc[face][ORC_FLOW].kind = ORC_NOSLIP;
    p->bc[face][ORC_SWIRL].kind = swirl_kind;
    p->bc[face][ORC_SWIRL].value = swirl;
    p->bc[face][ORC_THERMAL].kind = t_kind;
    p->bc[face][ORC_THERMAL].value = t;
}

static orc_params base(int Nr, int Nz, int cylinder)
{
    orc_params p;
    memset(&p, 0, sizeof(p));
    p.Nr = Nr;
    p.Nz = Nz;
    p.cylinder = cylinder;
    p.r_inner = cylinder ? 0.0 : 5.0;
    p.nu = 0.05;
    p.alpha = 0.07;
    p.omega3 = p.omega6 = p.omega7 = p.omega8 = 1.0;
    p.omega_psi3 = p.omega_psi4 = p.omega_phi3 = p.omega_phi4 = 1.0;
    p.gbeta = 1e-4;
    p.T0 = 0.5;
    p.deriv_mode = ORC_DERIV_PREVIOUS;
    return p;
}

/* Steps a lattice and calls every query on it; returns 0 when finite. */
static int exercise(const orc_params *p, const char *name)
{
    const int N = p->Nr * p->Nz;
    double *f = calloc((size_t)N * 6, sizeof(double));
    double *rho = f, *ur = f + N, *uz = f + 2 * N, *uth = f + 3 * N, *T = f + 4 * N;
    double *psi = f + 5 * N;
    for (int k = 0; k < N; ++k) {
        rho[k] = 1.0;
        ur[k] = 1e-3 * sin(0.7 * k);
        uz[k] = 1e-3 * cos(0.3 * k);
        uth[k] = 1e-3 * sin(0.11 * k);
        T[k] = 0.5 + 0.1 * cos(0.5 * k);
    }
    orc_state *s = orc_create(p, rho, ur, uz, uth, T);
    if (!s) {
        printf("%s: rejected\n", name);
        free(f);
        return 1;
    }
    orc_step(s, 150);
    double *then = malloc(sizeof(double) * 4 * N);
    orc_fields(s, NULL, then, then + N, then + 2 * N, then + 3 * N);
    orc_step(s, 7);
    orc_fields(s, rho, ur, uz, uth, T);
    double a = 0.0, b = 0.0, m = 0.0, lo = 0.0, hi = 0.0;
    orc_nusselt(s, &a, &b, &m);
    orc_stream_function(s, psi, &lo, &hi);
    const double r = orc_residual(N, ur, uz, uth, T, then, then + N, then + 2 * N, then + 3 * N, 7);
    const long len = orc_state_len(s);
    double *st = malloc(sizeof(double) * (size_t)len);
    orc_get_state(s, st);
    orc_set_state(s, st, orc_steps_done(s));
    double *pops = malloc(sizeof(double) * 19 * N);
    orc_get_populations(s, pops, pops + 9 * N, pops + 14 * N);
    const int ok = orc_all_finite(s) && isfinite(r) && isfinite(lo) && isfinite(hi);
    printf("%s: %d x %d, finite %d, residual %.3e, psi %.3e .. %.3e\n", name, p->Nr, p->Nz, ok, r,
           lo, hi);
    orc_destroy(s);
    free(st);
    free(pops);
    free(then);
    free(f);
    return ok ? 0 : 1;
}

int main(void)
{
    int bad = 0;
    orc_set_threads(2);

    /* annulus: walls all round, imposed values, buoyancy */
    orc_params p = base(9, 7, 0);
    wall(&p, ORC_R_IN, ORC_DIRICHLET, 1e-3, ORC_DIRICHLET, 1.0);
    wall(&p, ORC_R_OUT, ORC_OMEGA_R, 1e-4, ORC_DIRICHLET, 0.0);
    wall(&p, ORC_Z_LO, ORC_NOSLIP, 0.0, ORC_ADIABATIC, 0.0);
    wall(&p, ORC_Z_HI, ORC_NOSLIP, 0.0, ORC_ADIABATIC, 0.0);
    bad |= exercise(&p, "annulus");

    /* one-row and one-column lattices */
    orc_params q = p;
    q.Nz = 2;
    bad |= exercise(&q, "two rows");
    q = p;
    q.Nr = 2;
    bad |= exercise(&q, "two columns");

    /* periodic z, current-step derivatives */
    q = p;
    for (int fld = 0; fld < 3; ++fld) {
        q.bc[ORC_Z_LO][fld].kind = ORC_PERIODIC;
        q.bc[ORC_Z_HI][fld].kind = ORC_PERIODIC;
    }
    q.Nz = 1;
    q.deriv_mode = ORC_DERIV_CURRENT;
    bad |= exercise(&q, "periodic, one row");

    /* cylinder: axis, lids, a split top with a free surface and sloped T */
    orc_params c = base(8, 6, 1);
    for (int fld = 0; fld < 3; ++fld) c.bc[ORC_R_IN][fld].kind = ORC_MIRROR;
    wall(&c, ORC_R_OUT, ORC_OMEGA_R, -1e-4, ORC_DIRICHLET, 1.0);
    wall(&c, ORC_Z_LO, ORC_OMEGA_R, -1e-4, ORC_ADIABATIC, 0.0);
    wall(&c, ORC_Z_HI, ORC_OMEGA_R, 2e-3, ORC_DIRICHLET, 0.0);
    c.split[1] = 3;
    c.outer[1][ORC_FLOW].kind = ORC_SLIP;
    c.outer[1][ORC_SWIRL].kind = ORC_ADIABATIC;
    c.outer[1][ORC_THERMAL].kind = ORC_DIRICHLET;
    c.outer[1][ORC_THERMAL].value = -0.6;
    c.outer[1][ORC_THERMAL].slope = 0.2;
    bad |= exercise(&c, "split lid");

    /* a whole free surface over a split bottom */
    orc_params d = c;
    d.split[1] = 0;
    d.bc[ORC_Z_HI][ORC_FLOW].kind = ORC_SLIP;
    d.bc[ORC_Z_HI][ORC_SWIRL].kind = ORC_ADIABATIC;
    d.split[0] = 5;
    d.outer[0][ORC_FLOW].kind = ORC_NOSLIP;
    d.outer[0][ORC_SWIRL].kind = ORC_DIRICHLET;
    d.outer[0][ORC_SWIRL].value = 1e-3;
    d.outer[0][ORC_THERMAL].kind = ORC_ADIABATIC;
    bad |= exercise(&d, "free surface");

    /* imposed-velocity walls (inflow through the bottom, outflow at the top) */
    orc_params v = base(7, 9, 1);
    for (int fld = 0; fld < 3; ++fld) v.bc[ORC_R_IN][fld].kind = ORC_MIRROR;
    wall(&v, ORC_R_OUT, ORC_NOSLIP, 0.0, ORC_DIRICHLET, 0.0);
    wall(&v, ORC_Z_LO, ORC_NOSLIP, 0.0, ORC_DIRICHLET, 1.0);
    wall(&v, ORC_Z_HI, ORC_NOSLIP, 0.0, ORC_DIRICHLET, 0.0);
    v.bc[ORC_Z_LO][ORC_FLOW].kind = ORC_VELOCITY;
    v.bc[ORC_Z_LO][ORC_FLOW].value = 5e-3;
    v.bc[ORC_Z_HI][ORC_FLOW].kind = ORC_VELOCITY;
    v.bc[ORC_Z_HI][ORC_FLOW].value = 5e-3;
    bad |= exercise(&v, "inlet and outlet");

    /* invalid parameters are rejected without touching memory */
    orc_params x = c;
    x.split[1] = 8;
    if (orc_create(&x, NULL, NULL, NULL, NULL, NULL) != NULL) bad = 1;

    /* the node-level operators */
    double feq[9], geq[5], fp[9], gp[5], out[10];
    const double om[9] = {1, 1, 1, 1, 1.2, 1.2, 1, 1, 1};
    orc_equilibrium_f(1.01, 1e-3, -2e-3, feq);
    orc_equilibrium_adv(0.3, 1e-3, -2e-3, geq);
    orc_collide_f(feq, 1.01, 1e-3, -2e-3, 1e-6, 1e-6, -1e-6, om, fp);
    orc_collide_adv(geq, 0.3, 1e-3, -2e-3, 1e-6, om, gp);
    const double mom[5] = {1.0, 1e-3, 2e-3, 1e-3, 0.4}, dd[5] = {1e-4, 2e-4, -1e-4, 3e-5, 1e-3};
    orc_half_step(&c, 2.5, mom, dd, out);
    for (int k = 0; k < 10; ++k) bad |= !isfinite(out[k]);
    printf("%s\n", bad ? "FAILED" : "ok");
    return bad;
}
