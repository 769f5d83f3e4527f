/*
 * fslbm_oracle.c -- plain, slow FP64 CPU reference of the free-surface lattice
 * Boltzmann (FSLBM) time step of Schwarzmeier & Ruede, "Comparison of refilling
 * schemes in the free-surface lattice Boltzmann method" (arXiv 2207.14496).
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the oracle that the GPU library is
 * checked against.  Only the test suite, the smoke check and the CPU-baseline
 * leg of the benchmark may load it.  It shares no code, header, table or helper
 * with the GPU library: every constant below is written out here from the
 * paper and from the textbook D3Q19 lattice.
 *
 * Style: scalar nested loops in the order the method is stated, two PDF arrays
 * (no in-place streaming), FP64 throughout, no blocking or fusion.  Build with
 * -O2 -ffp-contract=off so that no multiply-add is contracted.
 *
 * Canonical state (what a caller hands in and gets back):
 *   flag[n]    1 = liquid, 2 = interface, 4 = gas          (Sec. 2.2, cell types)
 *   f[i*N+n]   post-collision PDFs f*_i(x,t) of liquid and interface cells
 *   m[n]       interface-cell mass (Sec. 2.2, mass definition); 0 elsewhere
 *   phi[n]     fill level: liquid 1, gas 0, interface m/rho
 *   reservoir  excess mass that found no receiving interface cell
 * Cell n = (z*ny + y)*nx + x.  Domain walls sit half a cell outside the box on
 * every non-periodic axis (no-slip, bounce-back).
 *
 * Readings of passages the paper leaves open (numbered as in the design notes):
 *   R1  c_s^2 = 1/3 (the printed square root is a typo; p0 = c_s^2 rho0 = 1/3).
 *   R2  step order: S0 surface geometry, S1 stream + free-surface BC + mass
 *       exchange, S2 collide, S3 mark, S4 resolve conflicts, S5 refill,
 *       S6 apply conversions, S7 excess mass.
 *   R3  the interface velocity in the free-surface BC and the neighbour rho, u
 *       in the refilling schemes come from the stored post-collision PDFs:
 *       rho = sum f*, u = sum c f* / rho - g/2.
 *   R4  gas density rho_G = 3 (p_V + 2 sigma kappa_m), kappa_m = -div(n^)/2.
 *   R5  Parker-Youngs normal: 3x3x3 stencil, weights 4/2/1, divided by 32.
 *   R6  walls: a stencil pair (c, -c) touching a wall is dropped and its weight
 *       removed from that axis' normaliser.
 *   R7  curvature uses the same stencil on the unit normal.
 *   R8  "surrounding" cells = the 18 D3Q19 neighbours.
 *   R9  conflicts: gas next to a filling cell becomes interface; an emptying
 *       cell next to a filling cell stays interface; liquid next to a remaining
 *       emptying cell becomes interface.
 *   R10 refill sources V: liquid or interface after R9, not newly created,
 *       not emptying.
 *   R11 rho_bar, u_bar: arithmetic mean over V in direction order.
 *   R12 EQ+NEQ uses the neighbour's own equilibrium; c^n = argmax_{i in V}
 *       c_i . n with the lowest index on ties (scores within 1e-12 |n|_1 of
 *       the maximum tie, so rounding noise cannot decide); n from the fill
 *       level after S1.
 *   R13 GEQ prefactor w rho tau / (2 c_s^2) (the printed 1/nu is read as tau).
 *   R14 EXT order drops to what the run of valid cells along c^n allows.
 *   R16 excess mass is split evenly over the D3Q19 neighbours that are
 *       interface after S6; none -> reservoir, spread over all interface cells.
 *   R17 Thuerey's forced filling/emptying table for interface-interface links.
 *   R18 force density F = rho g.
 *   R22 TRT: symmetric/antisymmetric split, Lambda = 3/16 by default.
 *   R27 SRT collision relaxes towards equilibrium: Omega = -omega (f - f_eq).
 *   R28 densities used in S6/S7 are sums of the cell's post-collision PDFs.
 *   R29 Smagorinsky model (Sec. 2.1, turbulence model): tau = tau0 + tau_t
 *       solves nu_t = c_s^2 tau_t = (C_S dx)^2 S with S = Qbar / (2 rho c_s^2 tau)
 *       (the total tau, as in the cited Hou et al. model), Qbar = sqrt(2 Q:Q),
 *       Q_ab = sum_i c_ia c_ib (f_i - f_eq_i) from the post-streaming PDFs and
 *       the collision's own equilibrium, dx = 1.  Hence
 *       tau_t = (sqrt(tau0^2 + 2 C_S^2 Qbar / (rho c_s^4)) - tau0) / 2.  The
 *       printed form puts the bracket after the root (tau_t != 0 at
 *       equilibrium) and the factor 2 sqrt2, which belongs to the cited
 *       papers' sqrt(Q:Q) rather than to this Qbar = sqrt(2) sqrt(Q:Q).  With
 *       TRT the model sets omega+ = 1/tau and omega- follows from Lambda.  The
 *       GEQ refill keeps the user-chosen tau0.
 *   R30 free-slip walls (Sec. 2.1): a population whose next cell lies in a
 *       wall comes back with the wall-normal components of its velocity
 *       reversed, in the cell shifted by the remaining (tangential)
 *       components; so the pair (n, i) is linked to that cell for streaming
 *       and for the mass exchange (mass stays conserved), and a gas cell
 *       there is rebuilt by anti-bounce-back like any gas source.  Classes,
 *       conflicts, refill sources, excess receivers and normals keep treating
 *       walls as no cells.
 *   R31 bubble model (Sec. 2.2, volume pressure p_V(t) = p_V(0) V(0)/V(t) of
 *       an enclosed gas volume, tracked through coalescence and segmentation):
 *       a bubble is a connected set of gas and interface cells (D3Q19 links,
 *       as R8); a cell holds the gas volume max(0, 1 - phi), a bubble V = the
 *       sum over its cells.  A set that holds a cell of the top layer
 *       (z = nz-1) is the atmosphere and keeps p_V(0).  Every other bubble
 *       carries an amount n = p V: at the end of a step, each bubble b of the
 *       step's start hands its amount p_b V_b to the bubbles of the step's
 *       end, shared by the gas volume of its cells that each of them holds, and
 *       p_k = n_k / V_k.  So a bubble without a topology change keeps p V
 *       (Boyle's law), a merge adds amounts, and the parts of a split share
 *       one pressure.  The free-surface condition uses
 *       rho_G = 3 (p_k + 2 sigma kappa_m) with the pressure of the cell's
 *       bubble.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define Q 19
#define LIQ 1
#define IFC 2
#define GAS 4

/* D3Q19 velocity set: rest, 6 faces, 12 edges; opposite pairs adjacent. */
static const int CX[Q] = {0, 1, -1, 0, 0, 0, 0, 1, -1, 1, -1, 1, -1, 1, -1, 0, 0, 0, 0};
static const int CY[Q] = {0, 0, 0, 1, -1, 0, 0, 1, -1, -1, 1, 0, 0, 0, 0, 1, -1, 1, -1};
static const int CZ[Q] = {0, 0, 0, 0, 0, 1, -1, 0, 0, 0, 0, 1, -1, -1, 1, 1, -1, -1, 1};
static const double W0 = 1.0 / 3.0, W1 = 1.0 / 18.0, W2 = 1.0 / 36.0;
static const double CS2 = 1.0 / 3.0; /* R1 */

static double wgt(int i) { return i == 0 ? W0 : (i <= 6 ? W1 : W2); }
static int opp(int i) { return i == 0 ? 0 : ((i & 1) ? i + 1 : i - 1); }

typedef struct {
    int nx, ny, nz;
    int periodic[3];
    int collision;     /* 0 = SRT, 1 = TRT */
    int refill;        /* 0 EQ, 1 EQ+NEQ, 2 GEQ, 3 EXT, 4 AVG */
    double omega;      /* relaxation rate (omega+ for TRT) */
    double trt_lambda; /* TRT magic parameter */
    double g[3];       /* gravitational acceleration, lattice units */
    double sigma;      /* surface tension */
    double p_volume;   /* volume (atmospheric) pressure p_V */
    double eps_phi;    /* conversion threshold */
    double smag_cs;    /* Smagorinsky constant C_S (0 = no turbulence model) */
    int free_slip;     /* walls: 0 no-slip (bounce-back), 1 free-slip (specular) */
    int bubble_model;  /* 0 one volume pressure p_V; 1 per-bubble pressures (R31) */
} orc_params;

/* Per-step counters that the tests use to check the conversion logic. */
typedef struct {
    long n_to_liquid, n_to_gas, n_new_from_gas, n_from_liquid, n_cancelled;
    long n_reservoir_events;
} orc_counts;

/* ---------------------------------------------------------------- lattice */

int orc_q(void) { return Q; }
void orc_lattice(int *cx, int *cy, int *cz, double *w, int *op)
{
    for (int i = 0; i < Q; ++i) {
        cx[i] = CX[i]; cy[i] = CY[i]; cz[i] = CZ[i]; w[i] = wgt(i); op[i] = opp(i);
    }
}

/* Neighbour of cell n shifted by (dx,dy,dz); -1 if that lies in a wall. */
static long nbr(const orc_params *p, long n, int dx, int dy, int dz)
{
    long nx = p->nx, ny = p->ny, nz = p->nz;
    long x = n % nx, y = (n / nx) % ny, z = n / (nx * ny);
    x += dx; y += dy; z += dz;
    if (x < 0 || x >= nx) { if (!p->periodic[0]) return -1; x = (x + nx) % nx; }
    if (y < 0 || y >= ny) { if (!p->periodic[1]) return -1; y = (y + ny) % ny; }
    if (z < 0 || z >= nz) { if (!p->periodic[2]) return -1; z = (z + nz) % nz; }
    return (z * ny + y) * nx + x;
}

/* Direction whose velocity is c with the components in mask negated. */
static int dir_of(int x, int y, int z)
{
    for (int k = 0; k < Q; ++k)
        if (CX[k] == x && CY[k] == y && CZ[k] == z) return k;
    return -1;
}

/*
 * Where a population leaving cell n along c_i goes next (R30): the cell at
 * n + c_i with direction i, or, when that lies in a wall, with free-slip walls
 * the cell n + c_i with the wall-crossing components left out and direction j
 * (those components of c_i reversed); with no-slip walls n itself, opp(i).
 * Returns 1 if a wall was hit.
 */
static int next_link(const orc_params *p, long n, int i, long *m, int *j)
{
    long nx = p->nx, ny = p->ny, nz = p->nz;
    long pos[3] = {n % nx, (n / nx) % ny, n / (nx * ny)};
    const long len[3] = {nx, ny, nz};
    int c[3] = {CX[i], CY[i], CZ[i]};
    int hit = 0;
    for (int a = 0; a < 3; ++a) {
        long q = pos[a] + c[a];
        if (q >= 0 && q < len[a]) { pos[a] = q; continue; }
        if (p->periodic[a]) { pos[a] = (q + len[a]) % len[a]; continue; }
        hit = 1;
        c[a] = -c[a];              /* reflected; the position stays in this layer */
    }
    if (!hit) { *m = (pos[2] * ny + pos[1]) * nx + pos[0]; *j = i; return 0; }
    if (!p->free_slip) { *m = n; *j = opp(i); return 1; }
    *m = (pos[2] * ny + pos[1]) * nx + pos[0];
    *j = dir_of(c[0], c[1], c[2]);
    return 1;
}

/* D3Q19 neighbour table of the current domain: entry i*N+n is the cell at
 * n + c_i, or -1 inside a wall.  Rebuilt whenever the domain changes. */
static int32_t *g_tab = NULL;
static int g_key[6] = {0, 0, 0, -1, -1, -1};

static const int32_t *nb_table(const orc_params *p)
{
    int key[6] = {p->nx, p->ny, p->nz, p->periodic[0], p->periodic[1], p->periodic[2]};
    if (g_tab && memcmp(key, g_key, sizeof key) == 0) return g_tab;
    long N = (long)p->nx * p->ny * p->nz;
    free(g_tab);
    g_tab = malloc(sizeof(int32_t) * Q * (size_t)N);
    for (int i = 0; i < Q; ++i)
        for (long n = 0; n < N; ++n) g_tab[(long)i * N + n] = (int32_t)nbr(p, n, CX[i], CY[i], CZ[i]);
    memcpy(g_key, key, sizeof key);
    return g_tab;
}

/* Neighbour of cell n along c_i (-1 = wall).  Every exported entry point that
 * reaches this calls nb_table(p) first. */
static long nb19(const orc_params *p, long n, int i)
{
    return g_tab[(long)i * ((long)p->nx * p->ny * p->nz) + n];
}

/* Equilibrium, Sec. 2.1 (second-order Maxwell-Boltzmann expansion). */
void orc_feq(double rho, const double u[3], double *feq)
{
    double uu = u[0] * u[0] + u[1] * u[1] + u[2] * u[2];
    for (int i = 0; i < Q; ++i) {
        double uc = u[0] * CX[i] + u[1] * CY[i] + u[2] * CZ[i];
        feq[i] = wgt(i) * rho * (1.0 + uc / CS2 + (uc * uc) / (2.0 * CS2 * CS2) - uu / (2.0 * CS2));
    }
}

static double feq_i(int i, double rho, const double u[3])
{
    double uu = u[0] * u[0] + u[1] * u[1] + u[2] * u[2];
    double uc = u[0] * CX[i] + u[1] * CY[i] + u[2] * CZ[i];
    return wgt(i) * rho * (1.0 + uc / CS2 + (uc * uc) / (2.0 * CS2 * CS2) - uu / (2.0 * CS2));
}

/* Guo forcing term without its (1 - omega/2) prefactor, Sec. 2.1. */
static void guo_hat(const double u[3], const double F[3], double *Fh)
{
    for (int i = 0; i < Q; ++i) {
        double uc = u[0] * CX[i] + u[1] * CY[i] + u[2] * CZ[i];
        double a0 = (CX[i] - u[0]) / CS2 + uc * CX[i] / (CS2 * CS2);
        double a1 = (CY[i] - u[1]) / CS2 + uc * CY[i] / (CS2 * CS2);
        double a2 = (CZ[i] - u[2]) / CS2 + uc * CZ[i] / (CS2 * CS2);
        Fh[i] = wgt(i) * (a0 * F[0] + a1 * F[1] + a2 * F[2]);
    }
}

static double omega_minus_of(double lambda, double omega_plus)
{
    /* Lambda = (1/omega+ - 1/2)(1/omega- - 1/2) */
    return 1.0 / (0.5 + lambda / (1.0 / omega_plus - 0.5));
}

/*
 * Relaxation rate of one cell (R29): the user-chosen omega, or with the
 * Smagorinsky model 1/tau from the non-equilibrium momentum flux of the
 * post-streaming PDFs f against the equilibrium feq of density rho.
 */
static double cell_omega(const orc_params *p, const double *f, const double *feq, double rho)
{
    if (!(p->smag_cs > 0.0)) return p->omega;
    double Qm[3][3] = {{0.0, 0.0, 0.0}, {0.0, 0.0, 0.0}, {0.0, 0.0, 0.0}};
    for (int i = 0; i < Q; ++i) {
        const int c[3] = {CX[i], CY[i], CZ[i]};
        double ne = f[i] - feq[i];
        for (int a = 0; a < 3; ++a)
            for (int b = 0; b < 3; ++b) Qm[a][b] += c[a] * c[b] * ne;
    }
    double qq = 0.0;
    for (int a = 0; a < 3; ++a)
        for (int b = 0; b < 3; ++b) qq += Qm[a][b] * Qm[a][b];
    double qbar = sqrt(2.0 * qq);
    double tau0 = 1.0 / p->omega;
    double cs2dx2 = p->smag_cs * p->smag_cs; /* Delta x_LES = 1 */
    double tau_t = 0.5 * (sqrt(tau0 * tau0 + 2.0 * cs2dx2 * qbar / (rho * CS2 * CS2)) - tau0);
    return 1.0 / (tau0 + tau_t);
}

/*
 * Collision of one cell's post-streaming PDFs f -> f* (in place), Sec. 2.1:
 * density and half-force-shifted velocity, equilibrium, SRT (R27) or TRT (R22),
 * Guo forcing with F = rho g (R18).
 */
void orc_collide(const orc_params *p, const double *g, double *f)
{
    double rho = 0.0, j[3] = {0.0, 0.0, 0.0};
    for (int i = 0; i < Q; ++i) {
        rho += f[i];
        j[0] += CX[i] * f[i]; j[1] += CY[i] * f[i]; j[2] += CZ[i] * f[i];
    }
    double F[3] = {rho * g[0], rho * g[1], rho * g[2]};
    double u[3];
    for (int a = 0; a < 3; ++a) u[a] = F[a] / (2.0 * rho) + j[a] / rho;
    double feq[Q], Fh[Q];
    orc_feq(rho, u, feq);
    guo_hat(u, F, Fh);
    const double omega = cell_omega(p, f, feq, rho);
    if (p->collision == 0) {
        double om = omega;
        for (int i = 0; i < Q; ++i)
            f[i] = f[i] - om * (f[i] - feq[i]) + (1.0 - om / 2.0) * Fh[i];
    } else {
        double op_ = omega, om_ = omega_minus_of(p->trt_lambda, omega);
        double out[Q];
        for (int i = 0; i < Q; ++i) {
            int k = opp(i);
            double fs = 0.5 * (f[i] + f[k]), fa = 0.5 * (f[i] - f[k]);
            double es = 0.5 * (feq[i] + feq[k]), ea = 0.5 * (feq[i] - feq[k]);
            double Fs = 0.5 * (Fh[i] + Fh[k]), Fa = 0.5 * (Fh[i] - Fh[k]);
            out[i] = f[i] - op_ * (fs - es) - om_ * (fa - ea)
                   + (1.0 - op_ / 2.0) * Fs + (1.0 - om_ / 2.0) * Fa;
        }
        for (int i = 0; i < Q; ++i) f[i] = out[i];
    }
}

/* The relaxation rate orc_collide would use for these post-streaming PDFs. */
double orc_cell_omega(const orc_params *p, const double *g, const double *f)
{
    double rho = 0.0, j[3] = {0.0, 0.0, 0.0};
    for (int i = 0; i < Q; ++i) {
        rho += f[i];
        j[0] += CX[i] * f[i]; j[1] += CY[i] * f[i]; j[2] += CZ[i] * f[i];
    }
    double u[3];
    for (int a = 0; a < 3; ++a) u[a] = rho * g[a] / (2.0 * rho) + j[a] / rho;
    double feq[Q];
    orc_feq(rho, u, feq);
    return cell_omega(p, f, feq, rho);
}

/* rho and u of a cell from its stored post-collision PDFs (R3). */
static void moments_post(const orc_params *p, const double *f, long N, long n,
                         double *rho, double u[3])
{
    double r = 0.0, j[3] = {0.0, 0.0, 0.0};
    for (int i = 0; i < Q; ++i) {
        double v = f[(long)i * N + n];
        r += v;
        j[0] += CX[i] * v; j[1] += CY[i] * v; j[2] += CZ[i] * v;
    }
    *rho = r;
    for (int a = 0; a < 3; ++a) u[a] = j[a] / r - p->g[a] / 2.0;
}

static double rho_post(const double *f, long N, long n)
{
    double r = 0.0;
    for (int i = 0; i < Q; ++i) r += f[(long)i * N + n];
    return r;
}

/* ------------------------------------------------ surface geometry (S0) */

/* The 13 stencil pairs (c, -c) of the 3x3x3 Parker-Youngs stencil and their
 * weights (4 face, 2 edge, 1 corner; R5). */
static const int PX[13] = {1, 0, 0, 1, 1, 1, 1, 0, 0, 1, 1, 1, 1};
static const int PY[13] = {0, 1, 0, 1, -1, 0, 0, 1, 1, 1, 1, -1, -1};
static const int PZ[13] = {0, 0, 1, 0, 0, 1, -1, 1, -1, 1, -1, 1, -1};
static const double PW[13] = {4, 4, 4, 2, 2, 2, 2, 2, 2, 1, 1, 1, 1};

/*
 * Parker-Youngs central-difference gradient of a cell field at cell n with the
 * wall narrowing of R6: a pair whose either end is a wall is dropped and its
 * weight taken out of the normaliser of each axis it contributes to.
 * field(k) is val[k*stride + comp] for k a cell index.
 */
static void py_gradient(const orc_params *p, long n, const double *val, int stride, int comp,
                        double out[3])
{
    double acc[3] = {0.0, 0.0, 0.0}, W[3] = {0.0, 0.0, 0.0};
    for (int k = 0; k < 13; ++k) {
        long a = nbr(p, n, PX[k], PY[k], PZ[k]);
        long b = nbr(p, n, -PX[k], -PY[k], -PZ[k]);
        if (a < 0 || b < 0) continue;
        double d = val[a * stride + comp] - val[b * stride + comp];
        int c[3] = {PX[k], PY[k], PZ[k]};
        for (int ax = 0; ax < 3; ++ax) {
            if (c[ax] == 0) continue;
            acc[ax] += PW[k] * c[ax] * d;
            W[ax] += 2.0 * PW[k];
        }
    }
    for (int ax = 0; ax < 3; ++ax) out[ax] = W[ax] > 0.0 ? acc[ax] / W[ax] : 0.0;
}

/* Interface normal n = grad(phi) at one cell (R5, R6). */
void orc_normal(const orc_params *p, const double *phi, long n, double out[3])
{
    py_gradient(p, n, phi, 1, 0, out);
}

/*
 * Normals on the band (interface cells and their 3x3x3 neighbours), then mean
 * curvature kappa_m = -div(n^)/2 at every interface cell (R4, R7), then the gas
 * density rho_G = 3 (p_V + 2 sigma kappa_m).  kappa may be NULL.
 */
void orc_surface(const orc_params *p, const uint8_t *flag, const double *phi,
                 const double *pvol, double *rhoG, double *kappa)
{
    long N = (long)p->nx * p->ny * p->nz;
    for (long n = 0; n < N; ++n) {
        rhoG[n] = 3.0 * (pvol ? pvol[n] : p->p_volume);
        if (kappa) kappa[n] = 0.0;
    }
    if (N <= 0 || (p->sigma == 0.0 && !kappa)) return;
    double *nh = calloc((size_t)N * 3, sizeof(double));
    uint8_t *band = calloc((size_t)N, 1);
    for (long n = 0; n < N; ++n) {
        if (flag[n] != IFC) continue;
        for (int dz = -1; dz <= 1; ++dz)
            for (int dy = -1; dy <= 1; ++dy)
                for (int dx = -1; dx <= 1; ++dx) {
                    long k = nbr(p, n, dx, dy, dz);
                    if (k >= 0) band[k] = 1;
                }
    }
    for (long n = 0; n < N; ++n) {
        if (!band[n]) continue;
        double g[3];
        py_gradient(p, n, phi, 1, 0, g);
        double len = sqrt(g[0] * g[0] + g[1] * g[1] + g[2] * g[2]);
        for (int a = 0; a < 3; ++a) nh[n * 3 + a] = len > 0.0 ? g[a] / len : 0.0;
    }
    for (long n = 0; n < N; ++n) {
        if (flag[n] != IFC) continue;
        double div = 0.0;
        for (int a = 0; a < 3; ++a) {
            double g[3];
            py_gradient(p, n, nh, 3, a, g);
            div += g[a];
        }
        double km = -0.5 * div;
        if (kappa) kappa[n] = km;
        rhoG[n] = 3.0 * ((pvol ? pvol[n] : p->p_volume) + 2.0 * p->sigma * km);
    }
    free(nh);
    free(band);
}

/* ------------------------------------------------------------- step */

enum { STD = 0, NOFLUID = 1, NOEMPTY = 2 };

/* Thuerey classes from the current cell types (R17). */
static int cell_class(const orc_params *p, const uint8_t *flag, long n)
{
    int has_liq = 0, has_gas = 0;
    for (int i = 1; i < Q; ++i) {
        long k = nb19(p, n, i);
        if (k < 0) continue;
        if (flag[k] == LIQ) has_liq = 1;
        if (flag[k] == GAS) has_gas = 1;
    }
    if (!has_liq) return NOFLUID;
    if (!has_gas) return NOEMPTY;
    return STD;
}

/* Mass flux factor of an interface-interface link after the forcing table (R17):
 * fin flows from the neighbour into the cell, fout from the cell to it. */
static double link_flux(int cc, int cn, double fin, double fout)
{
    if (cc == cn) return fin - fout;
    if (cc == STD) return cn == NOFLUID ? fin : -fout;
    if (cc == NOFLUID) return -fout;
    return fin; /* cc == NOEMPTY */
}

/* Refill of one newly created interface cell x (Sec. 3.1). */
static void refill_cell(const orc_params *p, const uint8_t *flag, const uint8_t *togas,
                        const double *phi, double *f, long N, long x)
{
    int valid[Q] = {0};
    long nb[Q];
    int nv = 0;
    double rs[Q], us[Q][3];
    for (int i = 1; i < Q; ++i) {
        nb[i] = nb19(p, x, i);
        long k = nb[i];
        if (k < 0) continue;
        /* R10: liquid or interface, not new (new cells are still gas-typed), not emptying */
        if (flag[k] == LIQ || (flag[k] == IFC && !togas[k])) {
            valid[i] = 1;
            ++nv;
            moments_post(p, f, N, k, &rs[i], us[i]);
        }
    }
    double fx[Q];
    double rb = 0.0, ub[3] = {0.0, 0.0, 0.0};
    if (nv > 0) {
        for (int i = 1; i < Q; ++i) {
            if (!valid[i]) continue;
            rb += rs[i];
            for (int a = 0; a < 3; ++a) ub[a] += us[i][a];
        }
        rb /= nv;
        for (int a = 0; a < 3; ++a) ub[a] /= nv;
    } else {
        rb = 1.0; /* unreachable: the filling neighbour is always valid */
    }
    orc_feq(rb, ub, fx); /* EQ */

    int scheme = p->refill;
    int cn = -1;
    if ((scheme == 1 || scheme == 3) && nv > 0) {
        double nrm[3];
        orc_normal(p, phi, x, nrm);
        /* c^n: largest c_i . n over valid directions; scores within a rounding
         * tolerance of the maximum count as tied and the lowest index wins */
        double best = -INFINITY, sc[Q];
        for (int i = 1; i < Q; ++i) {
            if (!valid[i]) continue;
            sc[i] = CX[i] * nrm[0] + CY[i] * nrm[1] + CZ[i] * nrm[2];
            if (sc[i] > best) best = sc[i];
        }
        double tol = 1e-12 * (fabs(nrm[0]) + fabs(nrm[1]) + fabs(nrm[2]));
        for (int i = 1; i < Q && cn < 0; ++i)
            if (valid[i] && sc[i] >= best - tol) cn = i;
    }
    if (scheme == 1 && cn > 0) { /* EQ+NEQ (R12) */
        double eqn[Q];
        orc_feq(rs[cn], us[cn], eqn);
        for (int i = 0; i < Q; ++i) fx[i] += f[(long)i * N + nb[cn]] - eqn[i];
    } else if (scheme == 2 && nv > 0) { /* GEQ (R13) */
        double du[3][3]; /* du[a][b] = d u_a / d x_b */
        int fwd[3] = {1, 3, 5}, bwd[3] = {2, 4, 6};
        for (int b = 0; b < 3; ++b) {
            int hp = valid[fwd[b]], hm = valid[bwd[b]];
            for (int a = 0; a < 3; ++a) {
                if (hp && hm) du[a][b] = (us[fwd[b]][a] - us[bwd[b]][a]) / 2.0;
                else if (hp) du[a][b] = us[fwd[b]][a] - ub[a];
                else if (hm) du[a][b] = ub[a] - us[bwd[b]][a];
                else du[a][b] = 0.0;
            }
        }
        double tau = 1.0 / p->omega;
        for (int i = 0; i < Q; ++i) {
            int c[3] = {CX[i], CY[i], CZ[i]};
            double s = 0.0;
            for (int a = 0; a < 3; ++a)
                for (int b = 0; b < 3; ++b)
                    s += (du[a][b] + du[b][a]) * (CS2 * (a == b ? 1.0 : 0.0) - c[a] * c[b]);
            fx[i] += wgt(i) * rb * tau / (2.0 * CS2) * s;
        }
    } else if (scheme == 3 && cn > 0) { /* EXT (R14) */
        long k1 = nb[cn];
        long k2 = nbr(p, k1, CX[cn], CY[cn], CZ[cn]);
        int v2 = k2 >= 0 && (flag[k2] == LIQ || (flag[k2] == IFC && !togas[k2]));
        long k3 = v2 ? nbr(p, k2, CX[cn], CY[cn], CZ[cn]) : -1;
        int v3 = k3 >= 0 && (flag[k3] == LIQ || (flag[k3] == IFC && !togas[k3]));
        for (int i = 0; i < Q; ++i) {
            double f1 = f[(long)i * N + k1];
            if (v2 && v3)
                fx[i] = 3.0 * f1 - 3.0 * f[(long)i * N + k2] + f[(long)i * N + k3];
            else if (v2)
                fx[i] = 2.0 * f1 - f[(long)i * N + k2];
            else
                fx[i] = f1;
        }
    } else if (scheme == 4 && nv > 0) { /* AVG */
        for (int i = 0; i < Q; ++i) {
            double s = 0.0;
            for (int j = 1; j < Q; ++j)
                if (valid[j]) s += f[(long)i * N + nb[j]];
            fx[i] = s / nv;
        }
    }
    for (int i = 0; i < Q; ++i) f[(long)i * N + x] = fx[i];
}

/*
 * Streaming into cell n (Sec. 2.1) with the boundary rules of Sec. 2.1/2.2:
 * a PDF arriving from a wall is bounced back, one arriving from a gas cell is
 * rebuilt by the anti-bounce-back condition with rho_G(n) and the cell's own
 * velocity (R3); all others are pulled from the neighbour.  fs holds f*(t).
 */
static void stream_cell(const orc_params *p, const uint8_t *flag, const double *fs,
                        const double *rhoG, long N, long n, double *fn)
{
    double rS = 0.0, uS[3] = {0.0, 0.0, 0.0};
    int need_u = 0;
    for (int i = 1; i < Q; ++i) {
        long s = nb19(p, n, opp(i));
        if (s < 0 && p->free_slip) { int jj; next_link(p, n, opp(i), &s, &jj); }
        if (s >= 0 && flag[s] == GAS) need_u = 1;
    }
    if (need_u) moments_post(p, fs, N, n, &rS, uS);
    fn[0] = fs[n];
    for (int i = 1; i < Q; ++i) {
        long s = nb19(p, n, opp(i));
        int io = opp(i);
        int k = i;                    /* direction in which the source sent it */
        if (s < 0 && p->free_slip) {
            /* specular wall (R30): the source is where opp(i) from n leads */
            int jj;
            next_link(p, n, io, &s, &jj);
            k = opp(jj);
        }
        if (s < 0) {
            fn[i] = fs[(long)io * N + n];                         /* bounce-back */
        } else if (flag[s] == GAS) {                               /* anti-bounce-back */
            fn[i] = feq_i(i, rhoG[n], uS) + feq_i(io, rhoG[n], uS) - fs[(long)io * N + n];
        } else {
            fn[i] = fs[(long)k * N + s];                           /* streaming */
        }
    }
}

/* Exposed for the unit tests: post-streaming PDFs of cell n given f*(t) and rho_G. */
void orc_stream_cell(const orc_params *p, const uint8_t *flag, const double *fs,
                     const double *rhoG, long n, double *fn)
{
    long N = (long)p->nx * p->ny * p->nz;
    nb_table(p);
    stream_cell(p, flag, fs, rhoG, N, n, fn);
}

/* Gas volume of a cell (R31). */
static double gas_volume(double phi) { return phi < 1.0 ? 1.0 - phi : 0.0; }

/* Bubbles (R31): the connected sets of gas and interface cells over D3Q19
 * links, each labelled with its smallest cell index (breadth-first from the
 * lowest unlabelled cell); liquid cells get -1. */
static void bubble_labels(const orc_params *p, const uint8_t *flag, long *lab)
{
    long N = (long)p->nx * p->ny * p->nz;
    long *queue = malloc(sizeof(long) * (N > 0 ? N : 1));
    for (long n = 0; n < N; ++n) lab[n] = -1;
    for (long s0 = 0; s0 < N; ++s0) {
        if (flag[s0] == LIQ || lab[s0] >= 0) continue;
        long head = 0, tail = 0;
        queue[tail++] = s0;
        lab[s0] = s0;
        while (head < tail) {
            long n = queue[head++];
            for (int i = 1; i < Q; ++i) {
                long k = nb19(p, n, i);
                if (k < 0 || flag[k] == LIQ || lab[k] >= 0) continue;
                lab[k] = s0;
                queue[tail++] = k;
            }
        }
    }
    free(queue);
}

/* The bubble pressures after a step (R31).  lab0 / V0: the bubbles of the
 * step's start and their volumes; pbub holds the pressures of the start on
 * entry and of the end on return (0 on liquid cells). */
static void bubble_update(const orc_params *p, const uint8_t *flag, const double *phi,
                          const long *lab0, const double *V0, double *pbub)
{
    long N = (long)p->nx * p->ny * p->nz, layer = (long)p->nx * p->ny;
    long *lab1 = malloc(sizeof(long) * (N > 0 ? N : 1));
    double *V1 = calloc((size_t)N + 1, sizeof(double)), *amount = calloc((size_t)N + 1, sizeof(double));
    double *kept = calloc((size_t)N + 1, sizeof(double));
    uint8_t *atm = calloc((size_t)N + 1, 1);
    bubble_labels(p, flag, lab1);
    for (long n = 0; n < N; ++n) {
        if (lab1[n] < 0) continue;
        V1[lab1[n]] += gas_volume(phi[n]);
        if (n / layer == p->nz - 1) atm[lab1[n]] = 1;
    }
    /* each old bubble's amount, shared by the gas volume of its cells that
     * are still gas or interface */
    for (long n = 0; n < N; ++n)
        if (lab0[n] >= 0 && lab1[n] >= 0) kept[lab0[n]] += gas_volume(phi[n]);
    for (long n = 0; n < N; ++n) {
        if (lab0[n] < 0 || lab1[n] < 0) continue;
        long b = lab0[n];
        if (kept[b] > 0.0) amount[lab1[n]] += pbub[b] * V0[b] * gas_volume(phi[n]) / kept[b];
    }
    for (long n = 0; n < N; ++n) {
        long k = lab1[n];
        if (k < 0) pbub[n] = 0.0;
        else if (atm[k] || !(V1[k] > 0.0) || !(amount[k] > 0.0)) pbub[n] = p->p_volume;
        else pbub[n] = amount[k] / V1[k];
    }
    free(lab1); free(V1); free(amount); free(kept); free(atm);
}

/*
 * One FSLBM time step on the canonical state (in place).  pbub: the bubble
 * pressure of every gas and interface cell (R31), or NULL without the bubble
 * model.  Returns 0.
 */
static int step_once(const orc_params *p, uint8_t *flag, double *f, double *m, double *phi,
                     double *reservoir, double *pbub, orc_counts *cnt)
{
    long N = (long)p->nx * p->ny * p->nz;
    double *fs = malloc(sizeof(double) * Q * N); /* f*(t) */
    double *rhoG = malloc(sizeof(double) * N);
    uint8_t *cls = calloc((size_t)N, 1);
    uint8_t *toliq = calloc((size_t)N, 1), *togas = calloc((size_t)N, 1);
    uint8_t *newg = calloc((size_t)N, 1), *froml = calloc((size_t)N, 1);
    uint8_t *conv = calloc((size_t)N, 1), *touched = calloc((size_t)N, 1);
    double *mex = calloc((size_t)N, sizeof(double));
    double *phis = malloc(sizeof(double) * N); /* phi(t) */
    memcpy(fs, f, sizeof(double) * Q * N);
    memcpy(phis, phi, sizeof(double) * N);

    /* the bubbles at the step's start and their volumes (R31) */
    const int bubbles = p->bubble_model && pbub;
    long *lab0 = NULL;
    double *V0 = NULL;
    if (bubbles) {
        lab0 = malloc(sizeof(long) * (N > 0 ? N : 1));
        V0 = calloc((size_t)N + 1, sizeof(double));
        bubble_labels(p, flag, lab0);
        for (long n = 0; n < N; ++n)
            if (lab0[n] >= 0) V0[lab0[n]] += gas_volume(phi[n]);
    }

    /* S0: surface geometry from phi(t). */
    orc_surface(p, flag, phi, bubbles ? pbub : NULL, rhoG, NULL);

    /* Thuerey classes of interface cells from flags(t). */
    for (long n = 0; n < N; ++n)
        if (flag[n] == IFC) cls[n] = (uint8_t)cell_class(p, flag, n);

    /* S1 + S2 per fluid cell. */
    for (long n = 0; n < N; ++n) {
        if (flag[n] != LIQ && flag[n] != IFC) continue;
        double fn[Q];
        stream_cell(p, flag, fs, rhoG, N, n, fn);
        if (flag[n] == IFC) {
            double dm = 0.0;
            for (int i = 1; i < Q; ++i) {
                long k = nb19(p, n, i);
                int kin = opp(i);     /* direction of the population k sends to n */
                if (k < 0 && p->free_slip) {
                    int jj;
                    if (next_link(p, n, i, &k, &jj) && k == n) continue;   /* returns to n itself */
                    kin = opp(jj);
                }
                if (k < 0 || flag[k] == GAS) continue;
                double fin = fs[(long)kin * N + k];
                double fout = fs[(long)i * N + n];
                if (flag[k] == LIQ) dm += fin - fout;
                else dm += 0.5 * (phis[n] + phis[k]) * link_flux(cls[n], cls[k], fin, fout);
            }
            m[n] = m[n] + dm;
        }
        double rho = 0.0;
        for (int i = 0; i < Q; ++i) rho += fn[i];
        if (flag[n] == IFC) phi[n] = m[n] / rho;
        orc_collide(p, p->g, fn);
        for (int i = 0; i < Q; ++i) f[(long)i * N + n] = fn[i];
    }

    /* S3: mark. */
    for (long n = 0; n < N; ++n) {
        if (flag[n] != IFC) continue;
        if (phi[n] > 1.0 + p->eps_phi) toliq[n] = 1;
        else if (phi[n] < 0.0 - p->eps_phi) togas[n] = 1;
    }

    /* S4: resolve (R9). */
    uint8_t *keep = calloc((size_t)N, 1);
    for (long n = 0; n < N; ++n) {
        if (!toliq[n]) continue;
        for (int i = 1; i < Q; ++i) {
            long k = nb19(p, n, i);
            if (k >= 0 && flag[k] == GAS) newg[k] = 1;
        }
    }
    for (long n = 0; n < N; ++n) {
        if (!togas[n]) continue;
        int near_fill = 0;
        for (int i = 1; i < Q; ++i) {
            long k = nb19(p, n, i);
            if (k >= 0 && toliq[k]) near_fill = 1;
        }
        keep[n] = (uint8_t)!near_fill;
    }
    for (long n = 0; n < N; ++n) {
        if (!togas[n]) continue;
        if (!keep[n]) { togas[n] = 0; if (cnt) cnt->n_cancelled++; }
    }
    for (long n = 0; n < N; ++n) {
        if (!togas[n]) continue;
        for (int i = 1; i < Q; ++i) {
            long k = nb19(p, n, i);
            if (k >= 0 && flag[k] == LIQ) froml[k] = 1;
        }
    }
    free(keep);

    /* S5: refill newly created interface cells (they are still gas-typed). */
    for (long n = 0; n < N; ++n)
        if (newg[n]) refill_cell(p, flag, togas, phi, f, N, n);

    /* S6: apply conversions. */
    for (long n = 0; n < N; ++n) {
        if (flag[n] == IFC && toliq[n]) {
            mex[n] = m[n] - rho_post(f, N, n);
            flag[n] = LIQ; phi[n] = 1.0; m[n] = 0.0; conv[n] = 1;
            if (cnt) cnt->n_to_liquid++;
        } else if (flag[n] == IFC && togas[n]) {
            mex[n] = m[n];
            flag[n] = GAS; phi[n] = 0.0; m[n] = 0.0; conv[n] = 1;
            for (int i = 0; i < Q; ++i) f[(long)i * N + n] = 0.0; /* PDFs invalid */
            if (cnt) cnt->n_to_gas++;
        } else if (flag[n] == GAS && newg[n]) {
            flag[n] = IFC; phi[n] = 0.0; m[n] = 0.0;
            if (cnt) cnt->n_new_from_gas++;
        } else if (flag[n] == LIQ && froml[n]) {
            flag[n] = IFC; phi[n] = 1.0; m[n] = rho_post(f, N, n);
            if (cnt) cnt->n_from_liquid++;
        }
    }

    /* S7: excess mass (R16). */
    for (long n = 0; n < N; ++n) {
        if (!conv[n]) continue;
        int nr = 0;
        for (int i = 1; i < Q; ++i) {
            long k = nb19(p, n, i);
            if (k >= 0 && flag[k] == IFC) ++nr;
        }
        if (nr == 0) {
            *reservoir += mex[n];
            if (cnt) cnt->n_reservoir_events++;
            continue;
        }
        double share = mex[n] / nr;
        for (int i = 1; i < Q; ++i) {
            long k = nb19(p, n, i);
            if (k >= 0 && flag[k] == IFC) { m[k] += share; touched[k] = 1; }
        }
    }
    if (*reservoir != 0.0) {
        long nif = 0;
        for (long n = 0; n < N; ++n) nif += flag[n] == IFC;
        if (nif > 0) {
            double share = *reservoir / nif;
            for (long n = 0; n < N; ++n)
                if (flag[n] == IFC) { m[n] += share; touched[n] = 1; }
            *reservoir = 0.0;
        }
    }
    for (long n = 0; n < N; ++n)
        if (touched[n]) phi[n] = m[n] / rho_post(f, N, n);

    if (bubbles) {
        bubble_update(p, flag, phi, lab0, V0, pbub);
        free(lab0); free(V0);
    }
    free(fs); free(rhoG); free(cls); free(toliq); free(togas); free(newg); free(froml);
    free(conv); free(touched); free(mex); free(phis);
    return 0;
}

int orc_step(const orc_params *p, uint8_t *flag, double *f, double *m, double *phi,
             double *reservoir, double *pbub, int nsteps, orc_counts *cnt)
{
    if (cnt) memset(cnt, 0, sizeof(*cnt));
    nb_table(p);
    for (int s = 0; s < nsteps; ++s) step_once(p, flag, f, m, phi, reservoir, pbub, cnt);
    return 0;
}

/* Bubble labels of a state (R31), for the tests. */
void orc_bubble_labels(const orc_params *p, const uint8_t *flag, long *lab)
{
    nb_table(p);
    bubble_labels(p, flag, lab);
}

/* Equilibrium initial PDFs f* = f_eq(rho, u) of liquid and interface cells;
 * u is [3][N]. Gas cells get 0. */
void orc_init_equilibrium(const orc_params *p, const uint8_t *flag, const double *rho,
                          const double *u, double *f)
{
    long N = (long)p->nx * p->ny * p->nz;
    for (long n = 0; n < N; ++n) {
        double fe[Q], un[3] = {u[n], u[N + n], u[2 * N + n]};
        if (flag[n] == LIQ || flag[n] == IFC) orc_feq(rho[n], un, fe);
        else for (int i = 0; i < Q; ++i) fe[i] = 0.0;
        for (int i = 0; i < Q; ++i) f[(long)i * N + n] = fe[i];
    }
}

/* Total liquid mass: sum of liquid densities, interface masses and reservoir. */
double orc_total_mass(const orc_params *p, const uint8_t *flag, const double *f, const double *m,
                      double reservoir)
{
    long N = (long)p->nx * p->ny * p->nz;
    double s = 0.0;
    for (long n = 0; n < N; ++n) {
        if (flag[n] == LIQ) s += rho_post(f, N, n);
        else if (flag[n] == IFC) s += m[n];
    }
    return s + reservoir;
}

/* Macroscopic fields of the canonical state: rho and u (R3) of fluid cells. */
void orc_macroscopic(const orc_params *p, const uint8_t *flag, const double *f, double *rho,
                     double *u)
{
    long N = (long)p->nx * p->ny * p->nz;
    for (long n = 0; n < N; ++n) {
        double r = 0.0, uu[3] = {0.0, 0.0, 0.0};
        if (flag[n] == LIQ || flag[n] == IFC) moments_post(p, f, N, n, &r, uu);
        rho[n] = r;
        u[n] = uu[0]; u[N + n] = uu[1]; u[2 * N + n] = uu[2];
    }
}

/* Exposed for the unit tests: refill one gas cell x marked as newly created,
 * with the given emptying marks, exactly as S5 does. */
void orc_refill_cell(const orc_params *p, const uint8_t *flag, const uint8_t *togas,
                     const double *phi, double *f, long x)
{
    long N = (long)p->nx * p->ny * p->nz;
    nb_table(p);
    refill_cell(p, flag, togas, phi, f, N, x);
}

/* Exposed for the unit tests: mass flux of an interface-interface link. */
double orc_link_flux(int cc, int cn, double fin, double fout) { return link_flux(cc, cn, fin, fout); }
