/*
 * lattice_oracle.c -- plain, slow, FP64 CPU oracle for the lattice field step
 * described in the CosmoLattice paper (arXiv:2102.01031).
 *
 * TEST INFRASTRUCTURE ONLY.  Only tests/, the package smoke check and the
 * CPU-baseline leg of bench.py may load this library.  It shares no code,
 * header, table or helper with the HIP library; it is compiled with gcc.
 *
 * Conventions (program variables of sec. 4.1-4.2, eq. FieldSpaceTimeNaturalVariables):
 *   - N^3 periodic lattice, spacing dx, site (x,y,z), index x + N*(y + N*z)
 *     (sec. 3.1, "Basic lattice definitions").
 *   - <X> = N^-3 sum_n X(n) is the volume average.
 *   - alpha-time eta, scale factor a, b = a' (sec. 4.5.2).
 *   - All volume sums use Neumaier-compensated summation, visited in plain
 *     z, y, x order, so the oracle's sums are (nearly) correctly rounded.
 *
 * Readings of points the paper leaves open (the paper defers the discrete
 * update formulas to its companion reference):
 *   R1  velocity-Verlet with self-consistent expansion: kick pi and b by h/2
 *       at the start point, drift a by h*b, drift phi with the mean scale
 *       factor (a_n + a_{n+1})/2 raised to alpha-3, kick pi by h/2 at the end
 *       point, recompute the energies there, kick b by h/2.  E_K is taken at
 *       integer times.
 *   R2  4th order velocity-Verlet = Yoshida's triple-jump composition of the
 *       whole second-order map (Yoshida 1990, Phys. Lett. A 150, 262).  The
 *       6th and 8th orders are the symmetric compositions of the same paper
 *       with 7 maps (solution A) and 15 maps (solution D); the 10th order is
 *       the triple jump S_10(h) = S_8(x1 h) S_8(x0 h) S_8(x1 h), x1 = 1/(2 - c),
 *       x0 = -c/(2 - c), c = 2^{1/9}: 3, 7, 15 and 45 second-order maps per step.
 *   R3  fixed background: every kick uses a(t) at the kick time and every
 *       drift uses a(t) at the midpoint time of the drift (closed form of
 *       eq. ScaleFactorPowerLaw).
 *   R4  leapfrog energies are measured on momenta synchronised to integer
 *       time by a half kick that is not written back (sec. 6.1 describes the
 *       sync before measurements).
 *   A3  leapfrog with self-consistent expansion (sec. 6.1 keeps the momentum
 *       averages of the kicks and the field averages of the drifts for the
 *       scale factor): fields and a at integer times, momenta and b = a' half a
 *       step behind.  A full kick at time n advances pi by h K_phi(a_n, phi_n)
 *       and b by h K_a(a_n, E_n), where E_G, E_V are those of phi_n and E_K is
 *       the mean of the kinetic energies of the momenta before and after the
 *       kick (both at a_n); then a_{n+1} = a_n + h b and phi drifts with
 *       ((a_n + a_{n+1})/2)^{alpha-3}.  The half kicks that leave or reach
 *       integer time (the first kick from synchronised momenta, the sync) take
 *       E_K of the momenta at the half step.  K_a is linear in E_K, so a sync
 *       followed by a half kick is the full kick: the trajectory does not
 *       depend on when it is synchronised, and the scheme is explicit and
 *       time-reversible.
 *   R5  U(1): compact formulation of the U(1) toolkit (sec. 3.2) with the
 *       plaquette V_i V_{j,+i} V*_{i,+j} V*_j and kicks equal to minus the
 *       derivative of the lattice Hamiltonian.  The complex field carries the
 *       1/sqrt(2) normalisation of eq. ChargedScalars.  With expansion the
 *       terms take the powers of a of reading U1 (at the U(1) code).
 *   R6  SU(2): compact formulation of the SU(N) toolkit (sec. 3.2) for a
 *       doublet and SU(2) links, Hamiltonian form with the electric field
 *       conjugate to the link under left multiplication, kicks equal to minus
 *       the derivative of the lattice Hamiltonian and the link drift
 *       U <- exp(-i h g dx E^a T_a) U; the magnetic term 2/(g^2 dx^4) (2 - Tr P)
 *       per plaquette is the normalisation the toolkit's expansion of Tr P
 *       fixes.  With expansion the terms take the powers of a of reading U1
 *       (below, at the SU(2) code).
 *   R14 Gauss-consistent initial gauge momenta: with the links at the
 *       identity (the initial condition of sec. 5.5.1) the Gauss law is the
 *       plain lattice divergence div- E = rho; its longitudinal solution uses
 *       the lattice Laplacian sum_i grad-_i grad+_i (the continuum i k_i / k^2
 *       of eq. GaugeCurrentFluc would leave a residual of order dx^2).
 *   R15 gauge models with the velocity-Verlet family: the second-order map
 *       kick(h/2) drift(h) kick(h/2) of the whole U(1) or SU(2) system, and
 *       the compositions of R2 above it; the kicks and drifts are those of the
 *       leapfrog (the paper applies its VV evolvers to gauge theories too).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

/* ------------------------------------------------------------------ */
/* Parameters                                                          */
/* ------------------------------------------------------------------ */

enum { ORC_PHI4 = 0, ORC_PHI4_CHI2 = 1 };
enum { ORC_NONE = 0, ORC_FIXED = 1, ORC_SELF = 2 };
enum { ORC_LF = 0, ORC_VV2 = 1, ORC_VV4 = 2, ORC_VV6 = 3, ORC_VV8 = 4, ORC_VV10 = 5 };

typedef struct orc_params {
    int32_t N;           /* lattice points per dimension                     */
    int32_t nfields;     /* number of real scalar fields: 1 (phi) or 2 (phi, chi) */
    int32_t potential;   /* ORC_PHI4: lambda/4 phi^4 ; ORC_PHI4_CHI2: + q/2 phi^2 chi^2 */
    int32_t expansion;   /* ORC_NONE (a=1), ORC_FIXED (power law), ORC_SELF (Friedmann) */
    int32_t integrator;  /* ORC_LF, ORC_VV2, ORC_VV4, ORC_VV6, ORC_VV8, ORC_VV10 */
    int32_t pad;
    double dx, dt;       /* lattice spacing and time step (program units)    */
    double lambda, q;    /* potential couplings                              */
    double alpha;        /* alpha-time exponent (eq. FLRWmetric)             */
    double kappa2;       /* (f_star/m_p)^2 in the Friedmann kernel              */
    double w_eos, H0;    /* fixed background: equation of state, initial H  */
    double t0, a0;       /* fixed background reference time and scale factor */
} orc_params;

/* The clock: time, scale factor and its derivative, and the leapfrog phase.
 * lf_stag = 0: momenta at integer time; +1 / -1: momenta half a step behind
 * (forward / backward run), so that a sync kick of lf_stag*dt/2 restores them. */
typedef struct orc_clock {
    double t, a, b;
    int32_t lf_stag;
    int32_t pad;
} orc_clock;

/* Threads.  Built with OpenMP, the site loops that write one value per site
 * (stencils, forces, kicks, drifts) are split over z planes; every volume sum
 * stays a single serial compensated sum in z, y, x order, so results do not
 * depend on the thread count.  Without OpenMP everything runs on one thread. */
int orc_set_threads(int n)
{
#ifdef _OPENMP
    if (n > 0) omp_set_num_threads(n);
    return omp_get_max_threads();
#else
    (void)n;
    return 1;
#endif
}

/* ------------------------------------------------------------------ */
/* Lattice helpers                                                     */
/* ------------------------------------------------------------------ */

static size_t at(int N, int x, int y, int z)
{
    return (size_t)x + (size_t)N * ((size_t)y + (size_t)N * (size_t)z);
}
static int up(int i, int N) { return i + 1 == N ? 0 : i + 1; }
static int dn(int i, int N) { return i == 0 ? N - 1 : i - 1; }

/* neighbour of (x,y,z) one unit along direction d (0=x,1=y,2=z), sign s=+1/-1 */
static size_t nbr(int N, int x, int y, int z, int d, int s)
{
    int c[3] = {x, y, z};
    c[d] = s > 0 ? up(c[d], N) : dn(c[d], N);
    return at(N, c[0], c[1], c[2]);
}

typedef struct { double s, c; } nsum;   /* Neumaier compensated sum */
static void nadd(nsum *k, double v)
{
    double t = k->s + v;
    if (fabs(k->s) >= fabs(v)) k->c += (k->s - t) + v;
    else                       k->c += (v - t) + k->s;
    k->s = t;
}
static double nval(const nsum *k) { return k->s + k->c; }

static size_t vol(int N) { return (size_t)N * (size_t)N * (size_t)N; }

/* ------------------------------------------------------------------ */
/* Lattice operators (sec. 3.1, eqs. forwardbackwardd and               */
/* ForwardBackwardMomentum)                                            */
/* ------------------------------------------------------------------ */

/* Laplacian as sum_i of backward(forward(f)):
 *   (Lap f)(n) = dx^-2 sum_i [ f(n+i) - 2 f(n) + f(n-i) ]                  */
int orc_laplacian(int N, double dx, const double *f, double *out)
{
    if (N < 1) return -1;
    #pragma omp parallel for schedule(static)
    for (int z = 0; z < N; ++z)
        for (int y = 0; y < N; ++y)
            for (int x = 0; x < N; ++x) {
                double s = 0.0;
                double f0 = f[at(N, x, y, z)];
                for (int d = 0; d < 3; ++d)
                    s += f[nbr(N, x, y, z, d, +1)] - 2.0 * f0 + f[nbr(N, x, y, z, d, -1)];
                out[at(N, x, y, z)] = s / (dx * dx);
            }
    return 0;
}

/* sum_n sum_i (forward derivative of f)^2 = sum_n sum_i ((f(n+i)-f(n))/dx)^2 */
double orc_grad2_sum(int N, double dx, const double *f)
{
    nsum k = {0, 0};
    for (int z = 0; z < N; ++z)
        for (int y = 0; y < N; ++y)
            for (int x = 0; x < N; ++x)
                for (int d = 0; d < 3; ++d) {
                    double g = (f[nbr(N, x, y, z, d, +1)] - f[at(N, x, y, z)]) / dx;
                    nadd(&k, g * g);
                }
    return nval(&k);
}

/* ------------------------------------------------------------------ */
/* Potential (sec. 4.2, eq. potentialExampleI in program units)        */
/*   term 0: lambda/4 phi^4     term 1: q/2 phi^2 chi^2                 */
/* ------------------------------------------------------------------ */

static double pot_term(const orc_params *p, int m, double phi, double chi)
{
    if (m == 0) return 0.25 * p->lambda * phi * phi * phi * phi;
    if (p->potential == ORC_PHI4_CHI2) return 0.5 * p->q * phi * phi * chi * chi;
    return 0.0;
}

static double pot_deriv(const orc_params *p, int s, double phi, double chi)
{
    if (s == 0) {
        double d = p->lambda * phi * phi * phi;
        if (p->potential == ORC_PHI4_CHI2) d += p->q * phi * chi * chi;
        return d;
    }
    return p->potential == ORC_PHI4_CHI2 ? p->q * phi * phi * chi : 0.0;
}

static int nterms(const orc_params *p) { return p->potential == ORC_PHI4_CHI2 ? 2 : 1; }

/* kernel of pi_s (sec. 4.5.2): K_s = a^{1+alpha} Lap(phi_s) - a^{3+alpha} dV/dphi_s */
static void kernel_field(const orc_params *p, double a, double *const *phi, int s,
                         double *out)
{
    int N = p->N;
    size_t V = vol(N);
    double *lap = (double *)malloc(V * sizeof(double));
    orc_laplacian(N, p->dx, phi[s], lap);
    double c1 = pow(a, 1.0 + p->alpha), c3 = pow(a, 3.0 + p->alpha);
    #pragma omp parallel for schedule(static)
    for (size_t n = 0; n < V; ++n) {
        double chi = p->nfields > 1 ? phi[1][n] : 0.0;
        out[n] = c1 * lap[n] - c3 * pot_deriv(p, s, phi[0][n], chi);
    }
    free(lap);
}

int orc_kernel(const orc_params *p, double a, double *const *phi, int s, double *out)
{
    if (s < 0 || s >= p->nfields) return -1;
    kernel_field(p, a, phi, s, out);
    return 0;
}

/* ------------------------------------------------------------------ */
/* Energies (eq. EK_EG_EV and the E definitions of sec. 4.5.2)         */
/*   E_K^s = <pi_s^2>/(2 a^6), E_G^s = <sum_i (grad+_i phi_s)^2>/(2 a^2),  */
/*   E_V^m = <V_m>                                                      */
/* ------------------------------------------------------------------ */

typedef struct { double EK[2], EG[2], EV[2]; } energies;

static energies energies_of(const orc_params *p, double *const *phi, double *const *pi, double a)
{
    energies E;
    memset(&E, 0, sizeof(E));
    int N = p->N;
    size_t V = vol(N);
    for (int s = 0; s < p->nfields; ++s) {
        nsum k = {0, 0};
        for (size_t n = 0; n < V; ++n) nadd(&k, pi[s][n] * pi[s][n]);
        E.EK[s] = nval(&k) / (double)V / (2.0 * pow(a, 6.0));
        E.EG[s] = orc_grad2_sum(N, p->dx, phi[s]) / (double)V / (2.0 * a * a);
    }
    for (int m = 0; m < nterms(p); ++m) {
        nsum k = {0, 0};
        for (size_t n = 0; n < V; ++n)
            nadd(&k, pot_term(p, m, phi[0][n], p->nfields > 1 ? phi[1][n] : 0.0));
        E.EV[m] = nval(&k) / (double)V;
    }
    return E;
}

static double EK_tot(const energies *E) { return E->EK[0] + E->EK[1]; }
static double EG_tot(const energies *E) { return E->EG[0] + E->EG[1]; }
static double EV_tot(const energies *E) { return E->EV[0] + E->EV[1]; }
static double rho_tot(const energies *E) { return EK_tot(E) + EG_tot(E) + EV_tot(E); }

/* kernel of b (sec. 4.5.2):
 *   K_a = a^{2 alpha + 1}/3 kappa^2 [ (alpha-2) E_K + alpha E_G + (alpha+1) E_V ] */
static double kernel_a(const orc_params *p, double a, const energies *E)
{
    double al = p->alpha;
    return pow(a, 2.0 * al + 1.0) / 3.0 * p->kappa2 *
           ((al - 2.0) * EK_tot(E) + al * EG_tot(E) + (al + 1.0) * EV_tot(E));
}

/* Fixed power-law background (eq. ScaleFactorPowerLaw):
 *   p = 2/(3(1+w) - 2 alpha),  a = a0 (1 + H0 (t - t0)/p)^p,  b = a' = a0 H0 (1 + H0 (t-t0)/p)^(p-1) */
int orc_fixed_background(const orc_params *p, double t, double *a, double *b)
{
    double pw = 2.0 / (3.0 * (1.0 + p->w_eos) - 2.0 * p->alpha);
    double u = 1.0 + p->H0 * (t - p->t0) / pw;
    if (u <= 0.0) return -1;
    *a = p->a0 * pow(u, pw);
    *b = p->a0 * p->H0 * pow(u, pw - 1.0);
    return 0;
}

static double fixed_a(const orc_params *p, double t)
{
    double a, b;
    orc_fixed_background(p, t, &a, &b);
    return a;
}

/* Hubble constraint (eq. NewFriedmannEQsI): b^2 = a^{2 alpha + 2} kappa^2 rho / 3.
 * Returns the positive root for b given the state (expanding universe). */
int orc_hubble_b0(const orc_params *p, double *const *phi, double *const *pi, double a, double *b0)
{
    energies E = energies_of(p, phi, pi, a);
    double rhs = pow(a, 2.0 * p->alpha + 2.0) * p->kappa2 * rho_tot(&E) / 3.0;
    if (rhs < 0.0) return -1;
    *b0 = sqrt(rhs);
    return 0;
}

/* ------------------------------------------------------------------ */
/* Integrators (sec. 4.5.2 Hamiltonian system, readings R1-R4)         */
/* ------------------------------------------------------------------ */

typedef struct {
    const orc_params *p;
    double **phi, **pi;
    double *K[2];          /* scratch for the kernels */
    double a, b;           /* scale factor and its momentum (SELF) */
    energies E;            /* energies at the current integer point (SELF) */
} stepper;

static void kick(stepper *st, double a_kick, double w)
{
    const orc_params *p = st->p;
    size_t V = vol(p->N);
    for (int s = 0; s < p->nfields; ++s) kernel_field(p, a_kick, st->phi, s, st->K[s]);
    for (int s = 0; s < p->nfields; ++s)
        #pragma omp parallel for schedule(static)
        for (size_t n = 0; n < V; ++n) st->pi[s][n] += w * st->K[s][n];
}

static void drift(stepper *st, double a_mid, double h)
{
    const orc_params *p = st->p;
    size_t V = vol(p->N);
    double c = h * pow(a_mid, p->alpha - 3.0);
    for (int s = 0; s < p->nfields; ++s)
        #pragma omp parallel for schedule(static)
        for (size_t n = 0; n < V; ++n) st->phi[s][n] += c * st->pi[s][n];
}

/* scale factor seen by a kick at time t */
static double a_at(stepper *st, double t)
{
    switch (st->p->expansion) {
    case ORC_FIXED: return fixed_a(st->p, t);
    case ORC_SELF: return st->a;
    default: return 1.0;
    }
}

/* One second-order velocity-Verlet map of size h starting at time t (reading R1/R3). */
static void vv2(stepper *st, double t, double h)
{
    const orc_params *p = st->p;
    int self = p->expansion == ORC_SELF;
    double a_n = a_at(st, t);
    kick(st, a_n, 0.5 * h);                                       /* pi half kick   */
    if (self) st->b += 0.5 * h * kernel_a(p, a_n, &st->E);        /* b half kick    */
    double a_n1, a_mid;
    if (self) {
        a_n1 = a_n + h * st->b;                                   /* a drift        */
        a_mid = 0.5 * (a_n + a_n1);
    } else if (p->expansion == ORC_FIXED) {
        a_n1 = fixed_a(p, t + h);
        a_mid = fixed_a(p, t + 0.5 * h);
    } else {
        a_n1 = 1.0;
        a_mid = 1.0;
    }
    drift(st, a_mid, h);                                          /* phi drift      */
    if (self) st->a = a_n1;
    kick(st, a_n1, 0.5 * h);                                      /* pi half kick   */
    if (self) {
        st->E = energies_of(p, st->phi, st->pi, a_n1);            /* energies       */
        st->b += 0.5 * h * kernel_a(p, a_n1, &st->E);             /* b half kick    */
    }
}

/* Yoshida's fourth-order weights (reading R2): w1 = 1/(2 - 2^{1/3}), w0 = 1 - 2 w1 */
void orc_yoshida4(double *w1, double *w0)
{
    double c = cbrt(2.0);
    *w1 = 1.0 / (2.0 - c);
    *w0 = -c / (2.0 - c);
}

/* Triple-jump weights of order n + 2 from order n (reading R2):
 * x1 = 1/(2 - c), x0 = -c/(2 - c), c = 2^{1/(n+1)}; n = 2 gives orc_yoshida4. */
void orc_triple_jump(int n, double *x1, double *x0)
{
    double c = pow(2.0, 1.0 / (double)(n + 1));
    if (n == 2) c = cbrt(2.0);
    *x1 = 1.0 / (2.0 - c);
    *x0 = -c / (2.0 - c);
}

/* Stage weights of one velocity-Verlet step of even order `order` (reading R2):
 * the step is the product of second-order maps of sizes w[0] h, w[1] h, ...
 *   order 2: one map;
 *   order 4: Yoshida's triple jump (w1, w0, w1);
 *   order 6: Yoshida (1990, Phys. Lett. A 150, 262) solution A, seven maps
 *            w3 w2 w1 w0 w1 w2 w3 with w0 = 1 - 2(w1 + w2 + w3);
 *   order 8: the same paper's solution D, fifteen maps w7 ... w1 w0 w1 ... w7;
 *   order 10: the triple jump of the order-8 step (x1, x0, x1 with
 *            c = 2^{1/9}), 45 maps.
 * Returns the number of maps (at most 45). */
int orc_vv_stages(int order, double *w)
{
    static const double yA[3] = {-1.17767998417887, 0.235573213359357, 0.784513610477560};
    static const double yD[7] = {0.102799849391985, -1.96061023297549, 1.93813913762276, -0.158240635368243,
                                 -1.44485223686048, 0.253693336566229, 0.914844246229740};
    if (order == 2) {
        w[0] = 1.0;
        return 1;
    }
    if (order == 4) {
        orc_triple_jump(2, &w[0], &w[1]);
        w[2] = w[0];
        return 3;
    }
    if (order == 6 || order == 8) {
        const int m = order == 6 ? 3 : 7;
        const double *y = order == 6 ? yA : yD;
        double sum = 0.0;
        for (int i = 0; i < m; ++i) sum += y[i];
        for (int i = 0; i < m; ++i) {
            w[i] = y[m - 1 - i];          /* outermost first */
            w[2 * m - i] = y[m - 1 - i];
        }
        w[m] = 1.0 - 2.0 * sum;
        return 2 * m + 1;
    }
    if (order == 10) {
        double inner[15], x1, x0;
        const int n = orc_vv_stages(8, inner);
        orc_triple_jump(8, &x1, &x0);
        for (int i = 0; i < n; ++i) {
            w[i] = x1 * inner[i];
            w[n + i] = x0 * inner[i];
            w[2 * n + i] = x1 * inner[i];
        }
        return 3 * n;
    }
    return 0;
}

/* One step of the velocity-Verlet map of even order `order` (>= 2) of size h
 * starting at time t: the second-order maps of orc_vv_stages in order. */
static void vv_order(stepper *st, int order, double t, double h)
{
    double w[45];
    const int n = orc_vv_stages(order, w);
    for (int i = 0; i < n; ++i) {
        vv2(st, t, w[i] * h);
        t += w[i] * h;
    }
}

/* Evolve |nsteps| steps (backward in time if nsteps < 0).
 * Return codes: 0 ok, -1 bad arguments, -2 unsupported combination,
 * -3 leapfrog state is staggered in the other direction (sync first). */
int orc_run(const orc_params *p, double *const *phi, double *const *pi, orc_clock *c, long nsteps)
{
    if (p->N < 1 || p->nfields < 1 || p->nfields > 2) return -1;
    if (p->integrator < ORC_LF || p->integrator > ORC_VV10) return -1;
    if (nsteps == 0) return 0;
    int dir = nsteps > 0 ? 1 : -1;
    long ns = nsteps > 0 ? nsteps : -nsteps;
    double h = dir * p->dt;
    size_t V = vol(p->N);

    stepper st;
    st.p = p;
    st.phi = (double **)phi;
    st.pi = (double **)pi;
    st.K[0] = (double *)malloc(V * sizeof(double));
    st.K[1] = (double *)malloc(V * sizeof(double));
    st.a = c->a;
    st.b = c->b;
    double t_start = c->t;

    if (p->integrator == ORC_LF) {
        if (c->lf_stag != 0 && c->lf_stag != dir) { free(st.K[0]); free(st.K[1]); return -3; }
        for (long k = 0; k < ns; ++k) {
            double t = t_start + (double)k * h;
            double w = (c->lf_stag == 0) ? 0.5 * h : h;  /* first kick after a sync is half */
            if (p->expansion == ORC_SELF) {
                /* reading A3 */
                energies Eb = energies_of(p, st.phi, st.pi, st.a);   /* pi before the kick, phi_n */
                kick(&st, st.a, w);
                energies Ea = energies_of(p, st.phi, st.pi, st.a);   /* pi after the kick, phi_n  */
                if (c->lf_stag == 0)
                    st.b += w * kernel_a(p, st.a, &Ea);
                else
                    st.b += 0.5 * h * kernel_a(p, st.a, &Eb) + 0.5 * h * kernel_a(p, st.a, &Ea);
                double a_n1 = st.a + h * st.b;
                drift(&st, 0.5 * (st.a + a_n1), h);
                st.a = a_n1;
            } else {
                kick(&st, a_at(&st, t), w);
                double a_mid = p->expansion == ORC_FIXED ? fixed_a(p, t + 0.5 * h) : 1.0;
                drift(&st, a_mid, h);
            }
            c->lf_stag = dir;
        }
    } else {
        if (p->expansion == ORC_SELF) st.E = energies_of(p, st.phi, st.pi, st.a);
        double w1, w0;
        orc_yoshida4(&w1, &w0);
        for (long k = 0; k < ns; ++k) {
            double t = t_start + (double)k * h;
            if (p->integrator == ORC_VV2) {
                vv2(&st, t, h);
            } else if (p->integrator == ORC_VV4) {
                vv2(&st, t, w1 * h);
                vv2(&st, t + w1 * h, w0 * h);
                vv2(&st, t + w1 * h + w0 * h, w1 * h);
            } else {
                vv_order(&st, 2 * p->integrator, t, h);   /* VV6: 6, VV8: 8, VV10: 10 */
            }
        }
    }
    c->t = t_start + (double)ns * h;
    if (p->expansion == ORC_SELF) {
        c->a = st.a;
        c->b = st.b;
    } else if (p->expansion == ORC_FIXED) {
        orc_fixed_background(p, c->t, &c->a, &c->b);
    } else {
        c->a = 1.0;
        c->b = 0.0;
    }
    free(st.K[0]);
    free(st.K[1]);
    return 0;
}

/* Leapfrog sync (sec. 6.1): bring staggered momenta to integer time, in place;
 * with self-consistent expansion b too, with E_K of the momenta at the half
 * step (reading A3). */
int orc_lf_sync(const orc_params *p, double *const *phi, double *const *pi, orc_clock *c)
{
    if (c->lf_stag == 0) return 0;
    stepper st;
    size_t V = vol(p->N);
    st.p = p;
    st.phi = (double **)phi;
    st.pi = (double **)pi;
    st.K[0] = (double *)malloc(V * sizeof(double));
    st.K[1] = (double *)malloc(V * sizeof(double));
    st.a = c->a;
    double w = 0.5 * c->lf_stag * p->dt;
    if (p->expansion == ORC_SELF) {
        energies E = energies_of(p, st.phi, st.pi, c->a);
        c->b += w * kernel_a(p, c->a, &E);
    }
    kick(&st, a_at(&st, c->t), w);
    c->lf_stag = 0;
    free(st.K[0]);
    free(st.K[1]);
    return 0;
}

/* Energies of the state, output layout (12 doubles):
 *   [0,1] E_K per field, [2,3] E_G per field, [4,5] E_V per term, [6] rho,
 *   [7] Hubble LHS b^2, [8] Hubble RHS a^{2alpha+2} kappa^2 rho/3,
 *   [9] (LHS-RHS)/(LHS+RHS), [10] a, [11] b at integer time.
 * Leapfrog momenta (and b with self-consistent expansion) are synchronised on
 * a copy (readings R4, A3). */
int orc_energy(const orc_params *p, double *const *phi, double *const *pi, const orc_clock *c,
               double *out)
{
    size_t V = vol(p->N);
    double *pis[2] = {NULL, NULL};
    for (int s = 0; s < p->nfields; ++s) {
        pis[s] = (double *)malloc(V * sizeof(double));
        memcpy(pis[s], pi[s], V * sizeof(double));
    }
    orc_clock cc = *c;
    if (c->lf_stag != 0) orc_lf_sync(p, phi, pis, &cc);
    energies E = energies_of(p, phi, pis, c->a);
    for (int s = 0; s < p->nfields; ++s) free(pis[s]);
    double rho = rho_tot(&E);
    double lhs = cc.b * cc.b;
    double rhs = pow(c->a, 2.0 * p->alpha + 2.0) * p->kappa2 * rho / 3.0;
    out[0] = E.EK[0]; out[1] = E.EK[1];
    out[2] = E.EG[0]; out[3] = E.EG[1];
    out[4] = E.EV[0]; out[5] = E.EV[1];
    out[6] = rho;
    out[7] = lhs;
    out[8] = rhs;
    out[9] = (lhs + rhs) != 0.0 ? (lhs - rhs) / (lhs + rhs) : 0.0;
    out[10] = c->a;
    out[11] = cc.b;
    return 0;
}

/* ------------------------------------------------------------------ */
/* Adjoint of the second-order velocity-Verlet map, two fields with     */
/* V = lambda/4 phi^4 + q/2 phi^2 chi^2, a = 1 or a fixed background a(t) */
/* (reading R3: kicks at a(t) of the kick, drifts at a(t + h/2)).        */
/*   forward: pi' = pi + h/2 K(a_n, phi); phi' = phi + h d pi';          */
/*            pi'' = pi' + h/2 K(a_n+1, phi')                            */
/*   K(a, phi) = kL Lap phi - kV grad V(phi), kL = a^{1+alpha},           */
/*   kV = a^{3+alpha}, d = a(t + h/2)^{alpha-3};                          */
/*   dK = kL Lap - kV H_V(phi)  (symmetric)                               */
/* ------------------------------------------------------------------ */

/* scale factor of the adjoint's background at time t */
static double adj_a(const orc_params *p, double t) { return p->expansion == ORC_FIXED ? fixed_a(p, t) : 1.0; }

/* out_s = kL Lap(l_s) - kV sum_r H_V(phi)_{sr} l_r  (transpose of dK, which is symmetric) */
static void jac_F_T(const orc_params *p, double *const *phi, double *const *l, double **out,
                    double *lap, double kL, double kV)
{
    size_t V = vol(p->N);
    for (int s = 0; s < 2; ++s) {
        orc_laplacian(p->N, p->dx, l[s], lap);
        for (size_t n = 0; n < V; ++n) {
            double f = phi[0][n], x = phi[1][n];
            double h00 = 3.0 * p->lambda * f * f + p->q * x * x;   /* d2V/dphi2   */
            double h01 = 2.0 * p->q * f * x;                         /* d2V/dphidchi */
            double h11 = p->q * f * f;                               /* d2V/dchi2   */
            double hl = s == 0 ? h00 * l[0][n] + h01 * l[1][n] : h01 * l[0][n] + h11 * l[1][n];
            out[s][n] = kL * lap[n] - kV * hl;
        }
    }
}

/* sum_n l(n) . dF/dq(phi(n)) at a = 1,  dF/dq = -(phi chi^2, phi^2 chi); a kick
 * at scale factor a scales it by kV */
static double dot_dFdq(const orc_params *p, double *const *phi, double *const *l)
{
    nsum k = {0, 0};
    size_t V = vol(p->N);
    for (size_t n = 0; n < V; ++n) {
        double f = phi[0][n], x = phi[1][n];
        nadd(&k, -l[0][n] * f * x * x);
        nadd(&k, -l[1][n] * f * f * x);
    }
    return nval(&k);
}

static int check_adj(const orc_params *p)
{
    if (p->nfields != 2 || p->potential != ORC_PHI4_CHI2 || p->expansion == ORC_SELF) return -2;
    return 0;
}

/* One VV2 step from time t of the state (phi, pi) together with its tangent
 * (dphi, dpi) along an extra coupling direction dq. All arrays are updated in place. */
int orc_vv2_tangent(const orc_params *p, double t, double *const *phi, double *const *pi,
                    double *const *dphi, double *const *dpi, double dq)
{
    if (check_adj(p)) return -2;
    size_t V = vol(p->N);
    double h = p->dt, al = p->alpha;
    double ak[2] = {adj_a(p, t), adj_a(p, t + h)};
    double dr = h * pow(adj_a(p, t + 0.5 * h), al - 3.0);
    double *lap = (double *)malloc(V * sizeof(double));
    double *J[2] = {(double *)malloc(V * sizeof(double)), (double *)malloc(V * sizeof(double))};
    double *K[2] = {(double *)malloc(V * sizeof(double)), (double *)malloc(V * sizeof(double))};
    for (int half = 0; half < 2; ++half) {
        /* kick at the current position: pi += h/2 K(phi); dpi += h/2 (dK dphi + dK/dq dq) */
        double kL = pow(ak[half], 1.0 + al), kV = pow(ak[half], 3.0 + al);
        jac_F_T(p, phi, dphi, J, lap, kL, kV);  /* dK symmetric: dK dphi = dK^T dphi */
        for (int s = 0; s < 2; ++s) kernel_field(p, ak[half], phi, s, K[s]);
        for (size_t n = 0; n < V; ++n) {
            double f = phi[0][n], x = phi[1][n];
            double dFq0 = -kV * f * x * x, dFq1 = -kV * f * f * x;
            pi[0][n] += 0.5 * h * K[0][n];
            pi[1][n] += 0.5 * h * K[1][n];
            dpi[0][n] += 0.5 * h * (J[0][n] + dFq0 * dq);
            dpi[1][n] += 0.5 * h * (J[1][n] + dFq1 * dq);
        }
        if (half == 0) {
            for (int s = 0; s < 2; ++s)
                for (size_t n = 0; n < V; ++n) {
                    phi[s][n] += dr * pi[s][n];
                    dphi[s][n] += dr * dpi[s][n];
                }
        }
    }
    free(lap); free(J[0]); free(J[1]); free(K[0]); free(K[1]);
    return 0;
}

/* Pull the adjoint (lphi, lpi) of the state after one VV2 step from time t
 * back to the state before it.  (phi_n, pi_n) is the state before the step
 * (unchanged).  *dq accumulates the coupling sensitivity of the step. */
int orc_vv2_adjoint_step(const orc_params *p, double t, double *const *phi_n, double *const *pi_n,
                         double *const *lphi, double *const *lpi, double *dq)
{
    if (check_adj(p)) return -2;
    size_t V = vol(p->N);
    double h = p->dt, al = p->alpha;
    double a0 = adj_a(p, t), a1 = adj_a(p, t + h), am = adj_a(p, t + 0.5 * h);
    double kL0 = pow(a0, 1.0 + al), kV0 = pow(a0, 3.0 + al), kL1 = pow(a1, 1.0 + al), kV1 = pow(a1, 3.0 + al);
    double dr = h * pow(am, al - 3.0);
    double *lap = (double *)malloc(V * sizeof(double));
    double *J[2] = {(double *)malloc(V * sizeof(double)), (double *)malloc(V * sizeof(double))};
    double *ph1[2] = {(double *)malloc(V * sizeof(double)), (double *)malloc(V * sizeof(double))};
    double *pi1[2] = {(double *)malloc(V * sizeof(double)), (double *)malloc(V * sizeof(double))};
    /* positions after the step: phi_{n+1} = phi_n + h d (pi_n + h/2 K(a_n, phi_n)) */
    for (int s = 0; s < 2; ++s) {
        memcpy(ph1[s], phi_n[s], V * sizeof(double));
        memcpy(pi1[s], pi_n[s], V * sizeof(double));
    }
    {
        stepper st;
        st.p = p; st.phi = ph1; st.pi = pi1; st.K[0] = J[0]; st.K[1] = J[1];
        kick(&st, a0, 0.5 * h);
        drift(&st, am, h);
    }
    /* second half kick: lphi += h/2 dK(a_{n+1}, phi_{n+1})^T lpi */
    *dq += 0.5 * h * kV1 * dot_dFdq(p, ph1, lpi);
    jac_F_T(p, ph1, lpi, J, lap, kL1, kV1);
    for (int s = 0; s < 2; ++s)
        for (size_t n = 0; n < V; ++n) lphi[s][n] += 0.5 * h * J[s][n];
    /* drift: lpi += h d lphi */
    for (int s = 0; s < 2; ++s)
        for (size_t n = 0; n < V; ++n) lpi[s][n] += dr * lphi[s][n];
    /* first half kick: lphi += h/2 dK(a_n, phi_n)^T lpi */
    *dq += 0.5 * h * kV0 * dot_dFdq(p, phi_n, lpi);
    jac_F_T(p, phi_n, lpi, J, lap, kL0, kV0);
    for (int s = 0; s < 2; ++s)
        for (size_t n = 0; n < V; ++n) lphi[s][n] += 0.5 * h * J[s][n];
    free(lap); free(J[0]); free(J[1]);
    free(ph1[0]); free(ph1[1]); free(pi1[0]); free(pi1[1]);
    return 0;
}

/* Observable: fraction of the energy in field f (0 phi, 1 chi),
 * O = (E_K^f + E_G^f)/rho at scale factor a (E_K = <pi^2>/(2 a^6),
 * E_G = <|grad phi|^2>/(2 a^2)).  Writes O and, if seeds are given,
 * dO/dphi_s(n), dO/dpi_s(n) and the explicit dO/dq. */
static double observable(const orc_params *p, double a, int f, double *const *phi, double *const *pi,
                         double **gphi, double **gpi, double *dOdq_explicit)
{
    size_t V = vol(p->N);
    energies E = energies_of(p, phi, pi, a);
    const double ia2 = 1.0 / (a * a), ia6 = ia2 * ia2 * ia2;
    double rho = rho_tot(&E);
    double X = E.EK[f] + E.EG[f];
    double O = X / rho;
    if (gphi) {
        double *lap = (double *)malloc(V * sizeof(double));
        double inv = 1.0 / ((double)V * rho);
        for (int s = 0; s < 2; ++s) {
            double wX = s == f ? 1.0 : 0.0;   /* d X / d(field s) weight */
            orc_laplacian(p->N, p->dx, phi[s], lap);
            for (size_t n = 0; n < V; ++n) {
                double dV = pot_deriv(p, s, phi[0][n], phi[1][n]);
                /* dE_G^s/dphi_s(n) = -Lap phi_s / (a^2 V) ; dE_V/dphi_s = dV/dphi_s / V */
                double dX = wX * (-lap[n]) * ia2;
                double drho = -lap[n] * ia2 + dV;
                gphi[s][n] = (dX - O * drho) * inv;
                gpi[s][n] = (wX * pi[s][n] - O * pi[s][n]) * ia6 * inv;
            }
        }
        free(lap);
        nsum kq = {0, 0};                                 /* dE_V/dq = <phi^2 chi^2 / 2> */
        for (size_t n = 0; n < V; ++n) nadd(&kq, 0.5 * phi[0][n] * phi[0][n] * phi[1][n] * phi[1][n]);
        *dOdq_explicit = -O * (nval(&kq) / (double)V) / rho;
    }
    return O;
}

int orc_observable(const orc_params *p, double *const *phi, double *const *pi, double *O,
                   double *const *gphi, double *const *gpi, double *dOdq)
{
    if (check_adj(p)) return -2;
    double d = 0.0;
    *O = observable(p, 1.0, 1, phi, pi, (double **)gphi, (double **)gpi, gphi ? &d : NULL);
    if (dOdq) *dOdq = d;
    return 0;
}

/* Observables the reverse sweep can start from: the energy fraction of one
 * field above, or one bin of the power spectrum of one field (defined with the
 * spectrum). */
enum { ORC_OBS_ENERGY_FRACTION = 0, ORC_OBS_SPECTRUM_BIN = 1 };
static double observable_kind(const orc_params *p, double a, int kind, int field, int bin, double *const *phi,
                              double *const *pi, double **gphi, double **gpi, double *dq);

/* Gradient of O(final state) of observable `kind` with respect to the initial
 * phi, pi and q for nsteps VV2 steps from time t_start, by reverse sweep with
 * segment recomputation: checkpoints every ceil(sqrt(nsteps)) steps, each
 * segment re-run forward from its checkpoint and stored, then pulled back step
 * by step. */
int orc_adjoint_vv2_kind(const orc_params *p, double t_start, int kind, int field, int bin, double *const *phi0,
                         double *const *pi0, long nsteps, double *O_out, double *const *gphi, double *const *gpi,
                         double *dOdq)
{
    if (check_adj(p)) return -2;
    if (kind != ORC_OBS_ENERGY_FRACTION && kind != ORC_OBS_SPECTRUM_BIN) return -1;
    if (field < 0 || field > 1 || (kind == ORC_OBS_SPECTRUM_BIN && bin < 1)) return -1;
    if (nsteps < 0) return -1;
    size_t V = vol(p->N), B = V * sizeof(double);
    long k = 1;
    while (k * k < nsteps) ++k;
    long ncp = nsteps / k + 1;
    double *cp = (double *)malloc((size_t)ncp * 4 * B);   /* phi0, phi1, pi0, pi1 per checkpoint */
    double *cur[4];
    for (int i = 0; i < 4; ++i) cur[i] = (double *)malloc(B);
    memcpy(cur[0], phi0[0], B); memcpy(cur[1], phi0[1], B);
    memcpy(cur[2], pi0[0], B);  memcpy(cur[3], pi0[1], B);
    orc_params pv = *p;
    pv.integrator = ORC_VV2;
    for (long n = 0; n <= nsteps; ++n) {
        if (n % k == 0)
            for (int i = 0; i < 4; ++i) memcpy(cp + ((size_t)(n / k) * 4 + i) * V, cur[i], B);
        if (n == nsteps) break;
        double tn = t_start + (double)n * p->dt;
        orc_clock c = {tn, adj_a(p, tn), 0, 0, 0};
        orc_run(&pv, cur, cur + 2, &c, 1);
    }
    /* seed at the final state */
    double *lphi[2] = {gphi[0], gphi[1]}, *lpi[2] = {gpi[0], gpi[1]};
    double q_acc = 0.0;
    *O_out = observable_kind(p, adj_a(p, t_start + (double)nsteps * p->dt), kind, field, bin, cur, cur + 2, lphi,
                             lpi, &q_acc);
    /* segment states: positions and momenta at steps s0..s1 */
    double *seg = (double *)malloc((size_t)(k + 1) * 4 * B);
    for (long s0 = ((nsteps - 1) / k) * k; nsteps > 0 && s0 >= 0; s0 -= k) {
        long s1 = s0 + k < nsteps ? s0 + k : nsteps;
        for (int i = 0; i < 4; ++i) memcpy(cur[i], cp + ((size_t)(s0 / k) * 4 + i) * V, B);
        for (long n = s0; n < s1; ++n) {
            for (int i = 0; i < 4; ++i) memcpy(seg + ((size_t)(n - s0) * 4 + i) * V, cur[i], B);
            double tn = t_start + (double)n * p->dt;
            orc_clock c = {tn, adj_a(p, tn), 0, 0, 0};
            orc_run(&pv, cur, cur + 2, &c, 1);
        }
        for (long n = s1 - 1; n >= s0; --n) {
            double *sp[2] = {seg + ((size_t)(n - s0) * 4 + 0) * V, seg + ((size_t)(n - s0) * 4 + 1) * V};
            double *sm[2] = {seg + ((size_t)(n - s0) * 4 + 2) * V, seg + ((size_t)(n - s0) * 4 + 3) * V};
            orc_vv2_adjoint_step(p, t_start + (double)n * p->dt, sp, sm, lphi, lpi, &q_acc);
        }
    }
    *dOdq = q_acc;
    free(seg);
    free(cp);
    for (int i = 0; i < 4; ++i) free(cur[i]);
    return 0;
}

int orc_adjoint_vv2(const orc_params *p, double *const *phi0, double *const *pi0, long nsteps,
                    double *O_out, double *const *gphi, double *const *gpi, double *dOdq)
{
    return orc_adjoint_vv2_kind(p, 0.0, ORC_OBS_ENERGY_FRACTION, 1, 0, phi0, pi0, nsteps, O_out, gphi, gpi, dOdq);
}

/* ------------------------------------------------------------------ */
/* Adjoint of the VV2 map with the self-consistent expansion (reading  */
/* R1), two fields.  One step from (phi_n, pi_n, a_n, b_n):             */
/*  (1) pi'  = pi_n + h/2 K(a_n, phi_n)                                  */
/*  (2) b'   = b_n + h/2 K_a(a_n, E(phi_n, pi_n, a_n))                   */
/*  (3) a1   = a_n + h b'                                                */
/*  (4) phi1 = phi_n + h abar^{alpha-3} pi',  abar = (a_n + a1)/2        */
/*  (5) pi1  = pi' + h/2 K(a1, phi1)                                     */
/*  (6) b1   = b' + h/2 K_a(a1, E(phi1, pi1, a1))                        */
/* with K_a(a, E) = C(a) Q, C = a^{2 alpha+1} kappa^2/3,                 */
/* Q = (alpha-2) E_K + alpha E_G + (alpha+1) E_V.  The adjoint pulls    */
/* (lphi, lpi, la, lb) back through (6) ... (1) in that order.           */
/* ------------------------------------------------------------------ */

/* Adds w dK_a/dphi_s(n) to gphi and w dK_a/dpi_s(n) to gpi at (a, phi, pi);
 * returns dK_a/da at fixed fields and sets *dkq = dK_a/dq:
 *   dE_G/dphi_s = -Lap phi_s/(a^2 V), dE_V/dphi_s = dV/dphi_s / V,
 *   dE_K/dpi_s = pi_s/(a^6 V), dE_K/da = -6 E_K/a, dE_G/da = -2 E_G/a,
 *   dE_V/dq = <phi^2 chi^2/2>. */
static double kernel_a_pullback(const orc_params *p, double a, double *const *phi, double *const *pi, double w,
                                double **gphi, double **gpi, double *dkq)
{
    size_t V = vol(p->N);
    double al = p->alpha;
    energies E = energies_of(p, phi, pi, a);
    double C = pow(a, 2.0 * al + 1.0) / 3.0 * p->kappa2;
    double Q = (al - 2.0) * EK_tot(&E) + al * EG_tot(&E) + (al + 1.0) * EV_tot(&E);
    double *lap = (double *)malloc(V * sizeof(double));
    for (int s = 0; s < 2; ++s) {
        orc_laplacian(p->N, p->dx, phi[s], lap);
        for (size_t n = 0; n < V; ++n) {
            double dV = pot_deriv(p, s, phi[0][n], phi[1][n]);
            gphi[s][n] += w * C * (al * (-lap[n]) / (a * a * (double)V) + (al + 1.0) * dV / (double)V);
            gpi[s][n] += w * C * (al - 2.0) * pi[s][n] / (pow(a, 6.0) * (double)V);
        }
    }
    free(lap);
    nsum kq = {0, 0};
    for (size_t n = 0; n < V; ++n) nadd(&kq, 0.5 * phi[0][n] * phi[0][n] * phi[1][n] * phi[1][n]);
    *dkq = C * (al + 1.0) * nval(&kq) / (double)V;
    return (2.0 * al + 1.0) * C * Q / a + C * ((al - 2.0) * (-6.0) * EK_tot(&E) / a + al * (-2.0) * EG_tot(&E) / a);
}

/* sum_n l . dK/da at (a, phi):  dK_s/da = (1+alpha) a^alpha Lap phi_s - (3+alpha) a^{2+alpha} dV/dphi_s */
static double kernel_da_dot(const orc_params *p, double a, double *const *phi, double *const *l)
{
    size_t V = vol(p->N);
    double al = p->alpha;
    double *lap = (double *)malloc(V * sizeof(double));
    nsum k = {0, 0};
    for (int s = 0; s < 2; ++s) {
        orc_laplacian(p->N, p->dx, phi[s], lap);
        for (size_t n = 0; n < V; ++n)
            nadd(&k, l[s][n] * ((1.0 + al) * pow(a, al) * lap[n] -
                                (3.0 + al) * pow(a, 2.0 + al) * pot_deriv(p, s, phi[0][n], phi[1][n])));
    }
    free(lap);
    return nval(&k);
}

/* Pull (lphi, lpi, *la, *lb) back through one self-consistent VV2 step from
 * the state (phi_n, pi_n, a_n, b_n) (unchanged); *dq accumulates. */
static void self_adjoint_step(const orc_params *p, double *const *phi_n, double *const *pi_n, double a_n,
                              double b_n, double **lphi, double **lpi, double *la, double *lb, double *dq)
{
    size_t V = vol(p->N), B = V * sizeof(double);
    double h = p->dt, al = p->alpha;
    double *pp[2], *ph1[2], *pi1[2], *J[2], *K[2];
    for (int s = 0; s < 2; ++s) {
        pp[s] = (double *)malloc(B);
        ph1[s] = (double *)malloc(B);
        pi1[s] = (double *)malloc(B);
        J[s] = (double *)malloc(B);
        K[s] = (double *)malloc(B);
    }
    double *lap = (double *)malloc(B);
    /* forward intermediates */
    energies En = energies_of(p, phi_n, pi_n, a_n);
    double bh = b_n + 0.5 * h * kernel_a(p, a_n, &En);
    double a1 = a_n + h * bh, abar = 0.5 * (a_n + a1);
    double dr = h * pow(abar, al - 3.0);
    for (int s = 0; s < 2; ++s) kernel_field(p, a_n, phi_n, s, K[s]);
    for (int s = 0; s < 2; ++s)
        for (size_t n = 0; n < V; ++n) {
            pp[s][n] = pi_n[s][n] + 0.5 * h * K[s][n];
            ph1[s][n] = phi_n[s][n] + dr * pp[s][n];
        }
    for (int s = 0; s < 2; ++s) kernel_field(p, a1, ph1, s, K[s]);
    for (int s = 0; s < 2; ++s)
        for (size_t n = 0; n < V; ++n) pi1[s][n] = pp[s][n] + 0.5 * h * K[s][n];
    double kL0 = pow(a_n, 1.0 + al), kV0 = pow(a_n, 3.0 + al), kL1 = pow(a1, 1.0 + al), kV1 = pow(a1, 3.0 + al);
    double la1 = *la, la0 = 0.0, dkq;
    /* (6) b1 = b' + h/2 K_a(a1, E(phi1, pi1, a1)) */
    double g6 = 0.5 * h * (*lb);
    la1 += g6 * kernel_a_pullback(p, a1, ph1, pi1, g6, lphi, lpi, &dkq);
    *dq += g6 * dkq;
    /* (5) pi1 = pi' + h/2 K(a1, phi1) */
    la1 += 0.5 * h * kernel_da_dot(p, a1, ph1, lpi);
    *dq += 0.5 * h * kV1 * dot_dFdq(p, ph1, lpi);
    jac_F_T(p, ph1, lpi, J, lap, kL1, kV1);
    for (int s = 0; s < 2; ++s)
        for (size_t n = 0; n < V; ++n) lphi[s][n] += 0.5 * h * J[s][n];
    /* (4) phi1 = phi_n + h abar^{alpha-3} pi' */
    nsum kd = {0, 0};
    for (int s = 0; s < 2; ++s)
        for (size_t n = 0; n < V; ++n) nadd(&kd, lphi[s][n] * pp[s][n]);
    double labar = h * (al - 3.0) * pow(abar, al - 4.0) * nval(&kd);
    for (int s = 0; s < 2; ++s)
        for (size_t n = 0; n < V; ++n) lpi[s][n] += dr * lphi[s][n];
    la1 += 0.5 * labar;
    la0 += 0.5 * labar;
    /* (3) a1 = a_n + h b' */
    la0 += la1;
    *lb += h * la1;
    /* (1) pi' = pi_n + h/2 K(a_n, phi_n), with lpi = the adjoint of pi' */
    la0 += 0.5 * h * kernel_da_dot(p, a_n, phi_n, lpi);
    *dq += 0.5 * h * kV0 * dot_dFdq(p, phi_n, lpi);
    jac_F_T(p, phi_n, lpi, J, lap, kL0, kV0);
    for (int s = 0; s < 2; ++s)
        for (size_t n = 0; n < V; ++n) lphi[s][n] += 0.5 * h * J[s][n];
    /* (2) b' = b_n + h/2 K_a(a_n, E(phi_n, pi_n, a_n)): direct terms of pi_n and phi_n */
    double g2 = 0.5 * h * (*lb);
    la0 += g2 * kernel_a_pullback(p, a_n, phi_n, pi_n, g2, lphi, lpi, &dkq);
    *dq += g2 * dkq;
    *la = la0;
    for (int s = 0; s < 2; ++s) {
        free(pp[s]);
        free(ph1[s]);
        free(pi1[s]);
        free(J[s]);
        free(K[s]);
    }
    free(lap);
}

/* dO/da at fixed fields for the energy fraction of field f:
 * O = X/rho, dX/da = -(6 E_K^f + 2 E_G^f)/a, drho/da = -(6 E_K + 2 E_G)/a. */
static double energy_fraction_da(const orc_params *p, double a, int f, double *const *phi, double *const *pi)
{
    energies E = energies_of(p, phi, pi, a);
    double rho = rho_tot(&E), O = (E.EK[f] + E.EG[f]) / rho;
    double dX = -(6.0 * E.EK[f] + 2.0 * E.EG[f]) / a, drho = -(6.0 * EK_tot(&E) + 2.0 * EG_tot(&E)) / a;
    return (dX - O * drho) / rho;
}

/* Gradient of O(final state) of observable `kind` after nsteps self-consistent
 * VV2 steps from (phi0, pi0, a0, b0), with respect to phi0, pi0, q, a0 and b0
 * (b0 an independent input here).  Every step's state is stored; the reverse
 * sweep pulls the adjoint back step by step. */
int orc_adjoint_vv2_self(const orc_params *p, int kind, int field, int bin, double *const *phi0, double *const *pi0,
                         double a0, double b0, long nsteps, double *O_out, double *const *gphi, double *const *gpi,
                         double *dOdq, double *dOda0, double *dOdb0)
{
    if (p->nfields != 2 || p->potential != ORC_PHI4_CHI2 || p->expansion != ORC_SELF) return -2;
    if (kind != ORC_OBS_ENERGY_FRACTION && kind != ORC_OBS_SPECTRUM_BIN) return -1;
    if (field < 0 || field > 1 || (kind == ORC_OBS_SPECTRUM_BIN && bin < 1)) return -1;
    if (nsteps < 0 || !(a0 > 0.0)) return -1;
    size_t V = vol(p->N), B = V * sizeof(double);
    double *st = (double *)malloc((size_t)(nsteps + 1) * 4 * B);
    double *ab = (double *)malloc((size_t)(nsteps + 1) * 2 * sizeof(double));
    double *cur[4];
    for (int i = 0; i < 4; ++i) cur[i] = st + (size_t)i * V;
    memcpy(cur[0], phi0[0], B); memcpy(cur[1], phi0[1], B);
    memcpy(cur[2], pi0[0], B);  memcpy(cur[3], pi0[1], B);
    orc_params pv = *p;
    pv.integrator = ORC_VV2;
    orc_clock c = {0.0, a0, b0, 0, 0};
    ab[0] = a0;
    ab[1] = b0;
    for (long n = 0; n < nsteps; ++n) {
        double *nx[4];
        for (int i = 0; i < 4; ++i) {
            nx[i] = st + ((size_t)(n + 1) * 4 + i) * V;
            memcpy(nx[i], st + ((size_t)n * 4 + i) * V, B);
        }
        orc_run(&pv, nx, nx + 2, &c, 1);
        ab[2 * (n + 1)] = c.a;
        ab[2 * (n + 1) + 1] = c.b;
    }
    double *fin[4];
    for (int i = 0; i < 4; ++i) fin[i] = st + ((size_t)nsteps * 4 + i) * V;
    double *lphi[2] = {gphi[0], gphi[1]}, *lpi[2] = {gpi[0], gpi[1]};
    double q_acc = 0.0, aT = ab[2 * nsteps];
    *O_out = observable_kind(p, aT, kind, field, bin, fin, fin + 2, lphi, lpi, &q_acc);
    double la = kind == ORC_OBS_ENERGY_FRACTION ? energy_fraction_da(p, aT, field, fin, fin + 2) : 0.0;
    double lb = 0.0;
    for (long n = nsteps - 1; n >= 0; --n) {
        double *sp[2] = {st + ((size_t)n * 4 + 0) * V, st + ((size_t)n * 4 + 1) * V};
        double *sm[2] = {st + ((size_t)n * 4 + 2) * V, st + ((size_t)n * 4 + 3) * V};
        self_adjoint_step(p, sp, sm, ab[2 * n], ab[2 * n + 1], lphi, lpi, &la, &lb, &q_acc);
    }
    *dOdq = q_acc;
    *dOda0 = la;
    *dOdb0 = lb;
    free(st);
    free(ab);
    return 0;
}

/* ------------------------------------------------------------------ */
/* U(1) sector: complex scalar + Abelian links, a = 1 (sec. 3.2 U(1)   */
/* toolkit, sec. 5.2 equations of motion, sec. 5.5.2 kernels; reading R5) */
/* phi = (phi0 + i phi1)/sqrt(2); psi = phi0 + i phi1 = sqrt(2) phi.     */
/* links V_i = exp(-i e dx A_i); plaquette angle                        */
/*   theta_ij(n) = e dx [A_j(n+i) - A_j(n) - A_i(n+j) + A_i(n)]           */
/* V = lambda/4 (|phi|^2 - v^2)^2, |phi|^2 = (phi0^2 + phi1^2)/2         */
/* ------------------------------------------------------------------ */

typedef struct orc_u1_params {
    int32_t N;
    int32_t expansion;                      /* ORC_NONE, ORC_FIXED, ORC_SELF (as for the scalars) */
    double dx, dt, lambda, v, e, kappa_g;   /* kappa_g = (f_star/omega_star)^2 */
    double alpha, kappa2;                   /* alpha-time exponent; (f_star/m_p)^2 */
    double w_eos, H0, t0, a0;               /* fixed background (eq. ScaleFactorPowerLaw); SELF: a0 */
} orc_u1_params;

/* U(1) sector in an expanding background (sec. 5.5.2, reading U1).  With
 * pi = a^{3-alpha} phi' and pi_A = a^{1-alpha} F_0i (eqs. momU1singlet,
 * momU1vec) the kernels of eq. kernelcomplexscalar and the one after it are
 * the a = 1 forces with each term scaled:
 *   K_phi = a^{1+alpha} (covariant Laplacian) - a^{3+alpha} (potential force),
 *   K_A   = a^{1+alpha} kappa_g J - a^{alpha-1} (magnetic force),
 * and the drifts are phi' = a^{alpha-3} pi, A_i' = a^{alpha-1} pi_A (eqs.
 * momU1singlet, momU1vec with A_0 = 0).  The energies of eq. energy-contrib in
 * these variables are the a = 1 ones divided by a^6 (scalar kinetic), a^2
 * (scalar gradient) and a^4 (electric, magnetic); the scale-factor kernel adds
 * (alpha - 1)(E_K^A + E_G^A) (the b' equation of sec. 5.5.2).  The Gauss law
 * (eq. GaussU1-eom) in these variables, div pi_A = 2 e kappa_g Im(phi* pi),
 * carries no power of a, and the kicks keep it exactly for any a.  Kicks and
 * drifts take a at the kick time and at the drift midpoint (fixed background,
 * reading R3), or follow readings R1 (velocity-Verlet) and A3 (leapfrog) with
 * self-consistent expansion. */

static void u1_fixed_ab(const orc_u1_params *p, double t, double *a, double *b)
{
    double pw = 2.0 / (3.0 * (1.0 + p->w_eos) - 2.0 * p->alpha);
    double u = 1.0 + p->H0 * (t - p->t0) / pw;
    *a = p->a0 * pow(u, pw);
    *b = p->a0 * p->H0 * pow(u, pw - 1.0);
}

int orc_u1_fixed_background(const orc_u1_params *p, double t, double *a, double *b)
{
    u1_fixed_ab(p, t, a, b);
    return 0;
}

static double theta(const orc_u1_params *p, double *const *A, int x, int y, int z, int i, int j)
{
    int N = p->N;
    return p->e * p->dx *
           (A[j][nbr(N, x, y, z, i, +1)] - A[j][at(N, x, y, z)] - A[i][nbr(N, x, y, z, j, +1)] +
            A[i][at(N, x, y, z)]);
}

/* forces = minus the derivative of the lattice Hamiltonian (at scale factor a):
 *   Fphi_c = a^{1+alpha} {Re,Im}(D^2 psi) - a^{3+alpha} lambda/2 (|phi|^2 - v^2) phi_c
 *   FA_i   = a^{1+alpha} kappa_g J_i
 *            - a^{alpha-1} (e dx^3)^-1 sum_{j != i} [sin theta_ij(n) - sin theta_ij(n-j)]
 *   J_i    = (e/dx) Im[ conj(psi(n)) V_i(n) psi(n+i) ]                       */
static int u1_forces_a(const orc_u1_params *p, double a, double *const *phi, double *const *A,
                       double *const *Fphi, double *const *FA)
{
    int N = p->N;
    double dx = p->dx, e = p->e;
    double cl = pow(a, 1.0 + p->alpha), cv = pow(a, 3.0 + p->alpha), cm_ = pow(a, p->alpha - 1.0);
    #pragma omp parallel for schedule(static)
    for (int z = 0; z < N; ++z)
        for (int y = 0; y < N; ++y)
            for (int x = 0; x < N; ++x) {
                size_t n = at(N, x, y, z);
                double pr = phi[0][n], pim = phi[1][n];
                double dre = 0.0, dim = 0.0;
                for (int i = 0; i < 3; ++i) {
                    size_t np = nbr(N, x, y, z, i, +1), nm = nbr(N, x, y, z, i, -1);
                    double cp = cos(e * dx * A[i][n]), sp = -sin(e * dx * A[i][n]);   /* V_i(n)   */
                    double cm = cos(e * dx * A[i][nm]), sm = sin(e * dx * A[i][nm]);  /* V_i(n-i)* */
                    /* V_i(n) psi(n+i) */
                    double ar = cp * phi[0][np] - sp * phi[1][np];
                    double ai = cp * phi[1][np] + sp * phi[0][np];
                    /* conj(V_i(n-i)) psi(n-i) */
                    double br = cm * phi[0][nm] - sm * phi[1][nm];
                    double bi = cm * phi[1][nm] + sm * phi[0][nm];
                    dre += ar - 2.0 * pr + br;
                    dim += ai - 2.0 * pim + bi;
                    /* current: Im[conj(psi) V psi(n+i)] = pr*ai - pim*ar */
                    double J = e / dx * (pr * ai - pim * ar);
                    double mag = 0.0;
                    for (int j = 0; j < 3; ++j) {
                        if (j == i) continue;
                        int c[3] = {x, y, z};
                        c[j] = dn(c[j], N);
                        mag += sin(theta(p, A, x, y, z, i, j)) - sin(theta(p, A, c[0], c[1], c[2], i, j));
                    }
                    FA[i][n] = cl * (p->kappa_g * J) - cm_ * (mag / (e * dx * dx * dx));
                }
                double m2 = 0.5 * (pr * pr + pim * pim);
                double vp = 0.5 * p->lambda * (m2 - p->v * p->v);
                Fphi[0][n] = cl * (dre / (dx * dx)) - cv * (vp * pr);
                Fphi[1][n] = cl * (dim / (dx * dx)) - cv * (vp * pim);
            }
    return 0;
}

int orc_u1_forces(const orc_u1_params *p, double *const *phi, double *const *A,
                  double *const *Fphi, double *const *FA)
{
    return u1_forces_a(p, 1.0, phi, A, Fphi, FA);
}

int orc_u1_forces_at(const orc_u1_params *p, double a, double *const *phi, double *const *A,
                     double *const *Fphi, double *const *FA)
{
    return u1_forces_a(p, a, phi, A, Fphi, FA);
}

/* U(1) energies and Gauss constraint. Output layout (12 doubles):
 *  [0] E_K^phi = <(pi0^2+pi1^2)/2>, [1] E_G^phi = <sum_i |V_i psi(n+i) - psi(n)|^2>/(2 dx^2),
 *  [2] E_V = <lambda/4 (|phi|^2-v^2)^2>, [3] E_K^A = <sum_i piA_i^2>/(2 kappa_g),
 *  [4] E_G^A = <sum_{i<j} (1 - cos theta_ij)>/(kappa_g e^2 dx^4), [5] rho,
 *  [6] max|G|, [7] max|div piA|, [8] max|charge|, [9] <|G|>, [10] <|div piA + charge|>
 *  with G = div^- piA - e kappa_g (phi0 pi1 - phi1 pi0) (eq. GaussU1-eom, a = 1)
 *  [11] <|div piA| + |charge|>.
 * Leapfrog momenta are synchronised on copies when lf_stag != 0. */
static void u1_energy_plain(const orc_u1_params *p, double a, double *const *phi, double *const *pi,
                            double *const *A, double *const *piA, double *out)
{
    int N = p->N;
    size_t V = vol(N);
    double dx = p->dx, e = p->e;
    nsum sk = {0, 0}, sg = {0, 0}, sv = {0, 0}, ska = {0, 0}, sga = {0, 0};
    nsum sG = {0, 0}, sLR = {0, 0}, sLRabs = {0, 0};
    double gmax = 0, dmax = 0, cmax = 0;
    for (int z = 0; z < N; ++z)
        for (int y = 0; y < N; ++y)
            for (int x = 0; x < N; ++x) {
                size_t n = at(N, x, y, z);
                nadd(&sk, 0.5 * (pi[0][n] * pi[0][n] + pi[1][n] * pi[1][n]));
                double g = 0.0, ka = 0.0, div = 0.0;
                for (int i = 0; i < 3; ++i) {
                    size_t np = nbr(N, x, y, z, i, +1), nm = nbr(N, x, y, z, i, -1);
                    double c = cos(e * dx * A[i][n]), s = -sin(e * dx * A[i][n]);
                    double ar = c * phi[0][np] - s * phi[1][np];
                    double ai = c * phi[1][np] + s * phi[0][np];
                    double dr = ar - phi[0][n], di = ai - phi[1][n];
                    g += dr * dr + di * di;
                    ka += piA[i][n] * piA[i][n];
                    div += (piA[i][n] - piA[i][nm]) / dx;
                }
                nadd(&sg, g / (2.0 * dx * dx));
                double m2 = 0.5 * (phi[0][n] * phi[0][n] + phi[1][n] * phi[1][n]);
                double u = m2 - p->v * p->v;
                nadd(&sv, 0.25 * p->lambda * u * u);
                nadd(&ska, ka / (2.0 * p->kappa_g));
                /* 1 - cos(theta) written as 2 sin^2(theta/2): the same quantity without
                   the cancellation that loses all digits for small plaquette angles */
                double mag = 0.0;
                for (int i = 0; i < 3; ++i)
                    for (int j = i + 1; j < 3; ++j) {
                        double sh = sin(0.5 * theta(p, A, x, y, z, i, j));
                        mag += 2.0 * sh * sh;
                    }
                nadd(&sga, mag / (p->kappa_g * e * e * dx * dx * dx * dx));
                double charge = e * p->kappa_g * (phi[0][n] * pi[1][n] - phi[1][n] * pi[0][n]);
                double G = div - charge;
                if (fabs(G) > gmax) gmax = fabs(G);
                if (fabs(div) > dmax) dmax = fabs(div);
                if (fabs(charge) > cmax) cmax = fabs(charge);
                nadd(&sG, fabs(G));
                nadd(&sLR, fabs(div + charge));
                nadd(&sLRabs, fabs(div) + fabs(charge));
            }
    const double a2 = a * a, a4 = a2 * a2, a6 = a4 * a2;
    out[0] = nval(&sk) / (double)V / a6;
    out[1] = nval(&sg) / (double)V / a2;
    out[2] = nval(&sv) / (double)V;
    out[3] = nval(&ska) / (double)V / a4;
    out[4] = nval(&sga) / (double)V / a4;
    out[5] = out[0] + out[1] + out[2] + out[3] + out[4];
    out[6] = gmax;
    out[7] = dmax;
    out[8] = cmax;
    out[9] = nval(&sG) / (double)V;
    out[10] = nval(&sLR) / (double)V;
    out[11] = nval(&sLRabs) / (double)V;
}

/* kernel of b with the gauge energies (sec. 5.5.2):
 *   K_a = a^{2 alpha + 1}/3 kappa^2 [(alpha-2) E_K^phi + alpha E_G^phi
 *         + (alpha-1)(E_K^A + E_G^A) + (alpha+1) E_V]   (energies as u1_energy_plain) */
static double u1_kernel_a(const orc_u1_params *p, double a, const double *E)
{
    double al = p->alpha;
    return pow(a, 2.0 * al + 1.0) / 3.0 * p->kappa2 *
           ((al - 2.0) * E[0] + al * E[1] + (al - 1.0) * (E[3] + E[4]) + (al + 1.0) * E[2]);
}

static void u1_kick(const orc_u1_params *p, double a, double *const *phi, double *const *pi,
                    double *const *A, double *const *piA, double w)
{
    size_t V = vol(p->N);
    double *F[5];
    for (int i = 0; i < 5; ++i) F[i] = (double *)malloc(V * sizeof(double));
    u1_forces_a(p, a, phi, A, F, F + 2);
    #pragma omp parallel for schedule(static)
    for (size_t n = 0; n < V; ++n) {
        pi[0][n] += w * F[0][n];
        pi[1][n] += w * F[1][n];
        for (int i = 0; i < 3; ++i) piA[i][n] += w * F[2 + i][n];
    }
    for (int i = 0; i < 5; ++i) free(F[i]);
}

/* Energies at integer time, output layout (17 doubles): [0 .. 11] as
 * u1_energy_plain at the clock's a; [12] a, [13] b at integer time,
 * [14] Hubble LHS b^2, [15] RHS a^{2 alpha + 2} kappa^2 rho / 3, [16] (LHS - RHS)/(LHS + RHS).
 * Leapfrog momenta (and b with self-consistent expansion) are synchronised on
 * copies (readings R4, A3). */
int orc_u1_energy(const orc_u1_params *p, double *const *phi, double *const *pi,
                  double *const *A, double *const *piA, const orc_clock *c, double *out)
{
    size_t V = vol(p->N), B = V * sizeof(double);
    double *ps[2], *pa[3];
    for (int i = 0; i < 2; ++i) { ps[i] = (double *)malloc(B); memcpy(ps[i], pi[i], B); }
    for (int i = 0; i < 3; ++i) { pa[i] = (double *)malloc(B); memcpy(pa[i], piA[i], B); }
    double b = c->b;
    if (c->lf_stag != 0) {
        double w = 0.5 * c->lf_stag * p->dt;
        if (p->expansion == ORC_SELF) {
            double E[12];
            u1_energy_plain(p, c->a, phi, ps, A, pa, E);
            b += w * u1_kernel_a(p, c->a, E);
        }
        u1_kick(p, c->a, phi, ps, A, pa, w);
    }
    u1_energy_plain(p, c->a, phi, ps, A, pa, out);
    for (int i = 0; i < 2; ++i) free(ps[i]);
    for (int i = 0; i < 3; ++i) free(pa[i]);
    double lhs = b * b, rhs = pow(c->a, 2.0 * p->alpha + 2.0) * p->kappa2 * out[5] / 3.0;
    out[12] = c->a;
    out[13] = b;
    out[14] = lhs;
    out[15] = rhs;
    out[16] = (lhs + rhs) != 0.0 ? (lhs - rhs) / (lhs + rhs) : 0.0;
    return 0;
}

/* Gauss residual of the stored (un-synchronised) pairing, same layout [6..11]. */
int orc_u1_gauss(const orc_u1_params *p, double *const *phi, double *const *pi,
                 double *const *A, double *const *piA, double *out)
{
    u1_energy_plain(p, 1.0, phi, pi, A, piA, out);
    return 0;
}

/* Hubble constraint (eq. FriedmannHubble) for b at the start: b0^2 = a^{2 alpha + 2} kappa^2 rho / 3 */
int orc_u1_hubble_b0(const orc_u1_params *p, double *const *phi, double *const *pi, double *const *A,
                     double *const *piA, double a, double *b0)
{
    double E[12];
    u1_energy_plain(p, a, phi, pi, A, piA, E);
    double rhs = pow(a, 2.0 * p->alpha + 2.0) * p->kappa2 * E[5] / 3.0;
    if (rhs < 0.0) return -1;
    *b0 = sqrt(rhs);
    return 0;
}

static void u1_drift_a(const orc_u1_params *p, double a_mid, double *const *phi, double *const *pi,
                       double *const *A, double *const *piA, double h)
{
    size_t V = vol(p->N);
    double cp = h * pow(a_mid, p->alpha - 3.0), ca = h * pow(a_mid, p->alpha - 1.0);
    #pragma omp parallel for schedule(static)
    for (size_t n = 0; n < V; ++n) {
        phi[0][n] += cp * pi[0][n];
        phi[1][n] += cp * pi[1][n];
        for (int i = 0; i < 3; ++i) A[i][n] += ca * piA[i][n];
    }
}

/* Staggered leapfrog for the U(1) system (a = 1): kick all momenta, then drift
 * phi and A.  Same staggering convention as orc_run. */
int orc_u1_run_lf(const orc_u1_params *p, double *const *phi, double *const *pi,
                  double *const *A, double *const *piA, orc_clock *c, long nsteps)
{
    if (nsteps == 0) return 0;
    int dir = nsteps > 0 ? 1 : -1;
    long ns = nsteps > 0 ? nsteps : -nsteps;
    double h = dir * p->dt;
    if (c->lf_stag != 0 && c->lf_stag != dir) return -3;
    double t_start = c->t;
    for (long k = 0; k < ns; ++k) {
        double t = t_start + (double)k * h;
        double w = c->lf_stag == 0 ? 0.5 * h : h;
        if (p->expansion == ORC_SELF) {
            /* reading A3 with every momentum-dependent energy (E_K^phi, E_K^A) */
            double Eb[12], Ea[12];
            u1_energy_plain(p, c->a, phi, pi, A, piA, Eb);
            u1_kick(p, c->a, phi, pi, A, piA, w);
            u1_energy_plain(p, c->a, phi, pi, A, piA, Ea);
            if (c->lf_stag == 0)
                c->b += w * u1_kernel_a(p, c->a, Ea);
            else
                c->b += 0.5 * h * u1_kernel_a(p, c->a, Eb) + 0.5 * h * u1_kernel_a(p, c->a, Ea);
            double a1 = c->a + h * c->b;
            u1_drift_a(p, 0.5 * (c->a + a1), phi, pi, A, piA, h);
            c->a = a1;
        } else if (p->expansion == ORC_FIXED) {
            double a, b, am;
            u1_fixed_ab(p, t, &a, &b);
            u1_kick(p, a, phi, pi, A, piA, w);
            u1_fixed_ab(p, t + 0.5 * h, &am, &b);
            u1_drift_a(p, am, phi, pi, A, piA, h);
        } else {
            u1_kick(p, 1.0, phi, pi, A, piA, w);
            u1_drift_a(p, 1.0, phi, pi, A, piA, h);
        }
        c->lf_stag = dir;
    }
    c->t = t_start + (double)ns * h;
    if (p->expansion == ORC_FIXED) {
        u1_fixed_ab(p, c->t, &c->a, &c->b);
    } else if (p->expansion == ORC_NONE) {
        c->a = 1.0;
        c->b = 0.0;
    }
    return 0;
}

int orc_u1_lf_sync(const orc_u1_params *p, double *const *phi, double *const *pi,
                   double *const *A, double *const *piA, orc_clock *c)
{
    if (c->lf_stag == 0) return 0;
    double w = 0.5 * c->lf_stag * p->dt;
    if (p->expansion == ORC_SELF) {
        double E[12];
        u1_energy_plain(p, c->a, phi, pi, A, piA, E);
        c->b += w * u1_kernel_a(p, c->a, E);
    }
    u1_kick(p, c->a, phi, pi, A, piA, w);
    c->lf_stag = 0;
    return 0;
}

/* ------------------------------------------------------------------ */
/* Power spectrum (sec. 3.1, eq. discretePS)                           */
/* ------------------------------------------------------------------ */
/* Unnormalised forward DFT f~(n~) = sum_n f(n) exp(-2 pi i n~.n / N), one
 * dimension at a time (plain O(N^4) sums, twiddles indexed by (k j) mod N).
 * Bin b holds the modes with b <= |n~| < b + 1, n~_i in (-N/2, N/2] (bin 0:
 * the zero mode only).  Per bin: the sum of |f~|^2 (compensated), the number
 * of modes and the discrete spectrum of eq. discretePS,
 *   Delta(b) = k_b^3 / (2 pi^2) (dx/N)^3 sum_b / (4 pi b^2),  k_b = b k_IR,
 * k_IR = 2 pi / (N dx), and Delta(0) = 0.  With this normalisation
 * sum_{b >= 1} (k_IR / k_b) Delta(b) = <f^2> - <f>^2 exactly (eq.
 * discretePSII).  Returns the number of bins filled or -1. */
static const double ORC_PI = 3.14159265358979323846;

/* sign -1: forward, sum_j x_j e^{-2 pi i k j/N}; sign +1: unnormalised inverse */
static void dft_axis(int N, double *re, double *im, int axis, const double *cs, const double *sn, int sign)
{
    double *tr = (double *)malloc((size_t)N * sizeof(double));
    double *ti = (double *)malloc((size_t)N * sizeof(double));
    size_t stride = axis == 0 ? 1 : (axis == 1 ? (size_t)N : (size_t)N * N);
    for (int a = 0; a < N; ++a)
        for (int b = 0; b < N; ++b) {
            size_t base;
            if (axis == 0) base = (size_t)N * ((size_t)a + (size_t)N * b);
            else if (axis == 1) base = (size_t)a + (size_t)N * N * b;
            else base = (size_t)a + (size_t)N * b;
            for (int k = 0; k < N; ++k) {
                double sr = 0.0, si = 0.0;
                for (int j = 0; j < N; ++j) {
                    int m = (int)(((long)k * j) % N);
                    double xr = re[base + stride * j], xi = im[base + stride * j];
                    /* (xr + i xi)(cos -+ i sin) */
                    if (sign < 0) {
                        sr += xr * cs[m] + xi * sn[m];
                        si += xi * cs[m] - xr * sn[m];
                    } else {
                        sr += xr * cs[m] - xi * sn[m];
                        si += xi * cs[m] + xr * sn[m];
                    }
                }
                tr[k] = sr;
                ti[k] = si;
            }
            for (int k = 0; k < N; ++k) {
                re[base + stride * k] = tr[k];
                im[base + stride * k] = ti[k];
            }
        }
    free(tr);
    free(ti);
}

/* Unnormalised forward DFT of a real N^3 array into (re, im), axis by axis;
 * cs, sn (N entries each) receive cos and sin of 2 pi j/N for later use. */
static void dft3_real(int N, const double *f, double *re, double *im, double *cs, double *sn)
{
    size_t V = vol(N);
    memcpy(re, f, V * sizeof(double));
    memset(im, 0, V * sizeof(double));
    for (int j = 0; j < N; ++j) {
        cs[j] = cos(2.0 * ORC_PI * j / N);
        sn[j] = sin(2.0 * ORC_PI * j / N);
    }
    for (int axis = 0; axis < 3; ++axis) dft_axis(N, re, im, axis, cs, sn, -1);
}

/* Shell of mode (x, y, z): the integer b with b <= |n~| < b + 1, where each
 * component n~ is the mode number taken in (-N/2, N/2]. */
static long shell_of(int N, int x, int y, int z)
{
    long nx = x <= N / 2 ? x : x - N, ny = y <= N / 2 ? y : y - N, nz = z <= N / 2 ? z : z - N;
    long m = nx * nx + ny * ny + nz * nz;
    long b = (long)sqrt((double)m);
    while ((b + 1) * (b + 1) <= m) ++b;
    while (b * b > m) --b;
    return b;
}

/* Weight of shell b >= 1 in eq. discretePS: Delta(b) = c_b sum_shell |f~|^2,
 * c_b = k_b^3/(2 pi^2) (dx/N)^3 / (4 pi b^2), k_b = b k_IR, k_IR = 2 pi/(N dx). */
static double shell_weight(int N, double dx, long b)
{
    double kb = b * (2.0 * ORC_PI / (N * dx)), v = dx / N;
    return kb * kb * kb / (2.0 * ORC_PI * ORC_PI) * v * v * v / (4.0 * ORC_PI * (double)b * b);
}

int orc_spectrum(int N, double dx, const double *f, int nbins, double *sum, double *delta, long *count)
{
    if (N < 1 || !f || nbins < 1) return -1;
    size_t V = vol(N);
    double *re = (double *)malloc(V * sizeof(double));
    double *im = (double *)calloc(V, sizeof(double));
    double *cs = (double *)malloc((size_t)N * sizeof(double));
    double *sn = (double *)malloc((size_t)N * sizeof(double));
    double *comp = (double *)calloc((size_t)nbins, sizeof(double));
    dft3_real(N, f, re, im, cs, sn);
    for (int b = 0; b < nbins; ++b) {
        sum[b] = 0.0;
        count[b] = 0;
    }
    int filled = 0;
    for (int z = 0; z < N; ++z)
        for (int y = 0; y < N; ++y)
            for (int x = 0; x < N; ++x) {
                long b = shell_of(N, x, y, z);
                if (b >= nbins) continue;
                size_t n = (size_t)x + (size_t)N * ((size_t)y + (size_t)N * z);
                double p = re[n] * re[n] + im[n] * im[n];
                /* Neumaier */
                double t = sum[b] + p;
                if (fabs(sum[b]) >= fabs(p)) comp[b] += (sum[b] - t) + p;
                else comp[b] += (p - t) + sum[b];
                sum[b] = t;
                count[b] += 1;
                if (b + 1 > filled) filled = (int)b + 1;
            }
    for (int b = 0; b < nbins; ++b) {
        sum[b] += comp[b];
        delta[b] = b == 0 ? 0.0 : shell_weight(N, dx, b) * sum[b];
    }
    free(re);
    free(im);
    free(cs);
    free(sn);
    free(comp);
    return filled;
}


/* Spectrum-bin observable (sec. 3.1, eq. discretePS): O = Delta(b) of field s,
 * with Delta(b) = c_b sum_{n in shell b} |f~(n)|^2, c_b = k_b^3/(2 pi^2)
 * (dx/N)^3 / (4 pi b^2).  Its derivative with respect to f(x) is
 * c_b 2 sum_{n in shell} Re[f~(n) e^{2 pi i n.x/N}], the unnormalised inverse
 * DFT of the shell-masked transform (real: each shell holds n and -n). */
static double spectrum_bin_value(int N, double dx, const double *f, int bin, double *g)
{
    size_t V = vol(N);
    double *re = (double *)malloc(V * sizeof(double));
    double *im = (double *)calloc(V, sizeof(double));
    double *cs = (double *)malloc((size_t)N * sizeof(double));
    double *sn = (double *)malloc((size_t)N * sizeof(double));
    dft3_real(N, f, re, im, cs, sn);
    double sum = 0.0, comp = 0.0;
    for (int z = 0; z < N; ++z)
        for (int y = 0; y < N; ++y)
            for (int x = 0; x < N; ++x) {
                long b = shell_of(N, x, y, z);
                size_t n = (size_t)x + (size_t)N * ((size_t)y + (size_t)N * z);
                if (b != bin) {
                    re[n] = im[n] = 0.0;
                    continue;
                }
                double p = re[n] * re[n] + im[n] * im[n];
                double t = sum + p;
                if (fabs(sum) >= fabs(p)) comp += (sum - t) + p;
                else comp += (p - t) + sum;
                sum = t;
            }
    sum += comp;
    double cb = bin == 0 ? 0.0 : shell_weight(N, dx, bin);
    if (g) {
        for (int axis = 0; axis < 3; ++axis) dft_axis(N, re, im, axis, cs, sn, +1);
        for (size_t n = 0; n < V; ++n) g[n] = 2.0 * cb * re[n];
    }
    free(re);
    free(im);
    free(cs);
    free(sn);
    return cb * sum;
}

/* Observable `kind` of the state and its gradient (seed of the adjoint):
 * ORC_OBS_ENERGY_FRACTION: energy fraction of phi_field; ORC_OBS_SPECTRUM_BIN: Delta(bin) of
 * phi_field, gradient in gphi[field] only, no explicit q dependence. */
static double observable_kind(const orc_params *p, double a, int kind, int field, int bin, double *const *phi,
                              double *const *pi, double **gphi, double **gpi, double *dq)
{
    if (kind == ORC_OBS_ENERGY_FRACTION) return observable(p, a, field, phi, pi, gphi, gpi, dq);
    size_t V = vol(p->N);
    for (int s = 0; s < 2; ++s) {
        if (gphi) memset(gphi[s], 0, V * sizeof(double));
        if (gpi) memset(gpi[s], 0, V * sizeof(double));
    }
    if (dq) *dq = 0.0;
    return spectrum_bin_value(p->N, p->dx, phi[field], bin, gphi ? gphi[field] : NULL);
}

int orc_observable_kind(const orc_params *p, double a, int kind, int field, int bin, double *const *phi,
                        double *const *pi, double *O, double *const *gphi, double *const *gpi, double *dOdq)
{
    if (p->nfields != 2 || p->potential != ORC_PHI4_CHI2) return -2;   /* any expansion: a is an argument */
    if (kind != ORC_OBS_ENERGY_FRACTION && kind != ORC_OBS_SPECTRUM_BIN) return -1;
    if (field < 0 || field > 1 || (kind == ORC_OBS_SPECTRUM_BIN && bin < 1)) return -1;
    double d = 0.0;
    if (!(a > 0.0)) return -1;
    *O = observable_kind(p, a, kind, field, bin, phi, pi, (double **)gphi, (double **)gpi, gphi ? &d : NULL);
    if (dOdq) *dOdq = d;
    return 0;
}

/* Lattice occupation number of scalar field s (eq. OccuppationNum), per radial
 * bin b >= 1 (shells as the spectrum):
 *   n_b = (a^2 L^3 / (2 N^6)) F [ omega_b <|f~|^2>_R
 *                                 + a^{2(1-alpha)}/omega_b <|f~' + (b_/a) f~|^2>_R ],
 * L = N dx, F = (f_star/omega_star)^2 (argument fstar2), <.>_R the shell sum
 * divided by 4 pi b^2 as in eq. discretePS, f' = a^{alpha-3} pi (the drift of
 * sec. 4.5.2), b_ = a', omega_b^2 = k_b^2 + a^2 <d^2V/dphi_s^2> with the volume
 * average over the lattice and k_b = b k_IR.  n_0 = 0.  Momenta must be at the
 * same time as the fields.  Returns the number of bins filled or -1. */
int orc_occupation(const orc_params *p, double a, double bdot, double *const *phi, double *const *pi, int field,
                   double fstar2, int nbins, double *n, long *count)
{
    const int N = p->N;
    if (N < 1 || nbins < 1 || field < 0 || field >= p->nfields || a <= 0.0) return -1;
    size_t V = vol(N);
    /* <d^2 V / dphi_s^2>: lambda/4 phi^4 gives 3 lambda phi^2; q/2 phi^2 chi^2
     * gives q chi^2 for phi and q phi^2 for chi */
    double vpp = 0.0;
    for (size_t i = 0; i < V; ++i) {
        double u = phi[0][i], w = p->nfields > 1 ? phi[1][i] : 0.0, d = 0.0;
        if (field == 0) {
            d = 3.0 * p->lambda * u * u;
            if (p->potential == ORC_PHI4_CHI2) d += p->q * w * w;
        } else if (p->potential == ORC_PHI4_CHI2) {
            d = p->q * u * u;
        }
        vpp += d;
    }
    vpp /= (double)V;
    double *fr = (double *)malloc(V * sizeof(double)), *fi = (double *)malloc(V * sizeof(double));
    double *pr = (double *)malloc(V * sizeof(double)), *pim = (double *)malloc(V * sizeof(double));
    double *cs = (double *)malloc((size_t)N * sizeof(double)), *sn = (double *)malloc((size_t)N * sizeof(double));
    double *sf = (double *)calloc((size_t)nbins, sizeof(double)), *sx = (double *)calloc((size_t)nbins, sizeof(double));
    dft3_real(N, phi[field], fr, fi, cs, sn);
    dft3_real(N, pi[field], pr, pim, cs, sn);
    const double cp = pow(a, p->alpha - 3.0), hub = bdot / a;
    for (int b = 0; b < nbins; ++b) count[b] = 0;
    int filled = 0;
    for (int z = 0; z < N; ++z)
        for (int y = 0; y < N; ++y)
            for (int x = 0; x < N; ++x) {
                long b = shell_of(N, x, y, z);
                if (b >= nbins) continue;
                size_t i = (size_t)x + (size_t)N * ((size_t)y + (size_t)N * z);
                double xr = cp * pr[i] + hub * fr[i], xi = cp * pim[i] + hub * fi[i];
                sf[b] += fr[i] * fr[i] + fi[i] * fi[i];
                sx[b] += xr * xr + xi * xi;
                count[b] += 1;
                if (b + 1 > filled) filled = (int)b + 1;
            }
    const double L = N * p->dx, N6 = (double)V * (double)V;
    const double pref = a * a * L * L * L / (2.0 * N6) * fstar2;
    const double kir = 2.0 * ORC_PI / L;
    for (int b = 0; b < nbins; ++b) {
        if (b == 0) {
            n[b] = 0.0;
            continue;
        }
        double kb = b * kir;
        double om = sqrt(kb * kb + a * a * vpp);
        n[b] = pref * (om * sf[b] + pow(a, 2.0 * (1.0 - p->alpha)) * sx[b] / om) / (4.0 * ORC_PI * (double)b * b);
    }
    free(fr);
    free(fi);
    free(pr);
    free(pim);
    free(cs);
    free(sn);
    free(sf);
    free(sx);
    return filled;
}

/* ------------------------------------------------------------------ */
/* SU(2) sector: doublet + SU(2) links, a = 1 (sec. 3.2 SU(N) toolkit, */
/* sec. 5 eqs. higgsSU2-eom, SU2eom, GaussSU2-eom, energy-contrib;     */
/* reading R6)                                                         */
/*                                                                     */
/* Doublet Phi = (psi0, psi1)/sqrt(2), psi0 = phi0 + i phi1,             */
/*   psi1 = phi2 + i phi3 (eq. ChargedScalars); momenta pi_c = phi_c'.   */
/* Links U_i(n) = exp(-i g dx B_i^a T_a), T_a = sigma_a/2, stored as four */
/*   reals (u0, u1, u2, u3) with U = u0 I - i sum_a u_a sigma_a.         */
/* Electric fields E_i^a(n), conjugate to U_i(n) under the left          */
/*   variation U -> exp(-i eps g dx T_a) U.                              */
/* Lattice Hamiltonian (sum over sites n):                              */
/*   H = sum_c pi_c^2/2 + sum_i |U_i psi(n+i) - psi(n)|^2 / (2 dx^2)      */
/*     + lambda/4 (|Phi|^2 - v^2)^2 + sum_{i,a} (E_i^a)^2 / 2              */
/*     + 2/(g^2 dx^4) sum_{i<j} (2 - Tr P_ij(n)),                        */
/*   P_ij(n) = U_i(n) U_j(n+i) U_i(n+j)^dag U_j(n)^dag (toolkit plaquette), */
/*   |Phi|^2 = sum_c phi_c^2 / 2.                                        */
/* Leapfrog: kick pi and E by h (-dH), drift phi += h pi,                */
/*   U <- exp(-i h g dx E^a T_a) U.                                      */
/* All products here are plain 2x2 complex matrices with the Pauli       */
/* matrices written out.                                                */
/* ------------------------------------------------------------------ */
#include <complex.h>

typedef struct orc_su2_params {
    int32_t N;
    int32_t expansion;                      /* ORC_NONE, ORC_FIXED, ORC_SELF (as for the scalars) */
    double dx, dt, lambda, v, g;
    double alpha, kappa2;                   /* alpha-time exponent; (f_star/m_p)^2 */
    double w_eos, H0, t0, a0;               /* fixed background (eq. ScaleFactorPowerLaw); SELF: a0 */
} orc_su2_params;

/* SU(2) sector in an expanding background (sec. 5.5.2, reading U1 applied to
 * the doublet and its links).  With pi_Phi = a^{3-alpha} Phi' and
 * pi_B = a^{1-alpha} G_0i (eqs. momSU2doublet, momSU2vec) the kernels of eq.
 * kernelsSU21 and the one after it are the a = 1 forces with each term scaled:
 *   K_Phi = a^{1+alpha} (covariant Laplacian) - a^{3+alpha} (potential force),
 *   K_B   = a^{1+alpha} J - a^{alpha-1} (staple force),
 * the drifts are Phi' = a^{alpha-3} pi_Phi and U <- exp(-i h a^{alpha-1} g dx
 * E^a T_a) U, the energies are the a = 1 ones over a^6 (doublet kinetic), a^2
 * (doublet gradient) and a^4 (electric, magnetic), and the scale-factor
 * kernel adds (alpha - 1)(E_K^B + E_G^B).  The Gauss law (eq. GaussSU2-eom)
 * in these variables carries no power of a.  Kicks and drifts take a as the
 * U(1) model does (readings R3, R1, A3). */

typedef struct { double complex m[2][2]; } mat2;

static const double complex PAULI[3][2][2] = {
    {{0.0, 1.0}, {1.0, 0.0}},
    {{0.0, -I}, {I, 0.0}},
    {{1.0, 0.0}, {0.0, -1.0}},
};

static mat2 m2_mul(mat2 a, mat2 b)
{
    mat2 c;
    for (int r = 0; r < 2; ++r)
        for (int s = 0; s < 2; ++s) c.m[r][s] = a.m[r][0] * b.m[0][s] + a.m[r][1] * b.m[1][s];
    return c;
}

static mat2 m2_dag(mat2 a)
{
    mat2 c;
    for (int r = 0; r < 2; ++r)
        for (int s = 0; s < 2; ++s) c.m[r][s] = conj(a.m[s][r]);
    return c;
}

/* u0 I - i sum_a u_a sigma_a */
static mat2 m2_from_quat(double u0, const double *u)
{
    mat2 c;
    for (int r = 0; r < 2; ++r)
        for (int s = 0; s < 2; ++s) {
            double complex v = (r == s) ? u0 : 0.0;
            for (int a = 0; a < 3; ++a) v += -I * u[a] * PAULI[a][r][s];
            c.m[r][s] = v;
        }
    return c;
}

/* inverse of m2_from_quat: u0 = Re Tr(M)/2, u_a = Re Tr(i sigma_a M)/2 */
static void m2_to_quat(mat2 M, double *q)
{
    q[0] = creal(M.m[0][0] + M.m[1][1]) / 2.0;
    for (int a = 0; a < 3; ++a) {
        double complex t = 0.0;
        for (int r = 0; r < 2; ++r)
            for (int s = 0; s < 2; ++s) t += I * PAULI[a][r][s] * M.m[s][r];
        q[1 + a] = creal(t) / 2.0;
    }
}

static mat2 su2_link(double *const *U, int i, size_t n)
{
    double u[3] = {U[4 * i + 1][n], U[4 * i + 2][n], U[4 * i + 3][n]};
    return m2_from_quat(U[4 * i][n], u);
}

static void su2_psi(double *const *phi, size_t n, double complex *psi)
{
    psi[0] = phi[0][n] + I * phi[1][n];
    psi[1] = phi[2][n] + I * phi[3][n];
}

static void m2_apply(mat2 M, const double complex *x, double complex *y)
{
    y[0] = M.m[0][0] * x[0] + M.m[0][1] * x[1];
    y[1] = M.m[1][0] * x[0] + M.m[1][1] * x[1];
}

/* the coordinates of site n shifted by s (+1/-1) along d */
static void shift(int N, const int *c, int d, int s, int *o)
{
    o[0] = c[0]; o[1] = c[1]; o[2] = c[2];
    o[d] = s > 0 ? up(o[d], N) : dn(o[d], N);
}

/* forces = minus the derivative of the lattice Hamiltonian:
 *   Fphi = {Re, Im} of D^2 psi - lambda/2 (|Phi|^2 - v^2) phi_c, with
 *     D^2 psi = dx^-2 sum_i [U_i(n) psi(n+i) - 2 psi(n) + U_i(n-i)^dag psi(n-i)]
 *   FE_i^a = (g/dx) Im[psi^dag T_a U_i psi(n+i)]
 *          - 2/(g dx^3) sum_{j != i} vec_a[U_i S+_ij] + vec_a[U_i S-_ij]
 *   with the staples S+_ij = U_j(n+i) U_i(n+j)^dag U_j(n)^dag and
 *   S-_ij = U_j(n+i-j)^dag U_i(n-j)^dag U_j(n-j), and vec_a[M] = u_a of
 *   M = u0 I - i u.sigma, i.e. -d Tr(exp(-i eps g dx T_a) U S)/d eps = g dx vec_a.  */
static int su2_forces_a(const orc_su2_params *p, double a, double *const *phi, double *const *U,
                        double *const *Fphi, double *const *FE)
{
    int N = p->N;
    double dx = p->dx, g = p->g;
    double cl = pow(a, 1.0 + p->alpha), cv = pow(a, 3.0 + p->alpha), cm_ = pow(a, p->alpha - 1.0);
    #pragma omp parallel for schedule(static)
    for (int z = 0; z < N; ++z)
        for (int y = 0; y < N; ++y)
            for (int x = 0; x < N; ++x) {
                int c[3] = {x, y, z};
                size_t n = at(N, x, y, z);
                double complex psi[2], d2[2] = {0.0, 0.0};
                su2_psi(phi, n, psi);
                for (int i = 0; i < 3; ++i) {
                    int cp[3], cm[3];
                    shift(N, c, i, +1, cp);
                    shift(N, c, i, -1, cm);
                    size_t np = at(N, cp[0], cp[1], cp[2]), nm = at(N, cm[0], cm[1], cm[2]);
                    double complex qp[2], qm[2], a[2], b[2];
                    su2_psi(phi, np, qp);
                    su2_psi(phi, nm, qm);
                    mat2 Ui = su2_link(U, i, n);
                    m2_apply(Ui, qp, a);                       /* U_i(n) psi(n+i)      */
                    m2_apply(m2_dag(su2_link(U, i, nm)), qm, b); /* U_i(n-i)^dag psi(n-i) */
                    for (int r = 0; r < 2; ++r) d2[r] += a[r] - 2.0 * psi[r] + b[r];
                    double vs[3] = {0.0, 0.0, 0.0};
                    for (int j = 0; j < 3; ++j) {
                        if (j == i) continue;
                        int cj[3], cmj[3], cimj[3];
                        shift(N, c, j, +1, cj);
                        shift(N, c, j, -1, cmj);
                        shift(N, cp, j, -1, cimj);
                        size_t nj = at(N, cj[0], cj[1], cj[2]), nmj = at(N, cmj[0], cmj[1], cmj[2]);
                        size_t nimj = at(N, cimj[0], cimj[1], cimj[2]);
                        mat2 Sp = m2_mul(m2_mul(su2_link(U, j, np), m2_dag(su2_link(U, i, nj))),
                                         m2_dag(su2_link(U, j, n)));
                        mat2 Sm = m2_mul(m2_mul(m2_dag(su2_link(U, j, nimj)), m2_dag(su2_link(U, i, nmj))),
                                         su2_link(U, j, nmj));
                        double qa[4], qb[4];
                        m2_to_quat(m2_mul(Ui, Sp), qa);
                        m2_to_quat(m2_mul(Ui, Sm), qb);
                        for (int k = 0; k < 3; ++k) vs[k] += qa[1 + k] + qb[1 + k];
                    }
                    for (int k = 0; k < 3; ++k) {
                        /* psi^dag T_k a, T_k = sigma_k / 2 */
                        double complex t = 0.0;
                        for (int r = 0; r < 2; ++r)
                            for (int s = 0; s < 2; ++s) t += conj(psi[r]) * 0.5 * PAULI[k][r][s] * a[s];
                        FE[3 * i + k][n] = cl * (g / dx * cimag(t)) - cm_ * (2.0 / (g * dx * dx * dx) * vs[k]);
                    }
                }
                double m2 = 0.0;
                for (int k = 0; k < 4; ++k) m2 += 0.5 * phi[k][n] * phi[k][n];
                double vp = 0.5 * p->lambda * (m2 - p->v * p->v);
                Fphi[0][n] = cl * (creal(d2[0]) / (dx * dx)) - cv * (vp * phi[0][n]);
                Fphi[1][n] = cl * (cimag(d2[0]) / (dx * dx)) - cv * (vp * phi[1][n]);
                Fphi[2][n] = cl * (creal(d2[1]) / (dx * dx)) - cv * (vp * phi[2][n]);
                Fphi[3][n] = cl * (cimag(d2[1]) / (dx * dx)) - cv * (vp * phi[3][n]);
            }
    return 0;
}

int orc_su2_forces(const orc_su2_params *p, double *const *phi, double *const *U,
                   double *const *Fphi, double *const *FE)
{
    return su2_forces_a(p, 1.0, phi, U, Fphi, FE);
}

int orc_su2_forces_at(const orc_su2_params *p, double a, double *const *phi, double *const *U,
                      double *const *Fphi, double *const *FE)
{
    return su2_forces_a(p, a, phi, U, Fphi, FE);
}

/* SU(2) energies and Gauss constraint.  Output layout (12 doubles):
 *  [0] E_K^Phi = <sum_c pi_c^2 / 2>, [1] E_G^Phi = <sum_i |U_i psi(n+i) - psi(n)|^2>/(2 dx^2),
 *  [2] E_V = <lambda/4 (|Phi|^2 - v^2)^2>, [3] E_K^B = <sum_{i,a} (E_i^a)^2>/2,
 *  [4] E_G^B = <2/(g^2 dx^4) sum_{i<j} (2 - Tr P_ij)>, [5] rho
 *  (at scale factor a: [0] over a^6, [1] over a^2, [3] and [4] over a^4),
 *  [6] max|G|, [7] max|div E|, [8] max|charge|, [9] <|G|>, [10] <|div E + charge|>,
 *  [11] <|div E| + |charge|>, with |.| the Euclidean norm over a and
 *  (eq. GaussSU2-eom at a = 1, the covariant backward divergence)
 *    div E^a = dx^-1 sum_i [E_i^a(n) - vec_a(U_i(n-i)^dag (E_i(n-i).sigma) U_i(n-i))],
 *    charge^a = g Im[psi^dag T_a pi_psi],  G = div E - charge.
 *  2 - Tr P = 2 (1 - p0) is evaluated as 2 |p|^2 / (1 + p0) for P = p0 - i p.sigma
 *  (the same number for a unitary P, det P = p0^2 + |p|^2 = 1, without the
 *  cancellation of 1 - p0 at small plaquette angles).                    */
static void su2_energy_plain(const orc_su2_params *p, double a, double *const *phi, double *const *pi,
                             double *const *U, double *const *E, double *out)
{
    int N = p->N;
    size_t V = vol(N);
    double dx = p->dx, g = p->g;
    nsum sk = {0, 0}, sg = {0, 0}, sv = {0, 0}, ske = {0, 0}, sgb = {0, 0};
    nsum sG = {0, 0}, sLR = {0, 0}, sLRabs = {0, 0};
    double gmax = 0, dmax = 0, cmax = 0;
    for (int z = 0; z < N; ++z)
        for (int y = 0; y < N; ++y)
            for (int x = 0; x < N; ++x) {
                int c[3] = {x, y, z};
                size_t n = at(N, x, y, z);
                double kin = 0.0, m2 = 0.0;
                for (int k = 0; k < 4; ++k) {
                    kin += 0.5 * pi[k][n] * pi[k][n];
                    m2 += 0.5 * phi[k][n] * phi[k][n];
                }
                nadd(&sk, kin);
                double complex psi[2], ppsi[2];
                su2_psi(phi, n, psi);
                su2_psi(pi, n, ppsi);
                double grad = 0.0, ke = 0.0, div[3] = {0.0, 0.0, 0.0};
                for (int i = 0; i < 3; ++i) {
                    int cp[3], cm[3];
                    shift(N, c, i, +1, cp);
                    shift(N, c, i, -1, cm);
                    size_t np = at(N, cp[0], cp[1], cp[2]), nm = at(N, cm[0], cm[1], cm[2]);
                    double complex qp[2], a[2];
                    su2_psi(phi, np, qp);
                    m2_apply(su2_link(U, i, n), qp, a);
                    for (int r = 0; r < 2; ++r) {
                        double complex d = a[r] - psi[r];
                        grad += creal(d) * creal(d) + cimag(d) * cimag(d);
                    }
                    /* E_i(n-i) transported to n */
                    mat2 X;
                    for (int r = 0; r < 2; ++r)
                        for (int s = 0; s < 2; ++s) {
                            X.m[r][s] = 0.0;
                            for (int k = 0; k < 3; ++k) X.m[r][s] += E[3 * i + k][nm] * PAULI[k][r][s];
                        }
                    mat2 Um = su2_link(U, i, nm);
                    mat2 Y = m2_mul(m2_mul(m2_dag(Um), X), Um);
                    for (int k = 0; k < 3; ++k) {
                        double complex t = 0.0;   /* vec_k of Y = sum y_k sigma_k: Tr(sigma_k Y)/2 */
                        for (int r = 0; r < 2; ++r)
                            for (int s = 0; s < 2; ++s) t += PAULI[k][r][s] * Y.m[s][r];
                        div[k] += (E[3 * i + k][n] - creal(t) / 2.0) / dx;
                        ke += E[3 * i + k][n] * E[3 * i + k][n];
                    }
                }
                nadd(&sg, grad / (2.0 * dx * dx));
                double u = m2 - p->v * p->v;
                nadd(&sv, 0.25 * p->lambda * u * u);
                nadd(&ske, 0.5 * ke);
                double mag = 0.0;
                for (int i = 0; i < 3; ++i)
                    for (int j = i + 1; j < 3; ++j) {
                        int ci[3], cj[3];
                        shift(N, c, i, +1, ci);
                        shift(N, c, j, +1, cj);
                        mat2 P = m2_mul(m2_mul(su2_link(U, i, n), su2_link(U, j, at(N, ci[0], ci[1], ci[2]))),
                                        m2_mul(m2_dag(su2_link(U, i, at(N, cj[0], cj[1], cj[2]))),
                                               m2_dag(su2_link(U, j, n))));
                        double q[4];
                        m2_to_quat(P, q);
                        mag += 2.0 * (q[1] * q[1] + q[2] * q[2] + q[3] * q[3]) / (1.0 + q[0]);
                    }
                nadd(&sgb, 2.0 * mag / (g * g * dx * dx * dx * dx));
                double Gn = 0.0, dn2 = 0.0, cn = 0.0, lr = 0.0;
                for (int k = 0; k < 3; ++k) {
                    double complex t = 0.0;
                    for (int r = 0; r < 2; ++r)
                        for (int s = 0; s < 2; ++s) t += conj(psi[r]) * 0.5 * PAULI[k][r][s] * ppsi[s];
                    double ch = g * cimag(t);
                    Gn += (div[k] - ch) * (div[k] - ch);
                    dn2 += div[k] * div[k];
                    cn += ch * ch;
                    lr += (div[k] + ch) * (div[k] + ch);
                }
                Gn = sqrt(Gn);
                dn2 = sqrt(dn2);
                cn = sqrt(cn);
                if (Gn > gmax) gmax = Gn;
                if (dn2 > dmax) dmax = dn2;
                if (cn > cmax) cmax = cn;
                nadd(&sG, Gn);
                nadd(&sLR, sqrt(lr));
                nadd(&sLRabs, dn2 + cn);
            }
    const double a2 = a * a, a4 = a2 * a2, a6 = a4 * a2;
    out[0] = nval(&sk) / (double)V / a6;
    out[1] = nval(&sg) / (double)V / a2;
    out[2] = nval(&sv) / (double)V;
    out[3] = nval(&ske) / (double)V / a4;
    out[4] = nval(&sgb) / (double)V / a4;
    out[5] = out[0] + out[1] + out[2] + out[3] + out[4];
    out[6] = gmax;
    out[7] = dmax;
    out[8] = cmax;
    out[9] = nval(&sG) / (double)V;
    out[10] = nval(&sLR) / (double)V;
    out[11] = nval(&sLRabs) / (double)V;
}

/* kernel of b with the gauge energies (sec. 5.5.2):
 *   K_a = a^{2 alpha + 1}/3 kappa^2 [(alpha-2) E_K^Phi + alpha E_G^Phi
 *         + (alpha-1)(E_K^B + E_G^B) + (alpha+1) E_V]   (energies as su2_energy_plain) */
static double su2_kernel_a(const orc_su2_params *p, double a, const double *E)
{
    double al = p->alpha;
    return pow(a, 2.0 * al + 1.0) / 3.0 * p->kappa2 *
           ((al - 2.0) * E[0] + al * E[1] + (al - 1.0) * (E[3] + E[4]) + (al + 1.0) * E[2]);
}

static void su2_fixed_ab(const orc_su2_params *p, double t, double *a, double *b)
{
    double pw = 2.0 / (3.0 * (1.0 + p->w_eos) - 2.0 * p->alpha);
    double u = 1.0 + p->H0 * (t - p->t0) / pw;
    *a = p->a0 * pow(u, pw);
    *b = p->a0 * p->H0 * pow(u, pw - 1.0);
}

int orc_su2_fixed_background(const orc_su2_params *p, double t, double *a, double *b)
{
    su2_fixed_ab(p, t, a, b);
    return 0;
}

static void su2_kick(const orc_su2_params *p, double a, double *const *phi, double *const *pi,
                     double *const *U, double *const *E, double w)
{
    size_t V = vol(p->N);
    double *F[13];
    for (int i = 0; i < 13; ++i) F[i] = (double *)malloc(V * sizeof(double));
    su2_forces_a(p, a, phi, U, F, F + 4);
    #pragma omp parallel for schedule(static)
    for (size_t n = 0; n < V; ++n) {
        for (int k = 0; k < 4; ++k) pi[k][n] += w * F[k][n];
        for (int k = 0; k < 9; ++k) E[k][n] += w * F[4 + k][n];
    }
    for (int i = 0; i < 13; ++i) free(F[i]);
}

/* exp(-i w g dx E^a T_a) = cos(th/2) I - i sin(th/2) (e.sigma), th = w g dx |E|, e = E/|E| */
static mat2 su2_exp(double wgdx, const double *Ev)
{
    double len = sqrt(Ev[0] * Ev[0] + Ev[1] * Ev[1] + Ev[2] * Ev[2]);
    double th = wgdx * len;
    double u[3] = {0.0, 0.0, 0.0};
    if (len > 0.0)
        for (int a = 0; a < 3; ++a) u[a] = sin(0.5 * th) * Ev[a] / len;
    return m2_from_quat(cos(0.5 * th), u);
}

/* drift by h with the scale factor a_mid of its midpoint: Phi += h a^{alpha-3} pi,
 * U <- exp(-i h a^{alpha-1} g dx E^a T_a) U */
static void su2_drift(const orc_su2_params *p, double a_mid, double *const *phi, double *const *pi,
                      double *const *U, double *const *E, double h)
{
    size_t V = vol(p->N);
    double cp = h * pow(a_mid, p->alpha - 3.0), cu = h * pow(a_mid, p->alpha - 1.0);
    #pragma omp parallel for schedule(static)
    for (size_t n = 0; n < V; ++n) {
        for (int k = 0; k < 4; ++k) phi[k][n] += cp * pi[k][n];
        for (int i = 0; i < 3; ++i) {
            double Ev[3] = {E[3 * i][n], E[3 * i + 1][n], E[3 * i + 2][n]};
            mat2 R = m2_mul(su2_exp(cu * p->g * p->dx, Ev), su2_link(U, i, n));
            double q[4];
            m2_to_quat(R, q);
            for (int k = 0; k < 4; ++k) U[4 * i + k][n] = q[k];
        }
    }
}

/* Energies at integer time, output layout (17 doubles): [0 .. 11] as
 * su2_energy_plain at the clock's a; [12] a, [13] b at integer time,
 * [14] Hubble LHS b^2, [15] RHS a^{2 alpha + 2} kappa^2 rho / 3, [16] (LHS - RHS)/(LHS + RHS).
 * Leapfrog momenta (and b with self-consistent expansion) are synchronised on
 * copies (readings R4, A3). */
int orc_su2_energy(const orc_su2_params *p, double *const *phi, double *const *pi,
                   double *const *U, double *const *E, const orc_clock *c, double *out)
{
    size_t V = vol(p->N), B = V * sizeof(double);
    double *ps[4], *pe[9];
    for (int i = 0; i < 4; ++i) { ps[i] = (double *)malloc(B); memcpy(ps[i], pi[i], B); }
    for (int i = 0; i < 9; ++i) { pe[i] = (double *)malloc(B); memcpy(pe[i], E[i], B); }
    double b = c->b;
    if (c->lf_stag != 0) {
        double w = 0.5 * c->lf_stag * p->dt;
        if (p->expansion == ORC_SELF) {
            double Eb[12];
            su2_energy_plain(p, c->a, phi, ps, U, pe, Eb);
            b += w * su2_kernel_a(p, c->a, Eb);
        }
        su2_kick(p, c->a, phi, ps, U, pe, w);
    }
    su2_energy_plain(p, c->a, phi, ps, U, pe, out);
    for (int i = 0; i < 4; ++i) free(ps[i]);
    for (int i = 0; i < 9; ++i) free(pe[i]);
    double lhs = b * b, rhs = pow(c->a, 2.0 * p->alpha + 2.0) * p->kappa2 * out[5] / 3.0;
    out[12] = c->a;
    out[13] = b;
    out[14] = lhs;
    out[15] = rhs;
    out[16] = (lhs + rhs) != 0.0 ? (lhs - rhs) / (lhs + rhs) : 0.0;
    return 0;
}

/* Hubble constraint (eq. FriedmannHubble) for b at the start: b0^2 = a^{2 alpha + 2} kappa^2 rho / 3 */
int orc_su2_hubble_b0(const orc_su2_params *p, double *const *phi, double *const *pi, double *const *U,
                      double *const *E, double a, double *b0)
{
    double En[12];
    su2_energy_plain(p, a, phi, pi, U, E, En);
    double rhs = pow(a, 2.0 * p->alpha + 2.0) * p->kappa2 * En[5] / 3.0;
    if (rhs < 0.0) return -1;
    *b0 = sqrt(rhs);
    return 0;
}

/* Gauss residual of the stored (un-synchronised) pairing, same layout [6..11]. */
int orc_su2_gauss(const orc_su2_params *p, double *const *phi, double *const *pi,
                  double *const *U, double *const *E, double *out)
{
    su2_energy_plain(p, 1.0, phi, pi, U, E, out);
    return 0;
}

/* Staggered leapfrog for the SU(2) system: kick all momenta, then drift the
 * doublet and the links.  Same staggering convention as orc_run; with
 * expansion as orc_u1_run_lf (reading A3 for the self-consistent case). */
int orc_su2_run_lf(const orc_su2_params *p, double *const *phi, double *const *pi,
                   double *const *U, double *const *E, orc_clock *c, long nsteps)
{
    if (nsteps == 0) return 0;
    int dir = nsteps > 0 ? 1 : -1;
    long ns = nsteps > 0 ? nsteps : -nsteps;
    double h = dir * p->dt;
    if (c->lf_stag != 0 && c->lf_stag != dir) return -3;
    double t_start = c->t;
    for (long k = 0; k < ns; ++k) {
        double t = t_start + (double)k * h;
        double w = c->lf_stag == 0 ? 0.5 * h : h;
        if (p->expansion == ORC_SELF) {
            double Eb[12], Ea[12];
            su2_energy_plain(p, c->a, phi, pi, U, E, Eb);
            su2_kick(p, c->a, phi, pi, U, E, w);
            su2_energy_plain(p, c->a, phi, pi, U, E, Ea);
            if (c->lf_stag == 0)
                c->b += w * su2_kernel_a(p, c->a, Ea);
            else
                c->b += 0.5 * h * su2_kernel_a(p, c->a, Eb) + 0.5 * h * su2_kernel_a(p, c->a, Ea);
            double a1 = c->a + h * c->b;
            su2_drift(p, 0.5 * (c->a + a1), phi, pi, U, E, h);
            c->a = a1;
        } else if (p->expansion == ORC_FIXED) {
            double a, b, am;
            su2_fixed_ab(p, t, &a, &b);
            su2_kick(p, a, phi, pi, U, E, w);
            su2_fixed_ab(p, t + 0.5 * h, &am, &b);
            su2_drift(p, am, phi, pi, U, E, h);
        } else {
            su2_kick(p, 1.0, phi, pi, U, E, w);
            su2_drift(p, 1.0, phi, pi, U, E, h);
        }
        c->lf_stag = dir;
    }
    c->t = t_start + (double)ns * h;
    if (p->expansion == ORC_FIXED) {
        su2_fixed_ab(p, c->t, &c->a, &c->b);
    } else if (p->expansion == ORC_NONE) {
        c->a = 1.0;
        c->b = 0.0;
    }
    return 0;
}

int orc_su2_lf_sync(const orc_su2_params *p, double *const *phi, double *const *pi,
                    double *const *U, double *const *E, orc_clock *c)
{
    if (c->lf_stag == 0) return 0;
    double w = 0.5 * c->lf_stag * p->dt;
    if (p->expansion == ORC_SELF) {
        double En[12];
        su2_energy_plain(p, c->a, phi, pi, U, E, En);
        c->b += w * su2_kernel_a(p, c->a, En);
    }
    su2_kick(p, c->a, phi, pi, U, E, w);
    c->lf_stag = 0;
    return 0;
}

/* ------------------------------------------------------------------ */
/* Gauss-consistent initial gauge momenta (sec. 5.5.1, eqs. kAi1 and      */
/* GaugeCurrentFluc; reading R14): with the links at the identity the   */
/* Gauss law reads div- E = rho, and its longitudinal solution on the   */
/* lattice is E_i = grad+_i chi with Lap chi = rho - <rho> (the lattice  */
/* Laplacian sum_i grad-_i grad+_i, so div- E = rho - <rho> exactly).    */
/* chi comes from the own DFT: chi~(k) = -rho~(k) / L(k),                */
/* L(k) = (4/dx^2) sum_i sin^2(pi k_i / N), chi~(0) = 0.                  */
/* ------------------------------------------------------------------ */

int orc_gauss_solve(int N, double dx, const double *rho, double *const *E)
{
    size_t V = vol(N);
    double *re = (double *)malloc(V * sizeof(double)), *im = (double *)malloc(V * sizeof(double));
    double *cs = (double *)malloc((size_t)N * sizeof(double)), *sn = (double *)malloc((size_t)N * sizeof(double));
    dft3_real(N, rho, re, im, cs, sn);
    for (int z = 0; z < N; ++z)
        for (int y = 0; y < N; ++y)
            for (int x = 0; x < N; ++x) {
                size_t n = at(N, x, y, z);
                double sx = sin(ORC_PI * x / N), sy = sin(ORC_PI * y / N), sz = sin(ORC_PI * z / N);
                double L = 4.0 / (dx * dx) * (sx * sx + sy * sy + sz * sz);
                if (n == 0) {
                    re[n] = 0.0;
                    im[n] = 0.0;
                } else {
                    re[n] = -re[n] / L;
                    im[n] = -im[n] / L;
                }
            }
    for (int axis = 0; axis < 3; ++axis) dft_axis(N, re, im, axis, cs, sn, +1);
    for (size_t n = 0; n < V; ++n) re[n] /= (double)V;   /* chi, real up to rounding */
    for (int z = 0; z < N; ++z)
        for (int y = 0; y < N; ++y)
            for (int x = 0; x < N; ++x) {
                size_t n = at(N, x, y, z);
                for (int i = 0; i < 3; ++i) E[i][n] = (re[nbr(N, x, y, z, i, +1)] - re[n]) / dx;
            }
    free(re);
    free(im);
    free(cs);
    free(sn);
    return 0;
}

/* SU(2): rho^a = g Im(psi^dag T_a pi_psi) of the stored doublet and momenta;
 * E_i^a from orc_gauss_solve for each a; mean[a] = <rho^a> (what no periodic
 * field can absorb).  Needs the links at the identity (returns -4 otherwise). */
int orc_su2_gauss_init(const orc_su2_params *p, double *const *phi, double *const *pi,
                       double *const *U, double *const *E, double *mean)
{
    int N = p->N;
    size_t V = vol(N);
    for (int i = 0; i < 3; ++i)
        for (size_t n = 0; n < V; ++n)
            if (U[4 * i][n] != 1.0 || U[4 * i + 1][n] != 0.0 || U[4 * i + 2][n] != 0.0 || U[4 * i + 3][n] != 0.0)
                return -4;
    double *rho = (double *)malloc(V * sizeof(double));
    for (int a = 0; a < 3; ++a) {
        nsum s = {0, 0};
        for (size_t n = 0; n < V; ++n) {
            double complex psi[2], pp[2], t = 0.0;
            su2_psi(phi, n, psi);
            su2_psi(pi, n, pp);
            for (int r = 0; r < 2; ++r)
                for (int q = 0; q < 2; ++q) t += conj(psi[r]) * 0.5 * PAULI[a][r][q] * pp[q];
            rho[n] = p->g * cimag(t);
            nadd(&s, rho[n]);
        }
        mean[a] = nval(&s) / (double)V;
        double *Ea[3] = {E[a], E[3 + a], E[6 + a]};
        orc_gauss_solve(N, p->dx, rho, Ea);
    }
    free(rho);
    return 0;
}

/* U(1): rho = e kappa_g (phi0 pi1 - phi1 pi0); pi_A from orc_gauss_solve
 * (the Abelian Gauss law does not involve the links). */
int orc_u1_gauss_init(const orc_u1_params *p, double *const *phi, double *const *pi, double *const *piA,
                      double *mean)
{
    int N = p->N;
    size_t V = vol(N);
    double *rho = (double *)malloc(V * sizeof(double));
    nsum s = {0, 0};
    for (size_t n = 0; n < V; ++n) {
        rho[n] = p->e * p->kappa_g * (phi[0][n] * pi[1][n] - phi[1][n] * pi[0][n]);
        nadd(&s, rho[n]);
    }
    mean[0] = nval(&s) / (double)V;
    orc_gauss_solve(N, p->dx, rho, piA);
    free(rho);
    return 0;
}

/* ------------------------------------------------------------------ */
/* Velocity-Verlet family for the gauge models (sec. 4.3 evolvers VV2..VV10 */
/* applied to the U(1) and SU(2) systems at a = 1; readings R2, R15): the   */
/* second-order map kick(h/2) drift(h) kick(h/2), composed with the       */
/* weights of orc_vv_stages (reading R2).                                   */
/* Plain composition: every half kick is applied on its own.               */
/* ------------------------------------------------------------------ */

/* One second-order map of size h from time t (reading R15; with expansion
 * readings R1 and R3), as u1_vv2. */
static void su2_vv2(const orc_su2_params *p, double *const *phi, double *const *pi, double *const *U,
                    double *const *E, orc_clock *c, double t, double h)
{
    if (p->expansion == ORC_SELF) {
        double En[12];
        su2_energy_plain(p, c->a, phi, pi, U, E, En);
        su2_kick(p, c->a, phi, pi, U, E, 0.5 * h);
        c->b += 0.5 * h * su2_kernel_a(p, c->a, En);
        double a1 = c->a + h * c->b;
        su2_drift(p, 0.5 * (c->a + a1), phi, pi, U, E, h);
        c->a = a1;
        su2_kick(p, c->a, phi, pi, U, E, 0.5 * h);
        su2_energy_plain(p, c->a, phi, pi, U, E, En);
        c->b += 0.5 * h * su2_kernel_a(p, c->a, En);
        return;
    }
    double a0 = 1.0, am = 1.0, a1 = 1.0, b;
    if (p->expansion == ORC_FIXED) {
        su2_fixed_ab(p, t, &a0, &b);
        su2_fixed_ab(p, t + 0.5 * h, &am, &b);
        su2_fixed_ab(p, t + h, &a1, &b);
    }
    su2_kick(p, a0, phi, pi, U, E, 0.5 * h);
    su2_drift(p, am, phi, pi, U, E, h);
    su2_kick(p, a1, phi, pi, U, E, 0.5 * h);
}

static void su2_vv(const orc_su2_params *p, double *const *phi, double *const *pi, double *const *U,
                   double *const *E, orc_clock *c, int order, double t, double h)
{
    double w[45];
    const int n = orc_vv_stages(order, w);
    for (int i = 0; i < n; ++i) {
        su2_vv2(p, phi, pi, U, E, c, t, w[i] * h);
        t += w[i] * h;
    }
}

/* order in {2, 4, 6, 8, 10}; momenta at integer time (lf_stag = 0) */
int orc_su2_run_vv(const orc_su2_params *p, double *const *phi, double *const *pi, double *const *U,
                   double *const *E, orc_clock *c, long nsteps, int order)
{
    if (c->lf_stag != 0) return -3;
    double h = nsteps >= 0 ? p->dt : -p->dt;
    long ns = nsteps >= 0 ? nsteps : -nsteps;
    double t_start = c->t;
    for (long k = 0; k < ns; ++k) su2_vv(p, phi, pi, U, E, c, order, t_start + (double)k * h, h);
    c->t = t_start + (double)ns * h;
    if (p->expansion == ORC_FIXED) su2_fixed_ab(p, c->t, &c->a, &c->b);
    return 0;
}

/* One second-order map of size h from time t (reading R15; with expansion
 * readings R1 and R3): kick(h/2) at a_n, [b kick with E_n, a drift], drift with
 * the midpoint a, kick(h/2) at a_{n+1}, [energies, b kick]. */
static void u1_vv2(const orc_u1_params *p, double *const *phi, double *const *pi, double *const *A,
                   double *const *piA, orc_clock *c, double t, double h)
{
    if (p->expansion == ORC_SELF) {
        double E[12];
        u1_energy_plain(p, c->a, phi, pi, A, piA, E);
        u1_kick(p, c->a, phi, pi, A, piA, 0.5 * h);
        c->b += 0.5 * h * u1_kernel_a(p, c->a, E);
        double a1 = c->a + h * c->b;
        u1_drift_a(p, 0.5 * (c->a + a1), phi, pi, A, piA, h);
        c->a = a1;
        u1_kick(p, c->a, phi, pi, A, piA, 0.5 * h);
        u1_energy_plain(p, c->a, phi, pi, A, piA, E);
        c->b += 0.5 * h * u1_kernel_a(p, c->a, E);
        return;
    }
    double a0 = 1.0, am = 1.0, a1 = 1.0, b;
    if (p->expansion == ORC_FIXED) {
        u1_fixed_ab(p, t, &a0, &b);
        u1_fixed_ab(p, t + 0.5 * h, &am, &b);
        u1_fixed_ab(p, t + h, &a1, &b);
    }
    u1_kick(p, a0, phi, pi, A, piA, 0.5 * h);
    u1_drift_a(p, am, phi, pi, A, piA, h);
    u1_kick(p, a1, phi, pi, A, piA, 0.5 * h);
}

static void u1_vv(const orc_u1_params *p, double *const *phi, double *const *pi, double *const *A,
                  double *const *piA, orc_clock *c, int order, double t, double h)
{
    double w[45];
    const int n = orc_vv_stages(order, w);
    for (int i = 0; i < n; ++i) {
        u1_vv2(p, phi, pi, A, piA, c, t, w[i] * h);
        t += w[i] * h;
    }
}

int orc_u1_run_vv(const orc_u1_params *p, double *const *phi, double *const *pi, double *const *A,
                  double *const *piA, orc_clock *c, long nsteps, int order)
{
    if (c->lf_stag != 0) return -3;
    double h = nsteps >= 0 ? p->dt : -p->dt;
    long ns = nsteps >= 0 ? nsteps : -nsteps;
    double t_start = c->t;
    for (long k = 0; k < ns; ++k) u1_vv(p, phi, pi, A, piA, c, order, t_start + (double)k * h, h);
    c->t = t_start + (double)ns * h;
    if (p->expansion == ORC_FIXED) u1_fixed_ab(p, c->t, &c->a, &c->b);
    return 0;
}
