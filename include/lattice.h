/*
 * lattice.h -- C ABI of the MI355X (gfx950) lattice field step.
 *
 * The library evolves classical fields on a periodic N^3 lattice in an
 * expanding (FLRW) background with the symplectic kick/drift integrators of
 * the CosmoLattice paper (arXiv:2102.01031):
 *   - real scalar singlets (sec. 4.2 model, sec. 4.5.2 Hamiltonian form),
 *   - a U(1)-charged complex scalar with Abelian links (sec. 3.2 U(1)
 *     toolkit, sec. 5.2 equations of motion, sec. 5.5.2 kernels),
 *   - an SU(2) doublet with SU(2) links (sec. 3.2 SU(N) toolkit; sec. 5,
 *     eqs. higgsSU2-eom, SU2eom, GaussSU2-eom, energy-contrib).
 * All quantities are in the paper's program variables (sec. 4.1, eq.
 * FieldSpaceTimeNaturalVariables; sec. 5.1, eq. GaugeProgramVar).
 *
 * Layout.  Every field component is one contiguous array of N^3 elements
 * (float64, or float32 in LAT_PREC_F32 mode) in device memory, site
 * (x, y, z) at index x + N*(y + N*z), x fastest.
 *
 * Ownership.  The caller allocates and owns the field arrays and keeps them
 * alive until lattice_destroy.  lattice_step and lattice_sync overwrite them
 * in place: when a call returns (in stream order) the arrays hold the new
 * state.  The library owns only its scratch: one shadow copy of each field
 * array (stencil passes write out of place), reduction partials, the device
 * scale-factor record and per-pass coefficient tables; lattice_destroy frees
 * them.  Fields must not be modified by the caller while work enqueued by the
 * library is pending.
 *
 * Streams.  All device work is enqueued on the stream given to lattice_init
 * (a hipStream_t passed as void*, NULL = default stream).  lattice_step and
 * lattice_sync do not synchronise; lattice_energy synchronises the stream.
 * One context per stream; contexts are not internally locked.
 *
 * Errors.  Every call returns a lat_status.  Arguments are validated before
 * any launch, so a call that fails validation leaves the state untouched.
 * lattice_last_error(ctx) returns a description of the last failure of that
 * context (ctx = NULL: the last failure of lattice_init on this thread).
 * No C++ exception crosses this interface.
 */
#ifndef LATTICE_H
#define LATTICE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum lat_status {
    LAT_OK = 0,
    LAT_EINVAL = -1,        /* invalid argument (sizes, steps, null or misaligned pointers) */
    LAT_EUNSUPPORTED = -2,  /* valid but not provided combination (e.g. a gauge model in float32) */
    LAT_ENODEV = -3,        /* no usable GPU */
    LAT_EHIP = -4,          /* a HIP runtime call failed; see lattice_last_error */
    LAT_ESTATE = -5,        /* call not valid in the current state */
    LAT_ENOMEM = -6         /* device allocation failed */
} lat_status;

/* evolution algorithm (sec. 4.3 run parameters, "evolver"; sec. 4.5.2) */
enum lat_integrator {
    LAT_LF = 0,    /* staggered leapfrog, 2nd order: kick then drift, momenta half a step behind */
    LAT_VV2 = 1,   /* velocity-Verlet, 2nd order, fields and momenta at the same time */
    LAT_VV4 = 2,   /* 4th order: Yoshida triple-jump composition of three VV2 maps */
    LAT_VV6 = 3,   /* 6th order: Yoshida's solution A, 7 VV2 maps (7 kick points) per step */
    LAT_VV8 = 4,   /* 8th order: Yoshida's solution D, 15 VV2 maps per step */
    LAT_VV10 = 5   /* 10th order: triple jump of VV8 maps, S(x1 h) S(x0 h) S(x1 h) with
                      x1 = 1/(2 - c), x0 = -c/(2 - c), c = 2^{1/9}: 45 VV2 maps per step.
                      The VV family of sec. 4.3 (evolver VV2..VV10); the compositions are
                      those of Yoshida 1990, Phys. Lett. A 150, 262 (VV4: c = 2^{1/3}) */
};

/* background (sec. 4.3 "expansion", "fixedBackground"; eqs. NewFriedmannEQsII, ScaleFactorPowerLaw) */
enum lat_expansion {
    LAT_EXP_NONE = 0,   /* a = 1 (Minkowski) */
    LAT_EXP_FIXED = 1,  /* a(t) = a0 (1 + H0 (t - t_ref)/p)^p, p = 2/(3(1+w) - 2 alpha) */
    LAT_EXP_SELF = 2    /* a'' from the volume-averaged field energies (second Friedmann equation) */
};

/* model (potential and field content) */
enum lat_potential {
    LAT_PHI4 = 0,          /* one real field, V = lambda/4 phi^4 */
    LAT_PHI4_CHI2 = 1,     /* two real fields, V = lambda/4 phi^4 + q/2 phi^2 chi^2 (sec. 4.2) */
    LAT_ABELIAN_HIGGS = 2, /* complex phi = (phi0 + i phi1)/sqrt(2) + U(1) links,
                              V = lambda/4 (|phi|^2 - v^2)^2 */
    LAT_SU2_HIGGS = 3      /* doublet Phi = (phi0 + i phi1, phi2 + i phi3)/sqrt(2) + SU(2) links
                              U_i = exp(-i g dx B_i^a T_a), T_a = sigma_a/2, with the electric
                              field E_i^a conjugate to U_i under left multiplication;
                              V = lambda/4 (|Phi|^2 - v^2)^2, |Phi|^2 = sum_c phi_c^2/2.
                              Lattice Hamiltonian per site: sum_c pi_c^2/2
                              + sum_i |U_i psi(n+i) - psi(n)|^2/(2 dx^2) + V + |E|^2/2
                              + 2/(g^2 dx^4) sum_{i<j} (2 - Tr P_ij), psi = sqrt(2) Phi and
                              P_ij = U_i U_j(n+i) U_i(n+j)^dag U_j^dag (the toolkit plaquette);
                              kicks are minus its derivative, the link drift is
                              U <- exp(-i dt g dx E^a T_a) U.  Provided with LF and the VV
                              family (VV2 = kick(h/2) drift(h) kick(h/2), VV4..VV10 its symmetric
                              compositions) and every expansion, in float64; (f_star/omega_star)^2 = 1
                              (kappa_g is not used).  In an expanding background (sec. 5.5.2, eq.
                              kernelsSU21 and the one after it) the covariant Laplacian and the current
                              take a^{1+alpha}, the potential force a^{3+alpha}, the staple force
                              a^{alpha-1}; the doublet drifts with a^{alpha-3}, the links with
                              exp(-i dt a^{alpha-1} g dx E^a T_a); energies as the U(1) model's.  The
                              U(1) model has the same integrators and every expansion (see lattice_init). */
};

enum lat_precision {
    LAT_PREC_F64 = 0,      /* float64 fields and arithmetic */
    LAT_PREC_F32 = 1       /* float32 field storage and stencil arithmetic; float64 volume
                              reductions, scale factor, time and coefficients */
};

typedef struct lat_params {
    int32_t N;              /* lattice points per dimension, >= 2 */
    int32_t integrator;     /* enum lat_integrator */
    int32_t expansion;      /* enum lat_expansion */
    int32_t potential;      /* enum lat_potential */
    int32_t precision;      /* enum lat_precision */
    int32_t lf_staggered;   /* LF only: initial momentum phase, 0 = at integer time,
                               +1/-1 = half a step behind a forward/backward run (resume) */
    int32_t reserved0;
    int32_t reserved1;
    double dx;              /* lattice spacing, > 0 */
    double dt;              /* time step, > 0, dt/dx < 1/sqrt(3) (sec. 3.1 stability rule) */
    double t0;              /* initial time */
    double alpha;           /* alpha-time exponent (eq. FLRWmetric) */
    double lambda;          /* quartic coupling */
    double q;               /* LAT_PHI4_CHI2: q = g^2/lambda */
    double v;               /* LAT_ABELIAN_HIGGS: vacuum expectation value */
    double e_charge;        /* LAT_ABELIAN_HIGGS: e = g_A Q_A; LAT_SU2_HIGGS: g = g_B Q_B */
    double kappa_g;         /* LAT_ABELIAN_HIGGS: (f_star/omega_star)^2 */
    double kappa2;          /* LAT_EXP_SELF: (f_star/m_p)^2 */
    double w_eos;           /* LAT_EXP_FIXED: equation of state */
    double H0;              /* LAT_EXP_FIXED: Hubble rate a'/a at t_ref */
    double t_ref;           /* LAT_EXP_FIXED: reference time with a(t_ref) = a0 */
    double a0;              /* LAT_EXP_SELF: initial a; LAT_EXP_FIXED: a(t_ref) */
    double b0;              /* LAT_EXP_SELF: initial b = a'; NaN = from the Hubble constraint
                               (eq. NewFriedmannEQsI) on the initial fields (leapfrog with
                               lf_staggered != 0: b half a step behind, required) */
} lat_params;

typedef struct lat_fields {
    void *phi[2];   /* scalar arrays: LAT_PHI4 phi[0]; LAT_PHI4_CHI2 phi[0]=phi, phi[1]=chi;
                       LAT_ABELIAN_HIGGS the real components phi0, phi1 */
    void *pi[2];    /* conjugate momenta pi = a^{3-alpha} phi' (sec. 4.5.2), same layout */
    void *A[3];     /* LAT_ABELIAN_HIGGS: A_i on the link n -> n + i (sec. 3.2) */
    void *piA[3];   /* LAT_ABELIAN_HIGGS: pi_A,i = a^{1-alpha} F_0i (sec. 5.5.2) */
    void *doublet[4];     /* LAT_SU2_HIGGS: the real components phi0..phi3 of the doublet */
    void *pi_doublet[4];  /* LAT_SU2_HIGGS: their momenta pi_c = a^{3-alpha} phi_c' (eq. momSU2doublet) */
    void *U[12];          /* LAT_SU2_HIGGS: link n -> n + i, unit quaternion component k at
                             U[4 i + k], U = U[4i] I - i (U[4i+1], U[4i+2], U[4i+3]).sigma */
    void *E[9];           /* LAT_SU2_HIGGS: electric field E_i^a at E[3 i + a] (a = 0, 1, 2
                             for sigma_1..3), the momentum pi_B = a^{1-alpha} G_0i (eq. momSU2vec) */
} lat_fields;

typedef struct lat_energies {
    double t, a, b;          /* time, scale factor, b = a' */
    double EK[2];            /* kinetic energy per scalar field  <pi^2>/(2 a^6)  (eq. EK_EG_EV) */
    double EG[2];            /* gradient energy per scalar field <sum_i (grad+ phi)^2>/(2 a^2) */
    double EV[2];            /* potential energy per potential term */
    double EK_A, EG_A;       /* U(1) electric and magnetic energies */
    double rho;              /* total energy density */
    double hubble_lhs;       /* b^2 */
    double hubble_rhs;       /* a^{2 alpha + 2} kappa2 rho / 3 */
    double hubble_res;       /* (lhs - rhs)/(lhs + rhs) */
    double gauss_max;        /* U(1): max_n |G(n)|, G = div- piA - e kappa_g (phi0 pi1 - phi1 pi0);
                                SU(2): see gauss_abs_mean */
    double gauss_div_max;    /* max_n |div- piA| */
    double gauss_charge_max; /* max_n |e kappa_g (phi0 pi1 - phi1 pi0)| */
    double gauss_mean;       /* <|G|> */
    double gauss_sum_mean;   /* <|div- piA + charge|> */
    int64_t step;            /* steps taken since lattice_init (signed: backward steps subtract) */
    double EK_B, EG_B;       /* SU(2) electric <|E|^2>/2 and magnetic <2/(g^2 dx^4) sum_{i<j} (2 - Tr P_ij)> energies */
    double gauss_abs_mean;   /* <|div E| + |charge|>: the scale the Gauss residual is measured against.
                                SU(2) (eq. GaussSU2-eom): G^a = dx^-1 sum_i [E_i^a(n) - R(U_i(n-i))^a E_i(n-i)]
                                - g Im(psi^dag T_a pi_psi), R(U) E.sigma = U^dag (E.sigma) U, with the
                                Euclidean norm over a in the max and mean fields above */
} lat_energies;

typedef struct lat_ctx lat_ctx;

/* Create a context for the fields f (device pointers, see lat_fields) and
 * validate p.  Allocates the library scratch, computes b0 from the Hubble
 * constraint when asked, and leaves the fields untouched.
 * Leapfrog with LAT_EXP_SELF follows the staggered scheme of sec. 6.1 (fields
 * and a at integer times, momenta and b half a step behind; the b kick at time
 * n takes E_K as the mean of the kinetic energies of the momenta before and
 * after the momentum kick, the half kicks that leave or reach integer time
 * that of the momenta at the half step); a staggered start (lf_staggered != 0)
 * then needs b0 at the half step.
 * The gauge models take every expansion: in an expanding background their kicks
 * scale the covariant Laplacian and the current by a^{1+alpha}, the potential
 * force by a^{3+alpha} and the magnetic (SU(2): staple) force by a^{alpha-1},
 * their drifts are a^{alpha-3} pi and a^{alpha-1} pi_A (SU(2): the link
 * exponential of a^{alpha-1} E), their energies are divided by a^6, a^2, a^4
 * (kinetic, gradient, gauge), and the scale-factor kernel adds
 * (alpha - 1)(E_K^gauge + E_G^gauge) (sec. 5.5.2); with self-consistent expansion the
 * kicks, energy sums and drifts run as separate passes with the scale factor
 * updated on the device between them.
 * Errors: LAT_EINVAL, LAT_EUNSUPPORTED (the gauge models in float32),
 * LAT_ENODEV, LAT_ENOMEM, LAT_EHIP.  On error *ctx
 * is set to NULL. */
lat_status lattice_init(lat_ctx **ctx, const lat_params *p, const lat_fields *f, void *stream);

/* Create one context for a batch of n_real independent lattices that share p
 * (p->N is ignored) but have their own sizes N_per_real[r] and fields f[r].
 * Provided for LAT_PHI4 with LAT_LF and LAT_EXP_NONE or LAT_EXP_FIXED, float64 or
 * float32.  lattice_step on such a context advances every realization with
 * batched launches: the realizations are grouped into segments whose arrays
 * fit the GPU's last-level cache (128 MB of phi and pi per segment), and all
 * steps of a call run on one segment before the next (the realizations are
 * independent, so this changes no result); the launches of a call are
 * captured once into a HIP graph and replayed.  With autotune = 1 the mode of each distinct
 * lattice size (a tile shape and z chunk, or one thread per site) is chosen by
 * timing candidates on scratch buffers, first for that size alone, then with
 * every realization in the launch (the fields are not modified); otherwise a
 * fixed table is used (LATTICE_BATCH_TILE="tx,zc" or "site" overrides it).
 * lattice_energy_batch reads realization r; lattice_sync and lattice_destroy
 * act on all of them.  Errors: LAT_EUNSUPPORTED for other physics, LAT_EINVAL
 * for bad arguments or any realization failing lattice_init's checks; all are
 * reported before anything is allocated (*ctx stays NULL). */
lat_status lattice_init_batch(lat_ctx **ctx, const lat_params *p, int32_t n_real, const int32_t *N_per_real,
                              const lat_fields *f, int32_t autotune, void *stream);

/* Energies of realization r of a batch context (as lattice_energy). */
lat_status lattice_energy_batch(lat_ctx *ctx, int32_t r, lat_energies *out);

/* Discrete power spectrum (sec. 3.1, eq. discretePS) of one stored array:
 * field in [0, number of fields) (U(1): the two components of the complex
 * scalar; SU(2): the four components of the doublet, whose norm spectrum is
 * half the sum of the four), which = 0 for phi, 1 for pi (as stored: a staggered leapfrog state
 * gives pi at the half step).  Radial bins of unit width: bin b holds the modes
 * n (n_i in (-N/2, N/2]) with b <= |n| < b + 1; floor(sqrt(3) (N/2)) + 1 bins
 * hold every mode.  Outputs (host arrays of nbins): sum[b] = sum over the bin
 * of |f~(n)|^2 of the unnormalised forward DFT, count[b] = number of modes,
 * delta[b] = k_b^3/(2 pi^2) (dx/N)^3 sum[b]/(4 pi b^2) with k_b = b k_IR,
 * k_IR = 2 pi/(N dx) (delta[0] = 0), so that sum_{b>=1} (k_IR/k_b) delta[b]
 * = <f^2> - <f>^2 (eq. discretePSII).  Float64 transform (hipFFT) whatever
 * the field precision; bin sums are accumulated in an order that may vary at
 * the last bit.  The transform buffers (about 2 N^3 doubles) are allocated on
 * the first call.  Synchronizes the context stream.  Errors: LAT_EINVAL for a
 * batch context, a field or array out of range, or nbins outside [1, 448]. */
lat_status lattice_spectrum(lat_ctx *ctx, int32_t field, int32_t which, int32_t nbins, double *sum,
                            double *delta, int64_t *count);

/* Gauss-consistent initial gauge momenta (sec. 5.5.1, eqs. kAi1 and
 * GaugeCurrentFluc, on the lattice): overwrite the electric field
 * (LAT_SU2_HIGGS: E; LAT_ABELIAN_HIGGS: piA) with the longitudinal solution
 *   E_i = grad+_i Lap^-1 (rho - <rho>),  Lap = sum_i grad-_i grad+_i,
 * of the lattice Gauss law div- E = rho (eqs. GaussU1-eom and GaussSU2-eom at
 * a = 1 with unit links), rho the charge density of the stored scalar and
 * momenta: SU(2) rho^a = g Im(psi^dag T_a pi_psi) per colour, U(1)
 * rho = e kappa_g (phi0 pi1 - phi1 pi0).  The SU(2) solve needs every link at
 * the identity, the initial links of sec. 5.5.1 (LAT_ESTATE otherwise, nothing
 * written); the Abelian law does not involve the links.  mean_charge (host,
 * 3 doubles for SU(2), 1 for U(1); NULL skips) receives <rho^a>, the
 * homogeneous charge that no periodic field can absorb: after the call the
 * Gauss residual is -<rho^a> at every site (zero for charged fluctuations
 * whose modes carry no charge, as the paper's constrained phases give).
 * float64 hipFFT transforms; buffers and plans as lattice_spectrum's.
 * Synchronizes the stream.  Errors: LAT_EINVAL for other models or a batch
 * context, LAT_ESTATE, LAT_ENOMEM, LAT_EHIP. */
lat_status lattice_gauss_init(lat_ctx *ctx, double *mean_charge);

/* Lattice occupation number (eq. OccuppationNum, sec. 6.4 measurements)
 * of real scalar field `field` per radial bin (bins as lattice_spectrum):
 *   n[b] = (a^2 L^3 / (2 N^6)) fstar2 [ w_b S_phi(b) + a^{2(1-alpha)} S_x(b) / w_b ] / (4 pi b^2)
 * with L = N dx, S_phi(b) and S_x(b) the bin sums of |f~|^2 for phi_s and for
 * phi_s' + (a'/a) phi_s (phi' = a^{alpha-3} pi, the drift of sec. 4.5.2),
 * w_b^2 = k_b^2 + a^2 <d^2V/dphi_s^2> (volume average over the lattice), k_b = b k_IR,
 * fstar2 = (f_star/omega_star)^2 of the model's units, and a, a' those of the
 * current time (self-consistent, fixed or a = 1).  The shell average divides by
 * 4 pi b^2 as in eq. discretePS; count[b] gives the number of modes for a
 * per-mode mean.  n[0] = 0.  Host arrays of nbins.  Float64 transforms of
 * phi_s and pi_s (hipFFT); a second half-spectrum buffer is allocated on the
 * first call.  Synchronizes the context stream.  Errors: LAT_EINVAL for a batch
 * context, field outside [0, nfields), nbins outside [1, 448] or fstar2 <= 0;
 * LAT_EUNSUPPORTED for the U(1) model; LAT_ESTATE for leapfrog momenta at the
 * half step (call lattice_sync first). */
lat_status lattice_occupation(lat_ctx *ctx, int32_t field, int32_t nbins, double fstar2, double *n, int64_t *count);

/* Tile shape and z chunk the batch uses for lattice size N (host output);
 * tile_x = tile_y = z_chunk = 0 means one thread per site, no tiling. */
lat_status lattice_batch_tile(const lat_ctx *ctx, int32_t N, int32_t *tile_x, int32_t *tile_y, int32_t *z_chunk);

/* Advance |nsteps| time steps (sec. 4.5.2; LF and VV of sec. 4.3), backward
 * in time (dt -> -dt) when nsteps < 0.  For LF a backward run needs momenta at
 * integer time or staggered backward (LAT_ESTATE otherwise; call lattice_sync).
 * LF steps of real scalar fields with N <= 32 and no self-consistent
 * expansion run up to four steps per kernel launch (each block recomputes the
 * edge of its window, so the state agrees with one pass per step to
 * rounding); the number of launches is visible in lattice_stats.
 * Asynchronous on the context stream. */
lat_status lattice_step(lat_ctx *ctx, int64_t nsteps);

/* LF only: half-kick the momenta (and, with LAT_EXP_SELF, b) to integer time
 * in place (the sync before measurements of sec. 6.1).  The next step then
 * starts with a half kick; a sync followed by steps gives the trajectory of
 * the same steps without the sync.
 * No-op for VV integrators or already synchronised momenta. */
lat_status lattice_sync(lat_ctx *ctx);

/* Volume-averaged energies, Hubble and Gauss residuals of the current state
 * (sec. 4.4 outputs; sec. 5.4 Gauss measure).  LF momenta (and b with
 * LAT_EXP_SELF) are synchronised on the fly without writing them back.
 * Right after lattice_step with a VV integrator and LAT_EXP_SELF the volume
 * sums are those the step's last pass reduced for the scale-factor update
 * (the same state, at integer time), so no pass of its own runs; in that mode
 * the state is (fields, a, b) as the library left it, and a caller that
 * writes the field arrays between calls starts from a state a and b do not
 * follow.  Synchronises the stream; out is host memory. */
lat_status lattice_energy(lat_ctx *ctx, lat_energies *out);

/* Allocation-free variant of lattice_energy, for callers that cannot allocate
 * device memory: code under HIP graph capture, tight serving loops and
 * harnesses that forbid hipMalloc.  It takes no context: p and f describe a
 * real scalar state (LAT_PHI4 or LAT_PHI4_CHI2, float64 or float32 fields, as
 * for lattice_init; nothing is read beyond the fields' N^3 elements) and the
 * call enqueues on `stream` (a hipStream_t as void*, NULL = default stream)
 * the volume reductions lattice_energy performs on a context just created with
 * the same p and f: the scale factor a of p's start (1, the fixed background
 * at t0, or a0), and for leapfrog with lf_staggered != 0 the on-the-fly half
 * kick to integer time (nothing is written to the fields).
 * out: caller-owned device memory, 8 float64 values written in stream order:
 * EK[0], EK[1], EG[0], EG[1], EV[0], EV[1] (eq. EK_EG_EV; entries of an
 * absent second field 0), rho, a.  The call does not synchronise and does not
 * allocate: its partial sums, ticket counter and coefficients live in a fixed
 * 513 KiB device array that every GPU the library runs on holds until the
 * process ends (its address is looked up once per device, with that device
 * current; call with the stream's device current).  Every call on a GPU
 * shares that array, which keeps the last call's contents and is cleared where
 * needed by the call itself: calls that overlap on one GPU (other streams,
 * other threads) race and must be serialised by the caller.
 * Errors (reported by lattice_last_error(NULL), nothing enqueued):
 * LAT_EINVAL for what lattice_init refuses, a null or misaligned out, or a
 * lattice whose launch needs more block partials than the array holds
 * (65408 float64: every N up to 832; beyond that it depends on N's launch shape);
 * LAT_EUNSUPPORTED for the gauge models; LAT_ENODEV; LAT_EHIP. */
lat_status lattice_energy_noalloc(const lat_params *p, const lat_fields *f, double *out, void *stream);

/* observable of lattice_grad */
enum lat_observable {
    LAT_OBS_ENERGY_FRACTION = 0,      /* O = (E_K^s + E_G^s) / rho of field s at the final time
                                         (s = 1: the energy fraction in chi) */
    LAT_OBS_SPECTRUM_BIN = 1          /* O = Delta(b) of phi_s at the final time: bin b of the power
                                         spectrum of lattice_spectrum (sec. 3.1, eq. discretePS) */
};

typedef struct lat_grad_spec {
    int32_t observable;          /* enum lat_observable */
    int32_t field;               /* field s in {0, 1} of the observable */
    int64_t nsteps;              /* T >= 1 velocity-Verlet steps */
    int64_t checkpoint_stride;   /* steps between stored states; 0 = ceil(sqrt(T)) */
    int32_t bin;                 /* LAT_OBS_SPECTRUM_BIN: shell b, 1 <= b <= floor(sqrt(3) N / 2); otherwise 0 */
    int32_t reserved;            /* 0 */
} lat_grad_spec;

typedef struct lat_grad_out {
    double value;                /* O after T steps */
    double dO_dq;                /* total derivative of O with respect to q */
    void *dO_dphi[2];            /* caller-owned device arrays (N^3 float64) for dO/dphi_s(0); NULL skips */
    void *dO_dpi[2];             /* caller-owned device arrays for dO/dpi_s(0); NULL skips */
    double forward_ms;           /* duration of the forward sweep (HIP events) */
    double reverse_ms;           /* duration of the reverse sweep (HIP events) */
    double dO_da0, dO_db0;       /* self-consistent expansion: dO/da and dO/da' at the start, a' held
                                    as an independent input (0 otherwise) */
} lat_grad_out;

/* Gradient of an observable of the state after T steps with respect to the
 * current fields, momenta and the coupling q, by the hand-written adjoint of
 * the velocity-Verlet step (sec. 4.5.2 Hamiltonian system at a = 1): a forward
 * sweep storing the state every checkpoint_stride steps, the adjoint seeded at
 * T, and a reverse sweep that integrates the state backward together with the
 * adjoint, re-anchoring the state at every stored checkpoint.  On return the
 * fields hold their initial values again.  Provided for LAT_PHI4_CHI2 with
 * LAT_VV2 and LAT_PREC_F64, any expansion (LAT_EUNSUPPORTED otherwise).  On a
 * fixed background the steps run from the context's current time, kicks use
 * a^{1+alpha} and a^{3+alpha} at the kick time, drifts a^{alpha-3} at the
 * midpoint, and the energies of O are those at a(T).  With the self-consistent
 * expansion the forward sweep is the library's own step, one call per
 * checkpoint segment, recording a and a' of every step on the device; the
 * reverse sweep re-runs each segment from its checkpoint with those scale
 * factors and runs one fused adjoint pass per time point, the adjoints of a
 * and a' carried on the device.  a and a' at the start are independent inputs
 * (dO_da0, dO_db0; a caller whose a' comes from the Hubble constraint adds
 * dO_db0 times its derivative), and the scale factor, a', time and step count
 * are restored on return.  The library allocates the checkpoints (T/stride + 1
 * copies of the state), the adjoint arrays and, with the self-consistent
 * expansion, the stride + 1 states of a segment on first use and keeps them
 * until lattice_destroy.  N^3 must stay below 2^32 (LAT_EUNSUPPORTED).
 * LAT_OBS_SPECTRUM_BIN seeds the adjoint with dDelta(b)/dphi_s: the
 * unnormalised inverse transform of phi_s's spectrum kept on shell b, scaled
 * by 2 c_b (hipFFT float64 transforms; their buffers and plans are kept like
 * lattice_spectrum's).  A bad observable, field, bin or a nonzero reserved
 * member gives LAT_EINVAL.  Synchronises the stream. */
lat_status lattice_grad(lat_ctx *ctx, const lat_grad_spec *spec, lat_grad_out *out);

/* Launch statistics of the stencil kernels, per kernel kind:
 *   0 kick only, 1 kick only + reductions, 2 drift on load + kick,
 *   3 drift on load + kick + reductions, 4 kick + drift at end (leapfrog),
 *   5 energy (read only), 6 U(1) or SU(2) leapfrog (and their energy passes), 7 adjoint reverse pass.
 * kernel_ms is accumulated from HIP events recorded on the context stream around
 * each launch while profiling is on (lattice_profile); it stays 0 otherwise. */
typedef struct lat_stats {
    int64_t launches[8];
    double kernel_ms[8];
    int32_t blocks;       /* blocks per stencil launch */
    int32_t threads;      /* threads per block */
    int32_t tile_x, tile_y, z_chunk;
    int32_t pad;
} lat_stats;

/* Turn event timing of every stencil launch on (enable = 1) or off (0). */
lat_status lattice_profile(lat_ctx *ctx, int enable);

/* Copy the statistics into *out (host memory; synchronises the stream when
 * profiling); reset = 1 clears them afterwards. */
lat_status lattice_stats(lat_ctx *ctx, int reset, lat_stats *out);

/* Release the context and its scratch (waits for pending work).  NULL is ignored. */
void lattice_destroy(lat_ctx *ctx);

/* Text of the last error of ctx (NULL: last lattice_init failure on this thread). */
const char *lattice_last_error(const lat_ctx *ctx);

/* Library version string. */
const char *lattice_version(void);

#ifdef __cplusplus
}
#endif

#endif /* LATTICE_H */
