/*
 * cstar.h -- C ABI of libcstar.so: the Wilson-clover Dirac operator with C*
 * boundary conditions on MI355X (gfx950), its lowest eigenvalues and the sign
 * of the Pfaffian (arXiv:2108.11989, section "Sign of the Pfaffian").
 *
 * General conventions
 *  - Every entry point returns a cstar_status; no C++ exception crosses the ABI.
 *    On failure cstar_last_error() returns a thread-local message.
 *  - Host pointers are caller-owned and only read (or written, for outputs)
 *    during the call.  Device pointers are caller-owned allocations on the
 *    gauge handle's device; the library never frees them.
 *  - All device work runs on the handle's stream (the stream passed at
 *    creation; NULL = the default stream).  Calls returning host results are
 *    synchronous; dirac_apply / pack / unpack are asynchronous.
 *  - One handle must not be used from two threads at once.
 *
 * Lattice and fields (paper, simulation setup and sign-of-the-Pfaffian sections)
 *  - Physical lattice T x L^3, T and L even and >= 2; coordinates (t,x1,x2,x3),
 *    mu = 0 is t.  C* boundary conditions in space, periodic gauge field in
 *    time, fermion time phase time_bc = +1 (periodic) or -1 (antiperiodic).
 *  - C* is realised on the x-doubled lattice (x1 in [0,2L)): the sites with
 *    x1 >= L hold the charge-conjugate field, so the operator acts on
 *    2*T*L^3 sites x 12 complex components = the 24V x 24V matrix of the paper.
 *  - su3: [T][L][L][L][4][3][3] complex128 (interleaved re,im), lexicographic
 *    with t slowest and x3 fastest.  theta: [T][L][L][L][4] float64, the U(1)
 *    angle; the quark link is exp(i q theta) U.  Only the physical lattice is
 *    passed; the library builds the conjugate copy.
 *  - Operator: (D psi)(x) = (4+m0) psi(x) + SW(x) psi(x)
 *      - 1/2 sum_mu [(1-g_mu) V(x,mu) psi(x+mu) + (1+g_mu) V(x-mu,mu)^H psi(x-mu)],
 *    SW = (i/4) sum_{mu,nu} sigma_{mu nu} [c_su3 Fhat_{mu nu} + q c_u1 Fhat^{U(1)}_{mu nu}],
 *    Fhat = (Q - Q^H)/8 from the four clover leaves, chiral basis with
 *    g5 = diag(1,1,-1,-1), C = i g0 g2.  Q = g5 D is Hermitian.
 *
 * Spinor layouts
 *  - canonical: [nrhs][T][2L][L][L][4][3] complex (complex128 for CSTAR_FP64,
 *    complex64 for the FP32 precisions).
 *  - native (what dirac_apply and the solvers read): per right-hand side a
 *    contiguous block of cstar_spinor_bytes() bytes, laid out as
 *      FP64: double2 [parity 2][component 12][Vh][mirror 2]
 *      FP32: float4  [parity 2][component-pair 6][Vh][mirror 2]
 *    where Vh = T*L^3/2, parity = (t+x1+x2+x3) mod 2 of the physical site,
 *    the in-parity index is (lexicographic physical index)/2, "mirror" is 0
 *    for x1 < L and 1 for the conjugate copy at x1+L, and component =
 *    3*spin + colour.  cstar_spinor_pack / _unpack convert between the two.
 */
#ifndef CSTAR_H
#define CSTAR_H

#include <stddef.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct cstar_gauge cstar_gauge;

typedef enum {
    CSTAR_OK = 0,
    CSTAR_EINVAL = -1,  /* bad argument: sizes, NaN/Inf input, null pointer */
    CSTAR_ENOMEM = -2,  /* device or host allocation failed */
    CSTAR_EDEVICE = -3, /* HIP runtime error or no device */
    CSTAR_ENOCONV = -4, /* eigensolver hit max_iter before tol */
    CSTAR_EAMBIG = -5,  /* a sign could not be decided (eigenvalue at zero) */
    CSTAR_ESTATE = -6   /* handle in a state that does not allow the call */
} cstar_status;

typedef enum {
    CSTAR_FP64 = 0,           /* FP64 spinors, FP64 links (18 reals), FP64 clover */
    CSTAR_FP32 = 1,           /* FP32 spinors, FP32 links (rows 0,1 + phase angle), FP32 clover */
    CSTAR_FP32_BF16LINKS = 2  /* FP32 spinors, BF16 links (rows 0,1) + FP32 phase angle, FP32 clover */
} cstar_prec;

typedef struct {
    int T, L;        /* physical lattice T x L^3 (even, >= 2) */
    int time_bc;     /* +1 periodic, -1 antiperiodic fermion time boundary */
    double q;        /* quark charge in units of the U(1) link angle */
    double csw_su3;  /* SU(3) Sheikholeslami-Wohlert coefficient */
    double csw_u1;   /* U(1) Sheikholeslami-Wohlert coefficient */
} cstar_params;

/* Thread-local message of the last failing call on this thread. */
const char *cstar_last_error(void);

/*
 * Create a handle for one gauge field and one quark charge: copies su3/theta
 * to the device, packs the links in every precision and computes the clover
 * term in FP64 on the GPU.  src_on_device != 0: su3/theta are device pointers
 * (same layout); the call then moves no data over PCIe.
 * Errors: EINVAL for odd/small T, L, time_bc not +-1, non-finite parameters
 * or field entries; ENOMEM; EDEVICE.
 */
cstar_status cstar_gauge_create(const cstar_params *params, const double *su3, const double *theta,
                                int src_on_device, void *stream, cstar_gauge **out);
void cstar_gauge_destroy(cstar_gauge *g);

/* Bytes of one native spinor of precision prec (per right-hand side). */
size_t cstar_spinor_bytes(const cstar_gauge *g, cstar_prec prec);
/* Number of sites of the x-doubled lattice, 2*T*L^3. */
long cstar_n_sites(const cstar_gauge *g);

/* canonical <-> native conversion of nrhs spinors (device pointers, asynchronous). */
cstar_status cstar_spinor_pack(cstar_gauge *g, cstar_prec prec, int nrhs, const void *canonical, void *native);
cstar_status cstar_spinor_unpack(cstar_gauge *g, cstar_prec prec, int nrhs, const void *native, void *canonical);

/*
 * out_j = D(m_j) in_j   (gamma5 != 0: out_j = Q(m_j) in_j = g5 D(m_j) in_j),
 * j < nrhs, on the x-doubled lattice (paper: D is the 24V x 24V operator on
 * the quark/antiquark doublet).  in/out: native layout, device, nrhs blocks of
 * cstar_spinor_bytes(prec) each, non-aliasing.  masses: host[nrhs] bare m0.
 * nrhs == 1 runs the single-vector kernel; nrhs > 1 applies all right-hand
 * sides in one launch.  At L = 32 in the FP32 forms a lane applies two (or
 * four) right-hand sides, so each link and clover load serves that many;
 * the groups of right-hand sides of one lattice tile run together and
 * re-read the gauge field from L2 or memory.  The schedule is chosen by
 * timing the candidates on the first launch of a kind (or read from the
 * file named by CSTAR_TUNE_CACHE); every schedule gives the same bits.
 * Asynchronous on the handle's stream (the first launch of a kind
 * synchronises it while it times the schedules).
 * Errors: EINVAL (null pointer, nrhs < 1 or > 4096, a non-finite mass, an
 * unknown precision, in and out overlapping), EDEVICE.
 */
cstar_status dirac_apply(cstar_gauge *g, int nrhs, const double *masses, cstar_prec prec, int gamma5,
                         const void *in, void *out);

/*
 * For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same
 * operation, arguments, layouts and results as dirac_apply, with no device
 * allocation and no schedule measurement (a schedule already chosen by the
 * tuner, else a fixed default).  The per-RHS masses are staged in a
 * library-owned device array of CSTAR_NOALLOC_MAX_RHS doubles (8 KiB per GPU,
 * held until the process ends), shared by every call on that GPU: calls that
 * overlap on one GPU race on it.  Asynchronous on the handle's stream.
 * Errors: EINVAL (as dirac_apply, and nrhs > CSTAR_NOALLOC_MAX_RHS), EDEVICE.
 */
#define CSTAR_NOALLOC_MAX_RHS 1024
cstar_status dirac_apply_noalloc(cstar_gauge *g, int nrhs, const double *masses, cstar_prec prec, int gamma5,
                                 const void *in, void *out);

/*
 * Even-odd decomposition (paper, mass-reweighting section, eq. detQ2 and the
 * definition of W_eo).  Sites of the doubled lattice are even or odd by
 * parity (t+x1+x2+x3) mod 2; every hop changes it.  D_oo, the restriction of
 * D to the odd sites, is the site-local term (4+m) + SW(x), and
 *   D_hat = D_ee - D_eo D_oo^{-1} D_oe  (on the even sites),  Q_hat = g5 D_hat,
 *   det D = det D_oo det D_hat.
 * Even vector: the parity-0 half of a native spinor (its first
 * cstar_even_bytes() bytes), per right-hand side.
 */
size_t cstar_even_bytes(const cstar_gauge *g, cstar_prec prec);
/* out_j = D_hat(m0) in_j (gamma5 != 0: Q_hat), j < nrhs; in/out: device, nrhs
 * even vectors each, non-aliasing.  The first call at a mass computes the
 * inverse blocks of (4+m0) + SW on the odd sites in FP64 (kept for the next
 * calls at that mass); the handle allocates them and an odd-site scratch
 * vector per right-hand side on first use.  Asynchronous on the handle's
 * stream.  Errors: EINVAL, ENOMEM, EDEVICE. */
cstar_status dirac_eo_apply(cstar_gauge *g, int nrhs, double m0, cstar_prec prec, int gamma5, const void *in,
                            void *out);
/* log W_eo(m, m') = (1/2) log|det[D_oo(m') D_oo(m)^{-1}]|, exact, in FP64: the
 * sum over odd sites of the log-moduli of the 6x6 block determinants (the
 * conjugate copy of a site contributes the same modulus).  Synchronous.
 * Errors: EINVAL, ENOMEM, EDEVICE. */
cstar_status cstar_log_w_eo(cstar_gauge *g, double m, double m_prime, double *log_w_eo);

typedef struct {
    cstar_prec inner;        /* precision of the filter applies (FP64 or an FP32 form) */
    double tol;              /* target: residual ||Q v - lambda v|| <= tol * max(|lambda|, lambda_floor) */
    int max_iter;            /* outer iterations */
    int block;               /* vectors per block (>= 2k, <= 64; 0 = 2k + max(8, k)) */
    int degree;              /* Chebyshev filter degree (0 = automatic) */
    int use_nn;              /* 1: learned preconditioner attached to the handle, if any;
                                2: the residuals themselves as extra directions (no network) */
    int warm_start;          /* 1: start from the Ritz block of this handle's previous converged call */
    unsigned long long seed; /* start vectors */
} cstar_eig_opts;

typedef struct {
    int iterations;          /* outer iterations */
    long applies_fp64;       /* single-RHS D applications in FP64 */
    long applies_inner;      /* single-RHS D applications in the inner precision */
    double seconds;          /* wall time of the call */
    double lambda_max_est;   /* upper spectral bound used by the filter */
    long nn_applies;         /* network applications (use_nn) */
    int nn_fallback;         /* 1: the preconditioned solve failed and the plain solver answered */
} cstar_eig_stats;

/*
 * The k eigenvalues of Q(m0) = g5 D(m0) smallest in modulus, counted once
 * per Kramers pair (paper: the spectrum of Q is doubly degenerate; lambda_n,
 * n = 1..12V, lists each pair once), signed, sorted by |lambda| ascending
 * (ties: lambda ascending).  evals/resid: host[k]; resid[i] is the FP64
 * residual norm ||Q v_i - lambda_i v_i|| of a unit vector v_i, a rigorous
 * bound on the distance of lambda_i to the spectrum.  evecs: nullable device
 * pointer, k native FP64 spinors.  stats: nullable.  Synchronous.
 * Errors: EINVAL (k < 1, k > 30), ENOCONV (max_iter reached; evals/resid hold
 * the last iterate), ENOMEM, EDEVICE.
 */
cstar_status q_lowest_eigs(cstar_gauge *g, double m0, int k, const cstar_eig_opts *opts, double *evals,
                           double *resid, void *evecs, cstar_eig_stats *stats);

typedef struct {
    double tol;              /* stop when the half-width bound <= tol * lambda_bar (0 = 1e-3) */
    int degree;              /* Chebyshev degree per outer step, <= 64 (0 = 8) */
    int plain_steps;         /* plain power steps before the Chebyshev steps (0 = 3) */
    int max_outer;           /* outer steps (0 = 500) */
    int max_cg;              /* CG iterations per inner solve (0 = 20000) */
    unsigned long long seed; /* start vector */
    cstar_prec inner;        /* inner CG arithmetic: CSTAR_FP64 (default), or an FP32 form: FP32
                                arithmetic on the FP32-row operator for the solves whose tolerance
                                is 1e-6 or looser (FP64 for the tighter ones) */
} cstar_lbar_opts;

typedef struct {
    int outer;               /* outer (power or Chebyshev) steps */
    int solves;              /* inner CG solves of Q^2 x = y */
    long cg_iterations;      /* CG iterations over all solves */
    long applies_fp64;       /* single-RHS D applications in FP64 */
    double beta;             /* final upper end of the damped interval of Q^-2 (0: none used) */
    double resid_q2;         /* ||Q^2 v - theta v|| of the final unit vector */
    double seconds;          /* wall time of the call */
    long applies_inner;      /* single-RHS D applications in the FP32 form of opts.inner */
} cstar_lbar_stats;

/*
 * lambda_bar(m0) = min |lambda(Q(m0))| by the power method with Chebyshev
 * acceleration applied to Q(m0)^-2, as the paper proposes for step A of the
 * sign algorithm (Sec. 3: only the smallest eigenvalue of |Q| is needed);
 * every product with Q^-2 is a conjugate-gradient solve on Q^2, in FP64, or
 * with opts.inner an FP32 form in FP32 arithmetic on the FP32-row operator
 * while the solve's tolerance is 1e-6 or looser (the Rayleigh quotient and
 * the residual bound are always FP64, so the inner precision cannot bias
 * the bound).
 * lambda_bar: host, sqrt(theta) with theta = v^H Q^2 v the final Rayleigh
 * quotient (an upper bound of lambda_bar^2).  bound: nullable host, the
 * half-width of the interval around lambda_bar that holds |lambda| of some
 * eigenvalue of Q, from r = ||Q^2 v - theta v||:
 * max(sqrt(theta) - sqrt(theta - r), sqrt(theta + r) - sqrt(theta)).  That it
 * is the smallest one rests on the iteration's convergence, as in the paper.
 * opts, stats: nullable.  Allocates 8 FP64 vectors (and, with an FP32 inner
 * form, 5 FP32 vectors and one more FP64 vector) on the handle's device and
 * frees them before it returns.  Synchronous.
 * Errors: EINVAL (bad options), ENOCONV (max_outer reached; the outputs hold
 * the last iterate), ENOMEM, EDEVICE.
 */
cstar_status q_lambda_bar_power(cstar_gauge *g, double m0, const cstar_lbar_opts *opts, double *lambda_bar,
                                double *bound, cstar_lbar_stats *stats);

typedef struct {
    cstar_eig_opts eig;  /* eigensolver options for every mass point */
    int k;               /* eigenvalues per mass point (>= 1) */
    double c;            /* step-A factor, slightly below 2 (paper); 0 = 1.9 */
    double m_max;        /* mass above which no crossing is possible; <= 0: computed
                            from the largest clover norm on the handle */
    int step_a_power;    /* 1: step A upward from the lowest path mass with lambda_bar
                            from q_lambda_bar_power (the paper's order), the block
                            solver only above where step A stops; 0: the block solver
                            from m_max down */
    double lbar_tol;     /* relative accuracy of lambda_bar in step A (0 = 1e-3) */
} cstar_sign_opts;

typedef struct {
    int n_points;        /* mass points solved (m_max, step-A, bisection and the path points that need it) */
    double m[512];       /* the masses, in the order solved */
    double lambda_bar[512];
    int n_crossings;     /* certified zero crossings between the target and m_max */
    long applies;        /* single-RHS D applications (all precisions) */
    double seconds;
    long nn_applies;     /* network applications (opts.eig.use_nn) */
    int nn_fallbacks;    /* mass points where the plain solver answered for the preconditioned one */
} cstar_sign_report;

/*
 * Sign of the Pfaffian W_sgn(m_i) = sign pf[C T D(m_i)] at every mass of
 * m_path (paper: pf[CTD] = prod_n lambda_n, so the sign flips each time an
 * eigenvalue of Q crosses zero as m0 moves, and it is +1 at very large mass).
 * The flow is followed down from m_max (above which no eigenvalue can reach
 * zero) to min(m_path) with step A of the paper (m <- m - c*lambda_bar(m);
 * the Feynman-Hellmann bound |lambda_n'(m0)| <= 1 excludes a crossing within
 * lambda_bar of a solved mass); a segment where these exclusion intervals
 * do not cover it is resolved by counting eigenvalues that pass zero between
 * certified levels, splitting the segment if needed.  A path point is solved
 * only when it lies in a segment certified by counting; inside an
 * exclusion-covered segment it has the sign of the segment's upper end.
 * m_path: host[n], any order.  sign_out: host[n], +1 or -1.  report: nullable.
 * Errors: EINVAL; EAMBIG (an eigenvalue within its error bound of zero at a
 * path point; sign_out holds 0 there); ENOCONV; ENOMEM; EDEVICE.
 */
cstar_status pfaffian_sign(cstar_gauge *g, const double *m_path, int n, const cstar_sign_opts *opts,
                           int *sign_out, cstar_sign_report *report);

/*
 * Rational approximation of the mass-reweighting section (eq. ratapprox):
 * R(x) = A prod_{i<n} (x + nu2[i]) / (x + mu2[i]) ~ x^{-1/4} on [ra, rb],
 * optimal of order (n, n) in the uniform relative error, measured as
 * |log(R(x) x^{1/4})| (Remez exchange).  Outputs: A; nu2[n], mu2[n] (the
 * paper's nu_i^2 and mu_i^2, ascending, positive); delta, the attained
 * maximum of |log(R(x) x^{1/4})| on [ra, rb].  Host only, synchronous.
 * Errors: EINVAL (n outside [1, 32], not 0 < ra < rb), ENOCONV.
 */
cstar_status cstar_ratapprox_quartic(int n, double ra, double rb, double *A, double *nu2, double *mu2,
                                     double *delta);

/*
 * Mass-reweighting factor (paper, mass-reweighting section, eq. Wmass and the
 * stochastic estimator after it): W_mass = det[R(Q_hat_m^2) R^{-1}(Q_hat_m'^2)]
 * for R(x) = A prod_{i<n} (x + nu2[i]) / (x + mu2[i]) (e.g. from
 * cstar_ratapprox_quartic; A cancels), estimated factor by factor with the
 * caller's Gaussian sources eta on the even sites:
 *   W_i ~ (1/nsrc) sum_l exp(-x_il),  x_il = (eta_l, R_i eta_l),
 *   R_i = (1 + dD S_i)^H (1 + dD S_i) - 1,  dD = D_hat_m' - D_hat_m,
 *   S_i = (D_hat_m + i g5 nu_i)^{-1} - (D_hat_m' + i g5 mu_i)^{-1}
 *         - (D_hat_m' + i g5 mu_i)^{-1} dD (D_hat_m + i g5 nu_i)^{-1}
 * (nu_i = sqrt(nu2[i]), mu_i = sqrt(mu2[i])); the Gaussian average of
 * exp(-x_i) is det(1 + R_i)^{-1}, the i-th factor of W_mass.  Every inverse
 * is a solve of Q_hat^2 + s^2 to relative FP64 residual tol (iterative
 * refinement: FP32 conjugate gradients on the FP32-row operator against the
 * FP64 residual, FP64 CG if the refinement stops gaining) followed by one
 * Q_hat.  eta: device, nsrc FP64 even vectors (with
 * density proportional to exp(-(eta, eta)) for the estimator).  expo: host
 * [n][nsrc], the x_il; log_w_mass: host, sum_i log((1/nsrc) sum_l exp(-x_il)).
 * stats: nullable.  Allocates 13 FP64 and 5 FP32 even vectors and a 64 MiB
 * reduction buffer and frees them before it returns.  Synchronous.
 * Errors: EINVAL, ENOMEM, ENOCONV (a solve did not converge), EDEVICE.
 */
typedef struct {
    long cg_iterations;  /* over all solves */
    long eo_applies;     /* applications of D_hat or Q_hat (FP64 or FP32 rows) */
    double seconds;
} cstar_wmass_stats;
cstar_status cstar_w_mass(cstar_gauge *g, double m, double m_prime, int n, const double *nu2, const double *mu2,
                          int nsrc, const void *eta, double tol, double *expo, double *log_w_mass,
                          cstar_wmass_stats *stats);

/*
 * W_sgn over an ensemble (paper, sign-of-the-Pfaffian section and summary:
 * the sign of the Pfaffian is a reweighting factor of every configuration,
 * the product over the quark flavours).  For each configuration c < n_cfg
 * and flavour f < n_flv: the sign of pf[C T D(m_target[f])] for the field
 * (su3[c], theta[c]) with charge charges[f] and the other parameters of base
 * (base->q is ignored), by pfaffian_sign with opts; one GPU, in turn, a
 * handle created and destroyed per (configuration, flavour).  A flavour
 * equal to an earlier one (same charge and mass) reuses its sign.
 * su3[c], theta[c]: as in cstar_gauge_create (host, or device with
 * src_on_device).  sign_out: host [n_cfg][n_flv], +1 / -1 (0 where
 * undecidable); product_out: host [n_cfg], the product over flavours;
 * seconds_out: nullable host [n_cfg].  Synchronous.
 * Errors: EINVAL; EAMBIG (some sign undecidable: the other entries are
 * valid); the first other error of a creation or a sign, with its
 * configuration and flavour in the message (outputs of later
 * configurations unset).
 */
cstar_status cstar_sign_ensemble(const cstar_params *base, int n_cfg, const double *const *su3,
                                 const double *const *theta, int src_on_device, int n_flv, const double *charges,
                                 const double *m_target, const cstar_sign_opts *opts, int *sign_out, int *product_out,
                                 double *seconds_out);

/*
 * Host logic of pfaffian_sign over any eigenvalue provider (the same driver
 * pfaffian_sign uses; a provider may be a test double).  provider(ctx, m, k,
 * evals, errs) must fill the k eigenvalues of Q(m) smallest in modulus, one
 * per Kramers pair, signed, with rigorous error bounds errs[], sorted by
 * |lambda|, and return 0 (nonzero = failure, reported as ENOCONV).
 */
typedef int (*cstar_eig_provider)(void *ctx, double m, int k, double *evals, double *errs);
cstar_status cstar_sign_driver(cstar_eig_provider provider, void *ctx, const double *m_path, int n,
                               int k, double c, double m_max, int *sign_out, cstar_sign_report *report);

/*
 * Host logic of pfaffian_sign with step_a_power = 1, over any providers
 * (paper, sign-of-the-Pfaffian section, step A): from the lowest path mass
 * upwards, m <- m + c (lambda_bar(m) - err(m)), where lbar(ctx, m, &lb,
 * &err) gives lambda_bar(m) = min |lambda(Q(m))| and a rigorous error bound
 * (return 0; nonzero = failure, reported as ENOCONV).  Past m_max every
 * path point has sign +1.  When lambda_bar decreases, or two consecutive
 * exclusion intervals do not overlap, the range up to the previous step-A
 * mass is crossing-free, and cstar_sign_driver with provider decides the
 * sign there and at the path points above it (step B).  Errors as
 * cstar_sign_driver.
 */
typedef int (*cstar_lbar_provider)(void *ctx, double m, double *lambda_bar, double *err);
cstar_status cstar_sign_driver_a(cstar_lbar_provider lbar, cstar_eig_provider provider, void *ctx,
                                 const double *m_path, int n, int k, double c, double m_max, int *sign_out,
                                 cstar_sign_report *report);

/*
 * Kernel timing of the Dirac-apply launches issued on this handle (by
 * dirac_apply and by the solvers): when enabled, HIP events are recorded on
 * the handle's stream around every launch.  Per precision p (cstar_prec):
 * launches[p] kernel launches, rhs[p] right-hand sides they applied, ms[p]
 * summed kernel time, operands[p] extra input vectors read by fused epilogues
 * (out = a D in + b y + c z reads y and z: two per right-hand side).
 * enable(on) resets the counters; read synchronises the stream.  Errors:
 * EINVAL for a null handle; EDEVICE.
 */
typedef struct {
    long launches[3];
    long rhs[3];
    double ms[3];
    long operands[3];
} cstar_apply_timing;
cstar_status cstar_timing_enable(cstar_gauge *g, int on);
cstar_status cstar_timing_read(cstar_gauge *g, cstar_apply_timing *out);

/* Largest spectral norm over sites of the clover term SW(x) (bounds the
 * mass above which Q(m) has no eigenvalue near zero: sigma_min(D) >= m0 - this). */
cstar_status cstar_clover_norm_max(cstar_gauge *g, double *out);

/*
 * Learned preconditioner (not part of the paper's method): a gauge-covariant
 * network M of three linear parallel-transport convolution layers, channels
 * 1 -> 8 -> 8 -> 1.  A layer maps Cin spinor fields to Cout:
 *   out_a(x) = sum_b sum_p W[a][b][p] (T_p in_b)(x),
 * W[a][b][p] a complex 4x4 spin matrix, p = 0 the identity and p = 1 + 2 mu + d
 * the hop in direction mu (d = 0: V(x,mu) psi(x+mu); d = 1:
 * V(x-mu,mu)^H psi(x-mu)) on the handle's x-doubled C* lattice with its FP32
 * links.  It is trained towards (Q^2)^-1, L = (1/N) sum_i |M(Q^2 x_i) - x_i|^2
 * / |x_i|^2, and used by q_lowest_eigs (opts.use_nn = 1 and a network
 * attached): every iteration appends the preconditioned residuals
 * M (A x_j - theta_j x_j) of the 2k lowest Ritz pairs of A = Q^2 to the
 * Chebyshev-filtered block (the search space always contains the plain
 * one; 2 * block + 2k <= 128).  The plain solver answers if the
 * preconditioned one fails (stats.nn_fallback).
 *
 * Weights: CSTAR_NN_PARAMS floats, layers in order, each [Cout][Cin][9][4][4]
 * complex with (re, im) interleaved.  Vectors: FP32 native spinor blocks
 * (cstar_spinor_bytes(g, CSTAR_FP32) bytes each) on the device, the handle's
 * stream.  A network may serve several handles of one device, one at a time.
 */
#define CSTAR_NN_PARAMS 23040
typedef struct cstar_nn cstar_nn;

/* weights: host [CSTAR_NN_PARAMS] or NULL for the identity network.  EINVAL
 * (non-finite weight), ENOMEM. */
cstar_status cstar_nn_create(const float *weights, cstar_nn **out);
void cstar_nn_destroy(cstar_nn *nn);
cstar_status cstar_nn_get_weights(cstar_nn *nn, float *out);     /* host [CSTAR_NN_PARAMS] */
cstar_status cstar_nn_set_weights(cstar_nn *nn, const float *w);  /* host [CSTAR_NN_PARAMS] */
/* y_j = M(b_j), j < nvec.  b and y may be the same block (in place), not
 * otherwise overlapping.  Asynchronous on the handle's stream. */
cstar_status cstar_nn_apply(cstar_nn *nn, cstar_gauge *g, int nvec, const void *b, void *y);
/* Adds to the network's FP64 gradient the gradient of
 *   (1/n_total) sum_{i<nvec} |M(b_i) - x_i|^2 / |x_i|^2
 * (gradient g = dL/dRe W + i dL/dIm W, same layout as the weights) and
 * returns that partial loss.  Synchronous.  EINVAL for a zero x_i. */
cstar_status cstar_nn_loss_grad(cstar_nn *nn, cstar_gauge *g, int nvec, const void *x, const void *b, int n_total,
                                double *loss);
cstar_status cstar_nn_get_grad(cstar_nn *nn, double *out);        /* host [CSTAR_NN_PARAMS] */
cstar_status cstar_nn_zero_grad(cstar_nn *nn);
/* One Adam step (bias-corrected) with the accumulated gradient, which is then cleared. */
cstar_status cstar_nn_adam_step(cstar_nn *nn, double lr, double beta1, double beta2, double eps);
/* Training on GPU: for every field f (same lattice), b = Q(m0)^2 x in FP32 for
 * the nvec target vectors x[f] (device FP32 native block); then `epochs`
 * passes over the fields in order, one Adam step (lr, 0.9, 0.999, 1e-8) per
 * field on the loss of its nvec pairs.  loss_history: nullable host[epochs],
 * the mean loss of each pass.  ENOCONV if the loss becomes non-finite. */
cstar_status cstar_nn_train(cstar_nn *nn, cstar_gauge *const *fields, int n_fields, const void *const *x, int nvec,
                            double m0, int epochs, double lr, double *loss_history);
/* Network used by q_lowest_eigs / pfaffian_sign on this handle when
 * opts.use_nn = 1 (not owned; NULL detaches). */
cstar_status cstar_nn_attach(cstar_gauge *g, cstar_nn *nn);

#ifdef __cplusplus
}
#endif
#endif
