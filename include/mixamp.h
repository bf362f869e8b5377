/*
 * mixamp: likelihood of the time-dependent amplitude model of
 * D0 -> K+ pi- pi+ pi- on AMD Instinct MI355X (gfx950).
 *
 * Method: Hasse et al., "Amplitude analysis of four-body decays using a
 * massively-parallel fitting framework" (arXiv:1702.06735):
 *   - Sec. 3, Eq. (2): A_f = sum_i c_i A_i, Abar_f = sum_i cbar_i A_i over
 *     quasi-two-body decay chains (spin factors, barrier factors, Breit-Wigner
 *     lineshapes, Bose symmetrisation over the two pi-);
 *   - Sec. 2, Eq. (1): the time-dependent rate B(Phi, t) in x, y and Gamma;
 *   - Sec. 3.1: normalisation by a Monte Carlo average over uniform phase
 *     space, here of B integrated over t in [0, inf) in closed form;
 *   - NLL = sum_data (Gamma t_i - ln B_i) + n_data ln(Nhat),
 *     Nhat = (1/n_mc) sum_mc T_j, T_j the time-integrated rate of MC event j.
 *
 * Conventions.
 *   Units GeV and ps. An event is 16 doubles: the four-momenta (E,px,py,pz)
 *   of K+, pi-(a), pi+, pi-(b), in that order, in the D0 rest frame.
 *   Parameter vector theta (n_theta = 2 (n_a + n_ab) + 8 doubles): (Re, Im) of
 *   the A_f coefficients in the order of mxa_model_desc.comp_a, then of the
 *   Abar_f coefficients in the order of comp_ab, then x, y, then mass and width
 *   of K*(892)0, rho(770)0 and a1(1260) [GeV].
 *
 * Errors. Every call returns an int32_t status (MXA_OK or a negative code);
 * no exception crosses this interface. mxa_last_error() gives a thread-local
 * message for the last failing call of the calling thread.
 *
 * Threads and streams. A context is bound to one device and, at a time, one
 * HIP stream (given at creation, changed by mxa_set_stream), and is not
 * thread-safe: use it from one thread at a time. Calls that return host
 * values synchronise that stream only. A fit server is
 * thread-safe: its calls may come from any thread, and one worker thread per
 * server, on a stream of its own, does all of its device work.
 */
#ifndef MIXAMP_H
#define MIXAMP_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define MXA_OK 0
#define MXA_EINVAL (-1)    /* bad argument, size, or event record */
#define MXA_ENOMEM (-2)    /* device or host allocation failed */
#define MXA_EDEVICE (-3)   /* no usable GPU, or a HIP runtime error */
#define MXA_EDOMAIN (-4)   /* theta outside the model's domain, or B_i <= 0 */
#define MXA_EAGAIN (-5)    /* result not ready yet */
#define MXA_ENOTFOUND (-6) /* unknown handle or ticket */

#define MXA_DATA 0 /* decay-time-tagged events entering sum ln B_i */
#define MXA_MC 1   /* uniform phase-space events entering Nhat */
#define MXA_DATA_BAR 2 /* models with cpv = 1: D0bar-tagged events, records
                          (K-, pi+(a), pi-, pi+(b)) in the D0bar rest frame;
                          the library takes their CP conjugate (3-momenta
                          negated, each slot read as its antiparticle) */

/* Arithmetic of an evaluation. MXA_FP64: everything in FP64.
 * MXA_FP32AMP: the per-event cache, lineshapes and amplitude sums in FP32;
 * Eq. (1), its time integral, logarithms and every sum over events in FP64. */
#define MXA_FP64 0
#define MXA_FP32AMP 1

/* Model description (Sec. 3: the user composes decay chains into A_f and
 * Abar_f). Basis chain index k (1..8), each Bose symmetrised:
 *   1 D->K*0 rho0 S-wave, 2 P-wave, 3 D-wave; 4 D->(K+pi-)_S rho0;
 *   5 D->a1(1260)- K+, a1->rho0 pi- S-wave; 6 same, D-wave;
 *   7 D->K1(1270)+ pi-, K1->K*0 pi+; 8 D->K1(1400)+ pi-, K1->K*0 pi+.
 * Lineshapes: K*0 and rho0 relativistic Breit-Wigner with mass-dependent
 * width and Blatt-Weisskopf barrier B'_1; a1 and K1 with constant width and
 * barrier B'_L at their decay vertex (q0 at the nominal K*0/rho0 mass);
 * barrier factor F_L(q_D) at the D vertex; radius r at every vertex. */
typedef struct mxa_model_desc {
  double m_D, m_K, m_pi;      /* parent and final-state masses [GeV] */
  double gamma;               /* D0 width Gamma = 1/tau [1/ps] */
  double r;                   /* Blatt-Weisskopf radius [1/GeV] */
  double m_ks_ref, m_rho_ref; /* nominal K*0 and rho0 masses used in the
                                 break-up momentum q0 of a1 and K1 */
  double m_k1a, g_k1a;        /* K1(1270)+ mass and width (fixed) */
  double m_k1b, g_k1b;        /* K1(1400)+ mass and width (fixed) */
  int32_t n_a, n_ab;          /* number of chains in A_f and Abar_f (0..8) */
  int32_t comp_a[8];          /* chain indices (1..8) of A_f, distinct */
  int32_t comp_ab[8];         /* chain indices (1..8) of Abar_f, distinct */
  double g_bkg;               /* > 0: the data hold a background component,
                                 uniform in phase space with decay times from
                                 g_bkg exp(-g_bkg t) [1/ps], whose fraction f
                                 is the last parameter; each data event's
                                 density is then (1 - f) B e^{-Gamma t} / Nhat
                                 + f g_bkg e^{-g_bkg t} and the NLL is minus
                                 the sum of its logarithms (an extension of
                                 the paper's model, which has none; contexts
                                 in either MC mode, mxa_nll_multi and the fit
                                 server of mxa_server_create). 0: no
                                 background component */
  int32_t cpv;                /* 1: CP violation in mixing (an extension; Eq.
                                 (1) assumes none): q/p = |q/p| e^{i phi} is
                                 free, |q/p| and phi the two parameters after
                                 the standard ones (before f with g_bkg > 0);
                                 D0-tagged data (MXA_DATA) have Eq. (1) with
                                 Abar_f -> (q/p) Abar_f, D0bar-tagged data
                                 (MXA_DATA_BAR) with Abar_f -> (p/q) Abar_f,
                                 each flavour its own normalisation, and
                                 NLL = sum (Gamma t - ln B) + n_D0 ln Nhat_D0
                                 + n_D0bar ln Nhat_D0bar; with g_bkg > 0 each
                                 flavour's signal term takes its own Nhat in
                                 the mixture density, the background and f
                                 shared. Not the fit server or mxa_nll_multi.
                                 0: off */
  double sigma_t;             /* > 0: Gaussian decay-time resolution of this
                                 width [ps] (an extension; Eq. (1) is for
                                 exact times): each data event's rate is
                                 Eq. (1) times e^{-Gamma t} convolved with the
                                 resolution, at the measured time (which may
                                 be negative), and the data term is minus its
                                 logarithm; the normalisation is unchanged.
                                 With g_bkg > 0 the background's decay
                                 times are convolved with it too. Not with
                                 the streamed fit server or data generation.
                                 0: none */
} mxa_model_desc;

typedef struct mxa_ctx mxa_ctx;

/* Number of parameters 2 (n_a + n_ab) + 8 (+ 1 with a background
 * component, + 2 with CP violation), or MXA_EINVAL for a bad model. */
int32_t mxa_n_theta(const mxa_model_desc* model);

/* Create a context on HIP device `device`, launching on `stream` (a
 * hipStream_t; NULL = the device's null stream). The model is copied.
 * *out receives the context (owned by the caller, freed by mxa_destroy).
 * Errors: MXA_EINVAL (bad model), MXA_EDEVICE (no such device). */
int32_t mxa_create(const mxa_model_desc* model, int32_t device, void* stream, mxa_ctx** out);

/* Free the context and all device memory it owns. NULL is accepted. */
int32_t mxa_destroy(mxa_ctx* ctx);

/* Load a sample (Secs. 3.1 and 5: data to fit, or phase-space MC for the
 * normalisation), replacing any previous sample of that kind.
 * p4: host [n][16] doubles; t: host [n] decay times [ps] for MXA_DATA and
 * MXA_DATA_BAR (NULL for MXA_MC). Both are borrowed for the duration of the call only. The call
 * validates every event (finite; |sum p - (m_D,0,0,0)| <= 1e-6 GeV per
 * component; |p_i^2 - m_i^2| <= 1e-6 GeV^2; 0 <= t < inf) and builds the
 * parameter-independent per-event cache on the device. n = 0 clears the
 * sample. Errors: MXA_EINVAL (bad kind, n < 0, NULL array, or an event that
 * fails validation: then the previous sample of that kind is gone),
 * MXA_ENOMEM. Synchronises the context's stream. */
int32_t mxa_load_events(mxa_ctx* ctx, int32_t kind, const double* p4, const double* t, int64_t n);

/* As mxa_load_events, but p4 and t are device pointers on the context's
 * device (for example torch tensors' data_ptr()), read by the device during
 * the call only. */
int32_t mxa_load_events_device(mxa_ctx* ctx, int32_t kind, const double* d_p4, const double* d_t,
                               int64_t n);

/* Number of events currently loaded for `kind`. */
int32_t mxa_sample_size(mxa_ctx* ctx, int32_t kind, int64_t* n);

/* Set theta (host, n_theta doubles, copied). Errors: MXA_EINVAL (wrong
 * n_theta, NULL); MXA_EDOMAIN (non-finite value, |y| >= 1, a width <= 0,
 * a mass at or below its decay threshold). */
int32_t mxa_set_params(mxa_ctx* ctx, const double* theta, int32_t n_theta);

/* Evaluate the NLL at the current theta: a data pass, an MC pass and the
 * reduction of their sums on the context's stream, then the NLL from the
 * sums on the host. *nll_out receives it. diag (may be NULL) receives 4 doubles: Nhat,
 * sum over data of (Gamma t_i - ln B_i), the scale S = sum |Gamma t_i - ln B_i|
 * + n_data |ln Nhat|, and the number of data events with B_i <= 0.
 * Errors: MXA_EINVAL (no MC loaded, bad precision, no theta set),
 * MXA_EDOMAIN (some B_i <= 0 or non-finite, or Nhat <= 0: *nll_out = +inf). */
int32_t mxa_nll(mxa_ctx* ctx, int32_t precision, double* nll_out, double* diag);

/* As mxa_nll, plus grad_out[0..n_theta-1] = dNLL/dtheta from a hand-written
 * adjoint in the same pass. */
int32_t mxa_nll_grad(mxa_ctx* ctx, int32_t precision, double* nll_out, double* grad_out,
                     double* diag);

/* mxa_nll_grad for callers that cannot allocate device memory (code under
 * graph capture, tight serving loops, harnesses that forbid hipMalloc): the
 * same kernels and the same result, bit for bit, but the per-workgroup
 * partial sums and the slot totals of the evaluation go to a fixed array
 * that every device running the library holds for the life of the process
 * (1.4 MiB: 2048 workgroups x 45 sums x (sum, error), plus 128 totals),
 * not to buffers the context allocates on first use. The call allocates
 * nothing; the context's own buffers (samples, result record) come from
 * mxa_create and mxa_load_events as before. A call writes every word of the
 * array it reads, so nothing needs clearing between calls. Calls on one
 * device share the array: calls that overlap in time on one device (other
 * contexts or streams) race, and the caller must serialise them.
 * Direct MC mode only: MXA_EINVAL in MXA_MC_GRAM mode (whose Gram matrix is
 * built on demand). Other errors as mxa_nll_grad; MXA_EINVAL if a launch
 * needed more than the array holds (no sample within the library's limits
 * does). */
int32_t mxa_nll_grad_noalloc(mxa_ctx* ctx, int32_t precision, double* nll_out, double* grad_out,
                             double* diag);

/* Per-event diagnostics of the loaded sample `kind` at the current theta:
 * out (host, [n][5] doubles, caller-owned): |A|^2, |Abar|^2, Re(A Abar*),
 * Im(A Abar*), and the rate: Eq. (1) at t_i for MXA_DATA, its time integral
 * for MXA_MC. */
int32_t mxa_event_terms(mxa_ctx* ctx, int32_t kind, int32_t precision, double* out);

/* Normalisation mode. MXA_MC_DIRECT (default): every evaluation makes a pass
 * over the MC sample. MXA_MC_GRAM: the masses and widths are treated as
 * fixed; the MC sum becomes quadratic forms in the coefficients with the
 * Gram matrix G_kl = sum_j B_k,j conj(B_l,j) of the chain amplitudes (built
 * on first use and again whenever the masses, widths or precision change),
 * and an evaluation streams the data only. The gradient entries of the
 * masses and widths are then NaN. */
#define MXA_MC_DIRECT 0
#define MXA_MC_GRAM 1
int32_t mxa_set_mc_mode(mxa_ctx* ctx, int32_t mode);

/* Build the MC Gram matrix at the current masses and widths (Sec. 3.1
 * normalisation with fixed lineshapes; matrix cores, FP64 accumulation) and,
 * if out is not NULL, copy it: out[(8 k + l) * 2 + {0, 1}] = Re, Im of
 * sum_j B_k,j conj(B_l,j) over the MC events, chains k, l = 1..8 at index
 * k-1, l-1 (zero rows and columns for chains in neither amplitude). */
int32_t mxa_gram(mxa_ctx* ctx, int32_t precision, double* out);

/* Many parameter sets that share the masses and widths (for example the
 * points of a numerical-gradient stencil, or a scan of the coefficients and
 * x, y): nll_out[s] (host, caller-owned, n_sets doubles) = the NLL at
 * thetas[s * n_theta .. s * n_theta + n_theta - 1] (host, row-major
 * [n_sets][n_theta]), 1 <= n_sets <= MXA_MAX_SETS. Per data event the chain
 * amplitudes are computed once and every set's A_f, Abar_f (Eq. (2)) follow
 * from one dense product on the matrix cores; the normalisation of every set
 * comes from the MC Gram matrix (built, or reused, as in MXA_MC_GRAM mode).
 * With a background component each set's data term takes that set's Nhat
 * (from the Gram matrix) and fraction; with a resolution, the resolved rate.
 * A set outside the model's domain, or with some B_i <= 0, gets +inf. The
 * context's parameters become the first set inside the domain. Errors:
 * MXA_EINVAL (sizes, NULL, sets with different masses or widths, no MC
 * sample, a model with CP violation), MXA_EDOMAIN (no set inside the
 * domain), MXA_EDEVICE, MXA_ENOMEM. */
#define MXA_MAX_SETS 64
int32_t mxa_nll_multi(mxa_ctx* ctx, int32_t precision, const double* thetas, int32_t n_sets,
                      double* nll_out);

/* Rebind the context to `stream` (a hipStream_t of the context's device;
 * NULL = the device's null stream) for the calls that follow, so that each
 * call can be issued on the caller's stream of the moment. Work queued on
 * the previous stream is waited for first, so that two streams never touch
 * the context's buffers at once. Errors: MXA_EINVAL (NULL context, or a
 * stream of another device), MXA_EDEVICE. */
int32_t mxa_set_stream(mxa_ctx* ctx, void* stream);

/* Kernel timing: when on, the MC pass of every mxa_nll / mxa_nll_grad call
 * (the dominant kernel of an evaluation) is bracketed by HIP events on the
 * context's stream; recording them adds a few microseconds per call.
 * mxa_kernel_time returns the summed duration [ms] and count of timed
 * launches since the last reset (reset = 1 clears them after reading). */
int32_t mxa_set_timing(mxa_ctx* ctx, int32_t on);
int32_t mxa_kernel_time(mxa_ctx* ctx, double* ms_total, int64_t* launches, int32_t reset);

/* Launch geometry of the data and MC passes for the loaded samples:
 * out4 = {workgroups, events per workgroup} of data, then of MC. */
int32_t mxa_launch_shape(mxa_ctx* ctx, int32_t grad, int64_t* out4);

/* ------------------------------------------------------------------------
 * Pseudo-experiments (Sec. 3.1 and the generation timing of Table 2):
 * candidates uniform in four-body phase space by GENBOD (F. James, CERN
 * 68-15, 1968), with decay times and accept-reject against Eq. (1) for data.
 *
 * Candidate i (i = first, first + 1, ...) of a sample with seed s takes 12
 * uniforms from Philox4x32-10 (Salmon et al., SC11): block j = 0..5 has
 * counter (i mod 2^32, i div 2^32, j, stream) and key (s mod 2^32,
 * s div 2^32), stream 0 for MXA_MC and 1 for MXA_DATA; each block gives two
 * uniforms (k + 1/2) 2^-52, k the top 52 bits of output words (0, 1) and
 * (2, 3). Uniforms 0, 1 pick the intermediate masses, 2 the GENBOD
 * acceptance u wmax < weight, 3..8 the three decay directions, 9, 10 the
 * decay time from exp(-Gamma t) cosh(y Gamma t), 11 the data acceptance
 * u E < B(Phi, t) with E = 2 cosh(y Gamma t) envelope, envelope a bound of
 * |A|^2 + |Abar|^2. All decisions are FP64.
 * ------------------------------------------------------------------------ */
typedef struct mxa_gen_stats {
  int64_t n_candidates;  /* candidates examined: first .. first + n_candidates - 1 */
  int64_t n_phase_space; /* of those, kept by the GENBOD weight */
  int64_t n_exceed;      /* MXA_DATA: of those, rate above the envelope (the draw
                            is then biased; redraw with a larger envelope) */
  uint64_t next;         /* first + n_candidates: the first candidate of a continuation */
} mxa_gen_stats;

/* Generate the first n kept events from candidate `first` on. kind MXA_MC:
 * uniform phase space; MXA_DATA: pseudo-data at the context's parameters
 * (mxa_set_params first). wmax: bound of the GENBOD weight (0: the library's
 * own, 1.01 x the maximum over a 1001 x 1001 grid of the two sorted
 * uniforms); envelope: M_Phi (MXA_DATA only). Outputs are DEVICE arrays on
 * the context's device, caller-owned: d_p4 [n][16] in the event layout of
 * mxa_load_events, d_t [n] (MXA_DATA; ignored for MXA_MC), d_idx [n] the
 * candidate index of each event (or NULL). Events come in candidate order;
 * the result does not depend on how the work is split. Synchronous.
 * Errors: MXA_EINVAL, MXA_EDEVICE, MXA_ENOMEM; MXA_EDOMAIN if fewer than
 * one candidate in 2^17 is kept. */
int32_t mxa_generate(mxa_ctx* ctx, int32_t kind, uint64_t seed, uint64_t first, int64_t n,
                     double wmax, double envelope, double* d_p4, double* d_t, int64_t* d_idx,
                     mxa_gen_stats* stats);

/* ------------------------------------------------------------------------
 * Fit server: continuous batching of pseudo-experiment fits (the toy studies
 * of Sec. 4). Each fit minimises the NLL of its own data over the free
 * coefficients and x, y (BFGS with a backtracking line search); the masses
 * and widths are fixed at the server's values, so the normalisation comes
 * from one shared MC Gram matrix and an evaluation streams the fit's data
 * only. A scheduler thread admits queued fits while a slot and the HBM
 * budget allow, evaluates every active fit in one batched device call per
 * tick (the totals of every fit reduced into host memory, where each fit's
 * NLL and gradient are formed), and frees a finished fit's slot and memory
 * at once.
 * A fit's result does not depend on the fits it shares launches with.
 * Models with a background component (g_bkg > 0: each fit also floats or
 * fixes the background fraction, the last parameter; every tick forms each
 * fit's Nhat from the Gram matrix before its data pass) or a decay-time
 * resolution (sigma_t > 0: data times may be negative) are served by
 * mxa_server_create; models with CP violation are not served.
 * The server functions are thread-safe.
 * ------------------------------------------------------------------------ */
#define MXA_MAX_THETA 40
#define MXA_FIT_QUEUED 0
#define MXA_FIT_RUNNING 1
#define MXA_FIT_CONVERGED 2
#define MXA_FIT_MAX_EVALS 3
#define MXA_FIT_FAILED 4
#define MXA_FIT_CANCELLED 5

typedef struct mxa_server mxa_server;

typedef struct mxa_fit_request {
  const double* p4;     /* [n][16] data events: host memory, copied by
                           mxa_fit_submit (or see events_on_device) */
  const double* t;      /* [n] decay times [ps], likewise */
  int64_t n;            /* 1 .. 524288 events */
  const double* theta0; /* n_theta start values (the masses and widths are
                           ignored by a server with fixed lineshapes) */
  const double* scale;  /* n_theta step scales; 0 fixes a parameter; the
                           minimiser works in theta / scale */
  int32_t max_evals;    /* evaluation cap (<= 0: 150) */
  double gtol;          /* converged when max |dNLL / d(theta/scale)| < gtol (<= 0: 1e-3) */
  double ftol;          /* or when two accepted steps each lower the NLL by
                           less than ftol max(1, |NLL|) (0: off) */
  double edm_tol;       /* or when the estimated distance to the minimum,
                           g^T H^-1 g / 2 with the minimiser's inverse-Hessian
                           estimate, falls below edm_tol (0: off; 1e-4 is the
                           usual choice for an NLL) */
  int32_t errors;       /* 1: after the minimisation, the covariance of the free
                           parameters from the Hessian of the NLL by central
                           differences of the gradient (2 evaluations per free
                           parameter, counted in n_evals); 0: none */
  int32_t gradient;     /* MXA_GRAD_ADJOINT (0): the library's adjoint;
                           MXA_GRAD_CENTRAL (1, mxa_fit with MXA_FP64 only): the
                           gradient of the free parameters by central
                           differences of the NLL with steps 1e-4 scale_i (the
                           numerically differentiated fit of Sec. 5): in
                           MXA_MC_GRAM mode, with the masses and widths fixed,
                           all 2 n_free + 1 points in one mxa_nll_multi call
                           (n_free <= 31), otherwise one mxa_nll per point */
  int32_t events_on_device; /* mxa_fit_submit only. 1: p4 and t are device
                           pointers on the server's device (for instance
                           pseudo-experiments from mxa_generate), ready when
                           the call is made; no copy is made: the fit's
                           admission reads them in place, so the caller keeps
                           them allocated and unchanged until the fit has
                           finished. 0: host pointers, copied by the call.
                           Errors: MXA_EINVAL if the pointers are not device
                           memory of the server's device. */
} mxa_fit_request;
#define MXA_GRAD_ADJOINT 0
#define MXA_GRAD_CENTRAL 1

typedef struct mxa_fit_result {
  double theta[MXA_MAX_THETA]; /* best point (n_theta entries) */
  double nll;                  /* NLL there */
  double grad_norm;            /* max |dNLL / d(theta/scale)| there */
  int32_t n_evals;             /* NLL+gradient evaluations used */
  int32_t status;              /* MXA_FIT_CONVERGED, _MAX_EVALS, _FAILED, _CANCELLED */
  int64_t n;                   /* data events */
  int64_t t_submit_ns, t_start_ns, t_done_ns; /* steady clock: submit, admission, done */
  int32_t errors_ok;           /* errors requested, Hessian positive definite */
  double err[MXA_MAX_THETA];   /* errors (0 for fixed parameters, and unless errors_ok) */
  double grad[MXA_MAX_THETA];  /* dNLL/dtheta at the best point (n_theta entries); the
                                  mass and width entries are NaN for a server with
                                  fixed lineshapes (the Gram normalisation has no
                                  lineshape derivative) */
  int64_t n_points;            /* NLL evaluations made: n_evals with the adjoint,
                                  n_evals (2 n_free + 1) with central differences */
} mxa_fit_result;

/* One fit of the context's loaded data sample (Sec. 4 fits: for example x and
 * y floating with the model fixed, the setting of the paper's fit-time
 * benchmark and sensitivity study). Minimises the NLL of mxa_nll_grad (with
 * the context's normalisation mode, MXA_MC_DIRECT or MXA_MC_GRAM) over the
 * parameters with req->scale > 0, from req->theta0, with the minimiser,
 * stopping rules and errors of the fit server; req->p4, req->t and req->n are
 * not used. Runs to completion on the calling thread, one mxa_nll_grad per
 * step (a trial point outside the model's domain counts as +inf). On return
 * the context's parameters are the best point; t_submit_ns = t_start_ns = the
 * call, t_done_ns its end. Errors: MXA_EINVAL (bad scale, no free parameter,
 * no sample loaded), MXA_EDOMAIN (theta0 outside the domain), and those of
 * mxa_nll_grad. */
int32_t mxa_fit(mxa_ctx* ctx, int32_t precision, const mxa_fit_request* req, mxa_fit_result* out);

/* Create a server on `device`. precision: MXA_FP64 or MXA_FP32AMP for every
 * fit: the precision in which each fit's chain amplitudes B_k (its basis:
 * with the lineshapes fixed, the per-event part of Eq. (2)) are computed once
 * and stored; every evaluation forms A_f, Abar_f from them and the NLL and
 * gradient in FP64. shape: the 6 fixed masses and widths (K*0, rho0, a1).
 * mc_p4: host [n_mc][16] phase-space events (copied; only their Gram matrix
 * is kept). hbm_budget_bytes is the device memory of the admitted fits: the
 * server allocates it once, here, and carves it into the fits' blocks, so
 * that admitting and retiring fits never allocates or frees device memory.
 * An active fit holds its basis (two columns per chain of the kernels' chain
 * set, 16 for the fourteen-chain model) in the server's precision plus the
 * FP64 decay time, on the event count rounded up to 64: 72 bytes per event
 * for MXA_FP32AMP, 136 for MXA_FP64, with 16 columns; a fit being admitted
 * also holds its staging: the events and times as copied from the host (136
 * bytes per event; none for events handed over on the device) and the 25
 * column tier-0 record its basis is computed from. A queued fit waits until
 * its bytes fit in the budget.
 * max_slots (1..256) bounds the fits evaluated together.
 * Errors: MXA_EINVAL, MXA_EDEVICE, MXA_ENOMEM (also when the budget cannot
 * be allocated). */
int32_t mxa_server_create(const mxa_model_desc* model, int32_t device, int32_t precision,
                          const double* shape, const double* mc_p4, int64_t n_mc,
                          int64_t hbm_budget_bytes, int32_t max_slots, mxa_server** out);

/* Create a server whose fits may float the masses and widths (the lineshape
 * parameters of Sec. 3, left fixed by mxa_server_create): each fit's theta0
 * supplies them and its scale may free them. The MC sample's tier-0 cache
 * (100 bytes per event for MXA_FP32AMP, 200 for MXA_FP64, on n_mc rounded up
 * to 64) stays on the device, outside hbm_budget_bytes, and every tick reads
 * it once for all active fits: each range of MC events is evaluated for every
 * active fit at its own point (Sec. 3.1 normalisation with the lineshapes
 * recomputed), one after another on one chip partition, so that the later
 * reads of a range come from cache. Device work per tick also holds
 * max_slots x nb x 43 x 16 bytes of partial sums (nb <= 1024 MC ranges).
 * Each active fit holds its tier-0 record (25 columns in the server's
 * precision and the FP64 decay time: 108 bytes per event for MXA_FP32AMP,
 * 208 for MXA_FP64), evaluated like a context's in that precision. A
 * fit's result depends only on its own data and parameters and the MC
 * sample. Other arguments and errors as mxa_server_create (n_mc <= 2^31 -
 * 1024; MXA_EINVAL also when an MC event fails validation, and for a model
 * with a background component, a decay-time resolution or CP violation). */
int32_t mxa_server_create_streamed(const mxa_model_desc* model, int32_t device, int32_t precision,
                                   const double* mc_p4, int64_t n_mc, int64_t hbm_budget_bytes,
                                   int32_t max_slots, mxa_server** out);

/* Queue a fit; *ticket identifies it. The request's arrays are copied; the
 * server keeps the fit's record (host memory) until mxa_fit_release.
 * Errors: MXA_EINVAL (bad request), MXA_ENOMEM (cache and staging larger than
 * the whole HBM budget), MXA_EDOMAIN (theta0 outside the model's domain). */
int32_t mxa_fit_submit(mxa_server* server, const mxa_fit_request* req, uint64_t* ticket);

/* Result of a finished fit: MXA_OK and *out filled, MXA_EAGAIN while it is
 * queued or running, MXA_ENOTFOUND for an unknown ticket. */
int32_t mxa_fit_poll(mxa_server* server, uint64_t ticket, mxa_fit_result* out);

/* As mxa_fit_poll, but blocks until the fit has finished. */
int32_t mxa_fit_wait(mxa_server* server, uint64_t ticket, mxa_fit_result* out);

/* Cancel a queued or running fit (it finishes with MXA_FIT_CANCELLED). */
int32_t mxa_fit_cancel(mxa_server* server, uint64_t ticket);

/* Forget a finished fit's record; its ticket becomes unknown. Errors:
 * MXA_ENOTFOUND (unknown ticket), MXA_EAGAIN (the fit is queued or running:
 * cancel it first, or wait). */
int32_t mxa_fit_release(mxa_server* server, uint64_t ticket);

/* out[8]: ticks, evaluations, active fits, queued fits, HBM bytes in use,
 * the most HBM bytes in use and the most active fits at any time since the
 * server was created, fit records held (unreleased tickets). */
int32_t mxa_server_stats(mxa_server* server, int64_t* out);

/* Evaluate each tick by replaying a captured graph (on = 1) or by direct
 * launches (on = 0, the default: less host time per tick on MI355X). The
 * results are the same either way. */
int32_t mxa_server_set_graph(mxa_server* server, int32_t on);

/* Stop the scheduler (unfinished fits are cancelled), wake the callers
 * blocked in mxa_fit_wait (they return the cancelled result, or MXA_EDEVICE
 * for a fit that never finished), wait until every call already inside the
 * server has returned, and free everything. No server call may start once
 * mxa_server_destroy has begun. */
int32_t mxa_server_destroy(mxa_server* server);

/* Thread-local message of the last failing call ("" if none). */
const char* mxa_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* MIXAMP_H */
