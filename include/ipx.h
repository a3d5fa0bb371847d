/*
 * ipx.h -- C ABI of libipx, an FP64 unbinned maximum-likelihood engine for
 * AMD Instinct MI355X (gfx950).
 *
 * The library evaluates NLL(theta) = -sum_i w_i ln P(x_i | theta) over an
 * event sample resident in device memory, and its gradient, for three
 * probability density families.  It is the per-call work that a minimizer or
 * sampler performs once per parameter vector (Ipanema-beta, arXiv:1706.01420,
 * Example 1: the FCN handed to Minuit; Example 2: the simultaneous angular fit
 * driven through the same FCN).
 *
 * Conventions (apply to every function below):
 *   - Every function returns ipx_status (0 = IPX_OK, negative = error) and
 *     never throws or aborts.  The message of the last error on the calling
 *     thread is returned by ipx_last_error().
 *   - theta, nll and grad are caller-owned HOST memory, read/written before the
 *     call returns.  theta holds the parameters in the order listed for the
 *     model (IPX_MODEL_*).
 *   - stream is a hipStream_t cast to void*; NULL selects the context's own
 *     stream.  Calls that return a value synchronise that stream before
 *     returning.
 *   - Parameters outside the model's domain return IPX_EDOMAIN with
 *     *nll = +inf and launch nothing.  An event with P <= 0 or a non-finite
 *     contribution makes the sum non-finite: the call returns IPX_EDOMAIN
 *     with *nll = +inf (ipx_count_bad_events counts such events).
 *   - NLL is -ln L (not -2 ln L); a minimizer uses errordef 0.5.
 */
#ifndef IPX_H
#define IPX_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define IPX_API __attribute__((visibility("default")))

typedef enum {
  IPX_OK = 0,
  IPX_EINVAL = -1,    /* bad argument (null pointer, size, model, column count) */
  IPX_ENOMEM = -2,    /* device or pinned-host allocation failed, or budget exceeded */
  IPX_EDEVICE = -3,   /* a HIP runtime call failed */
  IPX_EBUSY = -4,     /* resource busy (queue full, result not ready) */
  IPX_ENOTFOUND = -5, /* unknown handle or ticket */
  IPX_ETIMEOUT = -6,  /* wait timed out */
  IPX_EDOMAIN = -7,   /* parameters outside the domain, or a non-finite likelihood */
  IPX_ECANCELED = -8  /* a served request cancelled before it reached the device */
} ipx_status;

/*
 * Models.  Columns are FP64, one contiguous array per observable, in the
 * order given; parameters are FP64 in the order given.
 *
 * IPX_MODEL_MASS (Example 1: signal peak on an exponential background)
 *   columns: m [MeV], range [5200, 5500]
 *   theta:   f, mu, sigma, lambda            (4)
 *   P(m) = f G(m)/N_G + (1-f) E(m)/N_E, G = exp(-(m-mu)^2/(2 sigma^2)),
 *   E = exp(-lambda (m - 5200)), both normalised on the range (lambda = 0
 *   handled exactly).
 *
 * IPX_MODEL_MASSTIME (mass x decay time with per-event Gaussian resolution)
 *   columns: m, t [ps] in [0.3, 15], sigma_t [ps]
 *   theta:   f, mu, sigma_m, lambda, tau_s, tau_b, s     (7)
 *   P = f [G/N_G][F(t;1/tau_s,s sigma_t)/I] + (1-f)[E/N_E][F(t;1/tau_b,s sigma_t)/I]
 *   F = e^{-t/tau} convolved with a Gaussian of width s sigma_t, I = its
 *   integral over [0.3, 15]; conditional on sigma_t.
 *
 * IPX_MODEL_ANGTIME (Example 2: B_s -> J/psi KK time-dependent angular PDF,
 *   P wave + S wave, one flavour, |lambda| = 1, C_SP = 1, delta_0 = 0)
 *   columns: cos_k, cos_l, phi [rad], t [ps], sigma_t [ps], m [MeV]
 *   theta:   fL, fperp, Fs, delta_par, delta_perp, delta_S, Gamma, DeltaGamma,
 *            Delta_m, phi_s, mu_m, sigma_m                              (12)
 *   P = [sum_k f_k(Omega) sum_j C_kj T_j(t|sigma_t)] / [sum_j D_j I_j(sigma_t)]
 *       x G(m)/N_G, T_j the resolution-convolved e^{-Gamma t} x
 *       (cosh, sinh)(DeltaGamma t/2), (cos, sin)(Delta_m t), I_j their integrals
 *       over [0.3, 15], D_j = sum_k (integral f_k dOmega) C_kj.
 *
 * IPX_MODEL_ANGTIME_TAGGED (Example 2's flavour-tagged categories)
 *   columns: the six of IPX_MODEL_ANGTIME, then qd = q (1 - 2 omega): q = +1
 *            for a B_s tag, -1 for an anti-B_s tag, omega the event's mistag
 *            probability (qd = 0: untagged)
 *   theta:   as IPX_MODEL_ANGTIME                                       (12)
 *   P as IPX_MODEL_ANGTIME with the cos and sin terms (j = 3, 4) scaled by
 *   qd in the numerator and the normalisation alike: the normalised mixture
 *   (1 - omega) P(B_s) + omega P(anti-B_s) of the two flavours' densities,
 *   the anti-B_s one having c_k and d_k of the opposite sign.
 *
 * Both angular models take two per-dataset constants
 * (ipx_dataset_set_angular): the normalisation weights xi_k (default the
 * analytic integrals of a flat angular efficiency) and the S-P interference
 * factor C_SP of the sample's KK-mass bin (default 1), which scales the
 * S-P interference rows k = 8, 9, 10.
 */
/*
 * IPX_MODEL_IPATIA (Example 1 with its Ipatia signal, normalised numerically)
 *   columns: m [MeV], range [5200, 5500]
 *   theta:   f, mu, sigma, lambda, zeta, beta, a, n, a2, n2, k        (11)
 *   P(m) = f I(m - mu) / N_I + (1 - f) e^{-k (m - 5200)} / N_E, I the Ipatia
 *   shape (Santos, Dupertuis, NIM A 764 (2014) 150): a generalised-hyperbolic
 *   core q^{lambda - 1/2} K_{lambda - 1/2}(zeta q) e^{beta d}, d = m - mu,
 *   q = sqrt(1 + d^2 / (A^2 sigma^2)), A^2 = zeta K_lambda(zeta) /
 *   K_{lambda + 1}(zeta) (zeta = 0: q^{2 lambda - 1} e^{beta d} with
 *   A^2 = -2 (lambda + 1), lambda < -1), and power-law tails A (B -+ d)^{-n}
 *   below -a sigma and above a2 sigma matching the core's value and slope.
 *   N_I = dm sum_g I(m_g - mu) over 16384 midpoints m_g of the range (step
 *   dm), computed on the device at every call; N_E analytic.  Evaluated by
 *   nll_eval and ipx_event_logp only (no analytic gradient, no plans, no
 *   served requests: IPX_EINVAL).  Outside the domain (f in [0, 1],
 *   sigma, a, n, a2, n2 > 0, zeta >= 0, and tails that fall away from the
 *   core at both junctions) IPX_EDOMAIN.
 */
typedef enum {
  IPX_MODEL_MASS = 1,
  IPX_MODEL_MASSTIME = 2,
  IPX_MODEL_ANGTIME = 3,
  IPX_MODEL_ANGTIME_TAGGED = 4,
  IPX_MODEL_IPATIA = 5
} ipx_model;

/* dataset creation flags */
#define IPX_COPY_HOST 0u     /* cols/w are host pointers; data are copied to the device */
#define IPX_COPY_DEVICE 1u   /* cols/w are device pointers; data are copied device-to-device */
#define IPX_BORROW_DEVICE 2u /* cols/w are device pointers used in place; the caller keeps them alive */
#define IPX_KEEP_ORDER 4u    /* or-ed with a COPY flag: store events in the given order */
#define IPX_NO_WEIGHTS 8u    /* toy_generate: no weight column (unit weights) */

typedef struct ipx_ctx ipx_ctx;
typedef struct ipx_dataset ipx_dataset;

/* Create a context on HIP device `device` (owns a stream and small buffers). */
IPX_API ipx_status ipx_create(int device, ipx_ctx **out);
/* Destroy a context; datasets created on it must be destroyed first. */
IPX_API void ipx_destroy(ipx_ctx *ctx);
/* Message of the last failed call on this thread ("" if none). */
IPX_API const char *ipx_last_error(void);
/* Number of parameters / columns of a model, or -1 for an unknown model. */
IPX_API int ipx_model_nparams(int model);
IPX_API int ipx_model_ncols(int model);

/*
 * Create a dataset of n >= 0 events for `model`.
 *   cols:  ncols (= ipx_model_ncols(model)) pointers to n doubles each, in the
 *          model's column order (host or device memory per `flags`).
 *   w:     optional per-event weights (n doubles, same memory kind), NULL for 1.
 * With IPX_COPY_*, the library owns the device copy (one allocation, columns
 * padded to 256-byte boundaries); the models with a decay time store it in
 * resolution-band order (unless IPX_KEEP_ORDER): a stable sort by the key
 * (b << 58) | ((2^63 - 1 - bits(sigma_t)) >> 6), b = min(floor(2 t / sigma_t),
 * 20) (0 when not positive), i.e. by band, then by decreasing sigma_t, so that
 * the events of a wave need the same resolution corrections.  The NLL is a sum over events, so the order changes only its
 * rounding.  The dataset also holds the scratch for its
 * reduction partials, so calls on different datasets may run concurrently on
 * different streams; calls on one dataset must not overlap.
 */
IPX_API ipx_status ipx_dataset_create(ipx_ctx *ctx, int model, int64_t n, const double *const *cols,
                              int ncols, const double *w, unsigned flags, ipx_dataset **out);
IPX_API ipx_status ipx_dataset_destroy(ipx_ctx *ctx, ipx_dataset *ds);
/* Device bytes held by the dataset (columns, weights, scratch). */
IPX_API size_t ipx_dataset_bytes(const ipx_dataset *ds);
IPX_API int64_t ipx_dataset_size(const ipx_dataset *ds);
IPX_API int ipx_dataset_model(const ipx_dataset *ds);
/* Device pointer of column `col` (0..ncols-1) or of the weights (col = ncols,
 * NULL when unweighted). */
IPX_API ipx_status ipx_dataset_column(const ipx_dataset *ds, int col, const double **dev_ptr);
/* Copy events [offset, offset + count) of column `col` (or of the weights,
 * col = ncols) to host memory `host` (count doubles, caller-owned).  Events
 * are in storage order (resolution-band order for the time models unless
 * IPX_KEEP_ORDER).  Synchronous. */
IPX_API ipx_status ipx_dataset_read(ipx_ctx *ctx, const ipx_dataset *ds, int col, int64_t offset, int64_t count,
                                    double *host);

/*
 * Per-dataset constants of the angular models (Example 2: each category has
 * its own normalisation; a non-flat angular efficiency eps enters through the
 * weights xi_k = integral eps(Omega) f_k(Omega) dOmega, obtained by the
 * caller from simulated events or quadrature).
 *   xi:   10 doubles (host memory), or NULL for the flat-efficiency values
 *         (32 pi / 9 for k = 1, 2, 3, 7; 0 otherwise).
 *   c_sp: the S-P interference factor of the sample's KK-mass bin (1 = none
 *         of the interference is lost).
 * Applies to every later evaluation of the dataset (plain, batched, served,
 * simultaneous); requests already submitted keep the values they were
 * hoisted with.  IPX_EINVAL for a dataset of another model or non-finite
 * values.
 */
IPX_API ipx_status ipx_dataset_set_angular(ipx_ctx *ctx, ipx_dataset *ds, const double *xi, double c_sp);

/*
 * NLL of the dataset at theta (np = ipx_model_nparams(model) doubles).
 * The per-event terms are summed in a fixed order that depends only on the
 * dataset size: per-lane sequential sums over fixed event strides, a fixed
 * wave/workgroup tree per tile of events, then the tiles in index order.  The
 * result is therefore bitwise reproducible for the same dataset and theta,
 * whatever the launch size or concurrent traffic.
 */
IPX_API ipx_status nll_eval(ipx_ctx *ctx, const ipx_dataset *ds, const double *theta, int np, double *nll,
                    void *stream);

/*
 * NLL and its gradient dNLL/dtheta (np doubles written to grad), from a
 * hand-written adjoint kernel: each event accumulates the derivatives of its
 * term with respect to the per-call hoisted quantities (coefficients,
 * normalisations, decay constants); the host applies the Jacobian of the
 * hoisting.  The NLL value is bitwise equal to nll_eval's.
 * The gradient's domain is open where the model takes a square root of a
 * parameter: in IPX_MODEL_ANGTIME the interference coefficients are linear in
 * the amplitude moduli sqrt(|A_i|^2), whose slope is infinite where a squared
 * modulus vanishes, so nll_grad (and the gradient forms of nll_eval_batch
 * and served requests) require fL > 0, fperp > 0, fL + fperp < 1 and
 * 0 < Fs < 1; on that boundary they return IPX_EDOMAIN with *nll = +inf and
 * NaN gradients (nll_eval accepts it).
 */
IPX_API ipx_status nll_grad(ipx_ctx *ctx, const ipx_dataset *ds, const double *theta, int np, double *nll,
                    double *grad, void *stream);

/*
 * Allocation-free evaluation, for callers that cannot allocate device memory
 * (code under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc): nll_eval (grad == NULL) or nll_grad (grad != NULL) over
 * caller-owned device columns, with every per-call buffer (segment record,
 * hoisted constants, tile table, tile partials, reduced totals) in a fixed
 * device array of the library (about 6.9 MB per device, held from the first
 * ipx_create on that device until the process ends).  The call allocates
 * nothing, on the device or in pinned host memory.
 *   model, n, cols, ncols, w: as ipx_dataset_create with IPX_BORROW_DEVICE
 *          (device pointers, events in the given order, w NULL for unit
 *          weights); the results are bitwise those of nll_eval / nll_grad
 *          on such a dataset.
 *   n:     0 <= n <= 16,777,216 (2^24); larger n returns IPX_EINVAL.
 *   theta, np, nll, grad, stream: as nll_eval / nll_grad (synchronous).
 * All calls on one device share the array, which keeps the last call's
 * contents (every value a call reads was written earlier by the same call).
 * Within a process the library serialises the calls on a device with a lock;
 * callers that bypass it (another copy of the library in the same process)
 * must not overlap their calls on one device.
 * IPX_EINVAL for NULL arguments, a wrong model, column count or np, or n out
 * of range; IPX_EDOMAIN as nll_eval / nll_grad; IPX_EDEVICE for HIP errors.
 */
IPX_API ipx_status nll_eval_noalloc(ipx_ctx *ctx, int model, int64_t n, const double *const *cols, int ncols,
                                    const double *w, const double *theta, int np, double *nll, double *grad,
                                    void *stream);

/*
 * Batched evaluation (many datasets of one model, each at its own theta, in
 * one fused launch; the paper's pseudo-experiment studies fit hundreds of toys
 * with the same likelihood).  A plan fixes the list of datasets (all of the
 * same model, each appearing once) and owns the staging buffers; its first
 * evaluation in each mode (NLL only / NLL + gradient) is captured into a HIP
 * graph that later calls replay.  Each dataset keeps its canonical tiles and
 * partial buffers, so its result is bitwise the same as nll_eval/nll_grad on
 * the dataset alone, whatever else is in the batch.
 *   theta:  nb x np doubles (row j for dataset j), host memory.
 *   active: nb flags (nullable = all active); inactive entries are skipped and
 *           their outputs left untouched.
 *   nll:    nb doubles; grad: nb x np doubles or NULL for NLL only.
 * Entries outside the domain or with a non-finite likelihood get +inf (and
 * NaN gradients); the call then returns IPX_EDOMAIN after filling every other
 * entry.  Plans must not be used concurrently with each other or with plain
 * calls on the same datasets.  A dataset referenced by a plan cannot be
 * destroyed (IPX_EBUSY) until the plan is.
 */
typedef struct ipx_plan ipx_plan;
IPX_API ipx_status ipx_plan_create(ipx_ctx *ctx, int nb, ipx_dataset *const *ds, ipx_plan **out);
IPX_API void ipx_plan_destroy(ipx_plan *plan);
IPX_API ipx_status nll_eval_batch(ipx_ctx *ctx, ipx_plan *plan, const double *theta, const unsigned char *active,
                                  double *nll, double *grad, void *stream);

/*
 * Simultaneous fit over categories (Example 2: the angular PDF fitted in bins
 * of the KK mass and per flavour at once, each category normalised on its
 * own, the P-wave and mixing parameters shared, the S-wave fraction and phase
 * free per bin).  A simultaneous set holds ncat datasets of one angular model
 * (IPX_MODEL_ANGTIME or IPX_MODEL_ANGTIME_TAGGED), dataset c in KK-mass bin
 * bin[c] (0 <= bin[c] < nbins; the bin's C_SP is the dataset's, see
 * ipx_dataset_set_angular).  Its parameter vector (np = 10 + 2 nbins) is
 *   fL, fperp, delta_par, delta_perp, Gamma, DeltaGamma, Delta_m, phi_s,
 *   mu_m, sigma_m, then Fs_b, delta_S_b for b = 0 .. nbins - 1,
 * category c being evaluated at (fL, fperp, Fs_bin, delta_par, delta_perp,
 * delta_S_bin, Gamma, DeltaGamma, Delta_m, phi_s, mu_m, sigma_m).
 * nll_sim returns the sum of the categories' NLLs (added in category order)
 * and, if grad is not NULL, its gradient (np doubles); all categories run in
 * one batched launch (a plan over the datasets, created with the set).  A
 * category outside its domain, or with a non-finite likelihood, makes the
 * result +inf (NaN gradient) and the call return IPX_EDOMAIN.  The datasets
 * cannot be destroyed before the set (IPX_EBUSY).
 */
typedef struct ipx_sim ipx_sim;
IPX_API ipx_status ipx_sim_create(ipx_ctx *ctx, int ncat, ipx_dataset *const *ds, const int *bin, int nbins,
                                  ipx_sim **out);
IPX_API void ipx_sim_destroy(ipx_sim *sim);
IPX_API int ipx_sim_nparams(const ipx_sim *sim);
IPX_API ipx_status nll_sim(ipx_ctx *ctx, ipx_sim *sim, const double *theta, int np, double *nll, double *grad,
                           void *stream);

/*
 * Launch schedule of a plan's per-event kernel: how its tiles are handed to
 * workgroups.  Every tile writes its own partials and the reduction sums them
 * in tile order, so results are bitwise the same under every schedule; only
 * the time changes.
 *   workgroups: 0 = one workgroup per tile (the hardware dispatcher balances
 *               them); > 0 = that many workgroups, each striding over the
 *               tile table.
 *   order:      0 = tiles segment by segment; 1 = interleaved by local tile
 *               index (the first tile of every segment, then the second, ...).
 *   graph:      1 = each evaluation replays a HIP graph of its kernels
 *               (captured on first use); 0 = the kernels are launched directly.
 *   variant:    the per-event kernel's build (register budget and so waves per
 *               SIMD; see ipx_schedule.variant).
 * New plans start with {0, 0, 1, 0}.  ipx_plan_set_schedule synchronises the
 * context's stream and drops the plan's captured graphs (recaptured on the next
 * call).  IPX_EINVAL for negative workgroups, an unknown order, graph not 0/1
 * or a variant the model does not have.
 *
 * ipx_plan_autotune times the candidate schedules (one workgroup per tile,
 * 8 and 16 workgroups per compute unit; both orders when the plan has several
 * segments; graph replay and direct launches; both kernel variants of the
 * angular model) at theta (nb x np host doubles,
 * as for nll_eval_batch; grad != 0 times the gradient form) in `reps` rounds:
 * in each round every candidate is set and evaluated twice, the second call
 * timed.  It keeps the candidate with the smallest median wall time per call
 * on the plan and returns it in *best (*best_us: that median, may be NULL).
 * table/ntable (optional): on entry *ntable is the capacity of table, on return
 * the number of candidates written, each with its median time.
 */
typedef struct {
  int workgroups;
  int order;
  int graph;
  int variant;   /* per-event kernel build: 0 = default register budget; 1 (angular
                    model only) = the alternative: the gradient kernel at 3 waves
                    per SIMD (no register spills), the NLL-only kernel at 6 (at
                    most 80 registers); other models accept 0 only */
} ipx_schedule;
typedef struct {
  ipx_schedule schedule;
  double us;
} ipx_tune_entry;
IPX_API ipx_status ipx_plan_set_schedule(ipx_plan *plan, const ipx_schedule *schedule);
IPX_API ipx_status ipx_plan_get_schedule(const ipx_plan *plan, ipx_schedule *out);
IPX_API ipx_status ipx_plan_autotune(ipx_ctx *ctx, ipx_plan *plan, const double *theta, int grad, int reps,
                                     ipx_schedule *best, double *best_us, ipx_tune_entry *table, int *ntable);

/*
 * Served likelihood: a persistent device loop that evaluates requests from
 * many concurrent clients (minimizers, MCMC chains) over resident datasets
 * (the paper's samplers and fitters each call the likelihood once per
 * parameter vector).  Requests are admitted into device slots as slots and
 * scratch memory (the request's tile partials: kAccMax doubles per 1024-event
 * tile at most) free up, so requests arriving while others run join
 * the same launch; each request's result is bitwise the same as nll_eval /
 * nll_grad on its dataset alone.  The device loop ends by itself after an
 * idle period and is relaunched when work arrives.
 *   ipx_submit is thread safe and non-blocking (IPX_EBUSY if max_pending
 *   requests are already waiting; IPX_ENOMEM if the request alone exceeds the
 *   scratch budget).  Results are taken once, with ipx_poll (IPX_EBUSY while
 *   running) or ipx_wait (IPX_ETIMEOUT after timeout_ns; < 0 waits forever).
 *   ipx_cancel withdraws a request that is still waiting for a slot: its
 *   result becomes available at once with status IPX_ECANCELED (nll = +inf)
 *   and must still be taken with ipx_poll / ipx_wait.  A request already on
 *   the device, or finished, cannot be cancelled (IPX_EBUSY; it completes
 *   normally); an unknown ticket gives IPX_ENOTFOUND.
 *   ipx_server_drain blocks until every request submitted before it has
 *   finished (submissions during the drain return IPX_EBUSY); their results
 *   stay available to ipx_poll / ipx_wait, and the server accepts requests
 *   again afterwards.
 *   ipx_server_stop drains pending and in-flight requests, stops the device
 *   loop, wakes the clients blocked in ipx_wait (each returns its result, or
 *   IPX_ENOTFOUND if its request could not finish), waits until every call
 *   already inside the server has returned, and frees the server; results not
 *   yet taken are discarded.  No call on the server may start once
 *   ipx_server_stop has been called.  Datasets must outlive the requests on
 *   them.
 */
typedef struct ipx_server ipx_server;
typedef struct {
  int slots;               /* concurrent requests on the device (<= 64; 0 = 32) */
  size_t scratch_bytes;    /* scratch budget for admitted requests (0 = 2 GiB) */
  int workgroups;          /* persistent workgroups, one of which polls the host
                              (>= 2; 0 = 3 per compute unit) */
  int idle_iterations;     /* consecutive polls that find no new request and no
                              claimable work before the device loop exits
                              (0 = 20000, a few tens of ms); it is relaunched
                              when work arrives */
  int max_pending;         /* waiting requests accepted (0 = unlimited) */
  int policy;              /* how workgroups pick among admitted requests:
                              0 = each workgroup from its own starting slot
                              (admitted requests share the workgroups; the
                              lowest latency measured),
                              1 = the oldest admitted request first (its tiles
                              are all claimed before a younger one's),
                              2 = the request with the fewest unclaimed
                              tiles first */
} ipx_server_cfg;
typedef struct {
  const ipx_dataset *ds;
  const double *theta;     /* np doubles, copied at submission */
  int np;
  int want_grad;
} ipx_request;
typedef struct {
  int status;              /* IPX_OK, IPX_EDOMAIN, ... */
  int np;
  double nll;
  double grad[12];         /* np entries when the gradient was requested */
  double latency_us;       /* submission to completion */
} ipx_result;
IPX_API ipx_status ipx_server_start(ipx_ctx *ctx, const ipx_server_cfg *cfg, ipx_server **out);
IPX_API ipx_status ipx_submit(ipx_server *srv, const ipx_request *req, uint64_t *ticket);
IPX_API ipx_status ipx_poll(ipx_server *srv, uint64_t ticket, ipx_result *out);
IPX_API ipx_status ipx_wait(ipx_server *srv, uint64_t ticket, int64_t timeout_ns, ipx_result *out);
IPX_API ipx_status ipx_cancel(ipx_server *srv, uint64_t ticket);
IPX_API ipx_status ipx_server_drain(ipx_server *srv);
IPX_API ipx_status ipx_server_stop(ipx_server *srv);
/* Host-side counters of a running server (monitoring). */
typedef struct {
  uint64_t published;      /* requests handed to the device */
  uint64_t completed;      /* requests the device finished */
  uint64_t launches;       /* launches of the device loop */
  uint64_t pending;        /* waiting for a slot or scratch now */
  uint64_t in_flight;      /* in device slots now */
  uint64_t cancelled;      /* requests withdrawn by ipx_cancel */
} ipx_server_stats;
IPX_API ipx_status ipx_server_stats_read(ipx_server *srv, ipx_server_stats *out);

/*
 * Unbinned toy generation by accept-reject (Example 5 of the paper: toys
 * generated on the device by accept-reject from a counter-based stream).
 * Generates n events of `model` at theta_gen into a new dataset (*out, owned
 * by the caller, destroyed with ipx_dataset_destroy).
 *   Stream: Philox4x64-10, key (seed, toy_id), counter (c, b, model, 0) for
 *   candidate c and block b (1, 2, 3 blocks per candidate for models 1, 2, 3);
 *   uniforms ((word >> 12) + 0.5) 2^-52.  Candidate c is accepted on its own
 *   words; the output holds the first n accepted candidates (increasing c),
 *   in resolution-band order for models 2 and 3 unless flags has IPX_KEEP_ORDER.
 *   Model 3 also draws weights 0.8 + 0.2 u (the workload's efficiency weights)
 *   unless flags has IPX_NO_WEIGHTS.
 *   Each model's recipe (proposals, bounds, acceptance ratios) is documented
 *   in the library source; conditional on sigma_t the accepted events follow
 *   the model's PDF exactly.
 * stats (nullable): n_candidates = index of the n-th accepted candidate + 1;
 * n_violations = candidates whose acceptance ratio exceeded the bound (0 for
 * an exact sample).
 */
typedef struct {
  uint64_t n_candidates;
  uint64_t n_violations;
} ipx_toy_stats;
IPX_API ipx_status toy_generate(ipx_ctx *ctx, int model, const double *theta_gen, int np, uint64_t seed,
                                uint64_t toy_id, int64_t n, unsigned flags, ipx_dataset **out,
                                ipx_toy_stats *stats);
/*
 * Many toys at once (Example 5 of the paper: hundreds of pseudo-experiments):
 * out[j] (ntoys caller-owned datasets) holds exactly what toy_generate with
 * toy_id = toy_ids[j] and n = n[j] gives, with the same flags; each round
 * generates the candidates of every toy still short of events in one launch.
 * stats (nullable) has ntoys entries; n_violations counts the candidates
 * evaluated, which may extend past the last accepted one differently from
 * toy_generate.  On error no dataset is returned (out[j] = NULL).
 */
IPX_API ipx_status toy_generate_batch(ipx_ctx *ctx, int model, const double *theta_gen, int np, uint64_t seed,
                                      int ntoys, const uint64_t *toy_ids, const int64_t *n, unsigned flags,
                                      ipx_dataset **out, ipx_toy_stats *stats);

/*
 * Bad events: the number of events of ds whose contribution w_i ln P_i at
 * theta is not finite (P_i <= 0, or a non-finite column value or weight), the
 * events that make nll_eval / nll_grad return IPX_EDOMAIN with a non-finite
 * likelihood.  A separate diagnostic pass over the dataset (the evaluation
 * kernels only form the sum); synchronous on the context's stream; allocates
 * and frees its own device scratch.  *count receives the number (host memory).
 * IPX_EINVAL for NULL arguments or a wrong np, IPX_EDOMAIN for parameters
 * outside the model's domain (no launch), IPX_EDEVICE for HIP errors.
 */
IPX_API ipx_status ipx_count_bad_events(ipx_ctx *ctx, const ipx_dataset *ds, const double *theta, int np,
                                        int64_t *count);

/*
 * Per-event terms, for inspection (the paper's advice on debugging GPU code:
 * write intermediate per-event values to a device array and look at them):
 * out[i] = w_i ln P_i at theta for event i of ds in storage order (the order
 * ipx_dataset_read returns), i.e. the terms whose sum is -nll_eval(...); the
 * angular model's term includes its mass factor, ln(G(m)/N_G).
 *   out: DEVICE memory of ipx_dataset_size(ds) doubles, caller-owned (may be
 *        NULL when the dataset is empty).
 * Enqueued on `stream` (NULL: the context's stream) and synchronised before
 * returning.  IPX_EINVAL for NULL arguments or a wrong np; IPX_EDOMAIN for
 * parameters outside the model's domain (nothing written); IPX_EDEVICE for
 * HIP errors.
 */
IPX_API ipx_status ipx_event_logp(ipx_ctx *ctx, const ipx_dataset *ds, const double *theta, int np, double *out,
                                  void *stream);

/*
 * Binned path (Examples 3-5 of the paper on the binned side: a binned
 * maximum-likelihood fit of a mass spectrum; CL_s from binned pseudo-data,
 * with a signal shape filled per bin and convolved with a Gaussian on top of
 * an exponential background; binned toys as a Poisson count per bin).
 *
 * A histogram has nbins equal bins on [lo, hi) (width dx, centres
 * x_b = lo + (b + 1/2) dx), a signal template and observed counts.  The
 * template is a Gaussian core exp(-(x_b - mu)^2 / (2 sigma_core^2)) smeared
 * by a Gaussian of width sigma_smear (ipx_smear) and normalised to unit sum,
 * all computed on the device at creation.  The background template is
 * e_b = exp(-k (x_b - x_0)) / Z, Z = sum_b exp(-k b dx), and the expected
 * counts are nu_b = ns s_b + nb e_b.  Parameters theta = (ns, nb, k).
 *
 * ipx_smear: S_b = sum_j h_j g(x_b - x_j) dx over n bins of width dx, g the
 *   unit Gaussian density of width sigma (the rectangle rule of the
 *   convolution integral, no wrap-around); h and out are DEVICE arrays of n
 *   doubles (caller-owned, not overlapping); synchronous on `stream`.  Its
 *   work space ((2n - 1) + c n doubles, c <= 2048 input chunks, c n held to
 *   2^23 where n allows) is kept by the context, grown when a call needs
 *   more and freed by ipx_destroy; calls on one context take turns.
 * ipx_hist_create: counts (host, nullable = all zero) are non-negative
 *   integers stored as doubles; 1 <= nbins <= 2^24.
 * ipx_hist_read: which = 0 copies the signal template, 1 the counts, to host
 *   memory (nbins doubles).
 * nll_binned: NLL = sum_b [nu_b - n_b ln nu_b] (the constant sum_b ln n_b!
 *   dropped) and, if grad is not NULL, its gradient in (ns, nb, k); np = 3;
 *   IPX_EDOMAIN (+inf) for ns < 0, nb < 0, non-finite values, or a
 *   non-positive expected count where counts were seen.
 * ipx_binned_toy: the counts of one toy (host, nbins doubles) of hypothesis
 *   hyp (0: background only, nu_b = nb e_b; 1: signal + background): n_b is
 *   the smallest k with u <= F(k), F the Poisson CDF of nu_b summed from
 *   k = 0 (p_0 = e^{-nu}, p_k = p_{k-1} nu / k), u from Philox4x64-10 with
 *   key (seed, 0xB1), counter (b / 4, toy, hyp, 0), word b % 4, as
 *   ((word >> 12) + 0.5) 2^-52; at most floor(nu + 30 sqrt(nu + 1) + 30).
 *   Every expected count must be below 700 (e^{-nu} must not underflow),
 *   else IPX_EDOMAIN (also for cls_toys).
 * cls_toys: q = 2 sum_b [s_b - n_b ln(1 + s_b / b_b)] (s_b = ns S_b,
 *   b_b = nb e_b) for the observed counts (q_obs) and for ntoys toys of each
 *   hypothesis (toy ids 0 .. ntoys - 1, seed as above); n_b / n_sb = the
 *   toys with q >= q_obs, CL_b = n_b / ntoys, CL_s+b = n_sb / ntoys,
 *   CL_s = CL_s+b / CL_b.  q_toys (host, nullable): 2 ntoys doubles, the
 *   background-only toys' q then the signal + background toys'.  nb must be
 *   positive; 1 <= ntoys <= 2^24.  The toy kernel is timed by
 *   ipx_timing_enable / ipx_timing_read like the evaluation kernels.
 */
typedef struct ipx_hist ipx_hist;
typedef struct {
  double cl_sb;
  double cl_b;
  double cl_s;
  double q_obs;
  int64_t n_sb;
  int64_t n_b;
} ipx_cls_result;
IPX_API ipx_status ipx_smear(ipx_ctx *ctx, int n, double dx, double sigma, const double *h, double *out,
                             void *stream);
IPX_API ipx_status ipx_hist_create(ipx_ctx *ctx, int nbins, double lo, double hi, double mu, double sigma_core,
                                   double sigma_smear, const double *counts, ipx_hist **out);
IPX_API ipx_status ipx_hist_destroy(ipx_ctx *ctx, ipx_hist *hist);
IPX_API int ipx_hist_nbins(const ipx_hist *hist);
IPX_API ipx_status ipx_hist_read(ipx_ctx *ctx, const ipx_hist *hist, int which, double *host);
IPX_API ipx_status ipx_hist_set_counts(ipx_ctx *ctx, ipx_hist *hist, const double *counts);
IPX_API ipx_status nll_binned(ipx_ctx *ctx, const ipx_hist *hist, const double *theta, int np, double *nll,
                              double *grad, void *stream);
IPX_API ipx_status ipx_binned_toy(ipx_ctx *ctx, const ipx_hist *hist, const double *theta, uint64_t seed, int hyp,
                                  uint64_t toy, double *counts);
IPX_API ipx_status cls_toys(ipx_ctx *ctx, ipx_hist *hist, const double *theta, uint64_t seed, int ntoys,
                            ipx_cls_result *result, double *q_toys);

/*
 * Timing of the dominant kernel of nll_eval/nll_grad, measured with HIP events
 * recorded on the stream the kernel is launched on.  While enabled, each call
 * records a start/stop event pair around its per-event kernel; ipx_timing_read
 * returns the summed kernel milliseconds and the number of launches since the
 * last reset (it synchronises the recorded events).
 */
IPX_API ipx_status ipx_timing_enable(ipx_ctx *ctx, int enable);
IPX_API ipx_status ipx_timing_read(ipx_ctx *ctx, double *total_ms, int64_t *launches, int reset);

/*
 * The device's attainable FP64 rate, for reading a kernel's fraction of peak:
 * every lane of 8 workgroups per compute unit runs eight independent FP64
 * fused multiply-add chains (2 FLOP each) for 2 x 10^5 iterations; the best of
 * three launches gives *tflops, and the median over the workgroups of their
 * shader-clock cycles per wall-clock second during that launch gives
 * *clock_ghz.  Synchronous on the context's stream; allocates and frees its
 * own device buffers (~4 MB).  IPX_EINVAL for NULL arguments, IPX_EDEVICE for
 * HIP errors.
 */
IPX_API ipx_status ipx_fp64_peak_probe(ipx_ctx *ctx, double *tflops, double *clock_ghz);

/*
 * Self-check of the device elementary functions that the event kernels inline
 * (exp, ln, sin/cos, erfcx and the Faddeeva function w of the resolution
 * convolution), evaluated element by element on the context's device.
 *   fn = IPX_FN_EXP      y = e^x
 *        IPX_FN_LOG      y = ln x
 *        IPX_FN_SINCOS   y = sin x, y2 = cos x
 *        IPX_FN_ERFCX    y = e^{x^2} erfc(x), x >= 0
 *        IPX_FN_FADDEEVA y + i y2 = w(x + i x2), x2 >= 0 (upper half plane)
 * x, x2, y, y2: host arrays of n doubles (x2 read only for IPX_FN_FADDEEVA,
 * y2 written only for IPX_FN_SINCOS and IPX_FN_FADDEEVA; the others may be
 * NULL), owned by the caller; 0 <= n <= 2^28.  Synchronous; allocates and
 * frees its own device buffers.  IPX_EINVAL for an unknown fn, n out of range
 * or a missing buffer; IPX_EDEVICE for HIP errors.
 */
enum {
  IPX_FN_EXP = 0,
  IPX_FN_LOG = 1,
  IPX_FN_SINCOS = 2,
  IPX_FN_ERFCX = 3,
  IPX_FN_FADDEEVA = 4
};
IPX_API ipx_status ipx_math_eval(ipx_ctx *ctx, int fn, int64_t n, const double *x, const double *x2, double *y,
                                 double *y2);

#ifdef __cplusplus
}
#endif

#endif /* IPX_H */
