/*
 * nusht: nonuniform spherical harmonic transforms (spin 0 and spin s) on one AMD Instinct
 * MI355X (gfx950).
 *
 * Method: arXiv:2406.14542 (cuNUSHT), Sec. II.B.  The type-2 transform (synthesis, Eq. 3)
 * is factored as Y = N F D S (Eq. 5): S is an iso-latitude Legendre synthesis onto an
 * equi-spaced Clenshaw-Curtis ring grid, D doubles the map over the poles onto a torus
 * (Fig. 1), F is a 2D FFT and N a type-2 nonuniform FFT to the points.  The type-1
 * transform (adjoint, Eq. 2) is Y^H = S^H D^H F^H N^H (Eq. 6).  N uses the
 * exponential-of-semicircle (ES) kernel; plans are built once and reused (Sec. III).
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 * - Device pointers.  Every array argument of an execution call is a device pointer on the
 *   device that was current when the plan was created (for example a torch tensor's
 *   data_ptr()).  Nothing is copied to or from the host inside an execution call.
 * - Coefficients: complex128, interleaved (re, im), shape [nmaps][nalm], m-major triangle
 *   index(l, m) = m (2 lmax + 1 - m) / 2 + l for 0 <= m <= mmax, m <= l <= lmax.  Only m >= 0
 *   is stored: the map is real, so a_{l,-m} = (-1)^m conj(a_lm) (Eq. 3 with a real field).
 *   The imaginary part of a_l0 is ignored on input and written as 0 on output.
 * - Maps: float64, shape [nmaps][npts], in the caller's point order.
 * - Inner product on coefficients under which synthesis and adjoint are exact adjoints:
 *   <a, b>_m = sum_l [Re(a_l0* b_l0) + 2 sum_{m>0} Re(a_lm* b_lm)].
 * - Streams.  `stream` is a hipStream_t (0 = the null stream).  Execution calls only enqueue
 *   work and return; the caller keeps the buffers alive until the stream has finished.
 *   nusht_plan* and nusht_solve synchronise.  A plan runs on one stream at a time.
 * - Precision.  `dtype` selects the internal precision only; user arrays are always FP64.
 *   NUSHT_F64: everything in FP64.  NUSHT_MIXED (eps >= 1e-6; 1e-5 below sigma = 2):
 *   Legendre step, ring FFTs and point coordinates in FP64; torus, 2D FFTs, deconvolution,
 *   spreading and interpolation in FP32, with each point's grid offset formed in FP64 before
 *   the cast (Sec. IV: an FP32 nuFFT with FP32 coordinates cannot get below about 1e-4).
 * - Errors.  Every call returns a status code; nothing is thrown across the ABI.  On error
 *   no output is written by a call that fails validation on the host.
 */
#ifndef NUSHT_H
#define NUSHT_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct nusht_plan_s* nusht_plan_t;

enum { NUSHT_F64 = 0, NUSHT_MIXED = 1 };

enum {
    NUSHT_OK = 0,
    NUSHT_EINVAL = -1,     /* bad argument (host check) or bad point (device check in plan) */
    NUSHT_ENOMEM = -2,     /* device allocation failed */
    NUSHT_EDEVICE = -3,    /* HIP or rocFFT call failed */
    NUSHT_ENOCONV = -4,    /* nusht_solve: true residual above tol; iterate, residual written */
    NUSHT_EPRECISION = -5  /* NUSHT_MIXED requested below its floor: eps < 1e-6 at sigma >= 2,
                              eps < 1e-5 at sigma < 2 */
};

/* How the torus spectrum is produced from the Legendre output.
   NUSHT_DFS_PAPER: S includes a phi-FFT per ring, D doubles the (theta, phi) ring map and F
     is a full 2D FFT of the torus, exactly the composition of Eq. (5)/(6).
   NUSHT_DFS_FUSED: the phi-FFT inside S and the phi half of F cancel (Sec. III, last
     paragraphs): the doubling is applied per m in (theta, m) space and only a 1D FFT over
     the doubled theta axis remains.  Same result up to rounding. */
enum { NUSHT_DFS_FUSED = 0, NUSHT_DFS_PAPER = 1 };

typedef struct {
    double sigma;        /* fine-grid upsampling factor; 0 -> 2.0 */
    int width;           /* ES kernel width w in grid cells; 0 -> from eps and sigma */
    double beta_per_w;   /* ES shape beta = beta_per_w * w; 0 -> 2.30 at sigma = 2, else
                            0.97 pi (1 - 1/(2 sigma)) */
    int dfs_mode;        /* NUSHT_DFS_FUSED (default) or NUSHT_DFS_PAPER */
    int timing;          /* nonzero: record one hipEvent pair per stage (nusht_stage_times) */
    int deterministic;   /* nonzero: the adjoint adds in a fixed order, so repeated calls give
                            identical bits (the Legendre adjoint then writes per-pair-chunk
                            partial sums, nmaps * nalm * 16 bytes per 256 ring pairs, and adds
                            them in order; spreading is fixed-order in every plan) */
    int kernel_eval;     /* NUSHT_KERNEL_POLY (default): interpolation and spreading form the ES
                            taps from per-tap polynomials of degree w fitted at plan time (used
                            when the fit deviates from the kernel by at most eps / 20);
                            NUSHT_KERNEL_EXACT: from sqrt and exp at every tap */
    int reserved[4];     /* must be zero */
} nusht_plan_opts;

enum { NUSHT_KERNEL_POLY = 0, NUSHT_KERNEL_EXACT = 1 };

/* Sizes a plan uses; filled by nusht_geometry_for and nusht_plan_info. */
typedef struct {
    int lmax, mmax;
    int nrings;          /* N_r: CC rings theta_j = j pi / (N_r - 1), N_r >= lmax + 2 */
    int ntorus;          /* N_t = 2 (N_r - 1): rows of the doubled map */
    int nphi;            /* N_phi >= 2 mmax + 2, even: samples per ring */
    int n1, n2;          /* fine grid (theta, phi), >= sigma (2 lmax + 1), sigma (2 mmax + 1) */
    int width;           /* ES width w */
    double beta;         /* ES shape beta */
    double sigma;
    int tile;            /* side of the square point-binning tiles on the fine grid */
    int dtype;
    int dfs_mode;
    int64_t npts;
    int64_t nalm;
    int64_t ntiles_used; /* tiles holding at least one point (plan only; 0 from nusht_geometry_for) */
    int kernel_eval;     /* taps the plan's point kernels use: NUSHT_KERNEL_POLY or _EXACT (plan only) */
    double kernel_poly_dev; /* largest deviation of the tap polynomials from the kernel (plan only) */
} nusht_geometry;

/* Number of stored coefficients for (lmax, mmax); -1 if the arguments are invalid. */
int64_t nusht_nalm(int lmax, int mmax);

/* Sizes that nusht_plan_ex would choose (host only, touches no device).
   Returns NUSHT_EINVAL / NUSHT_EPRECISION like nusht_plan_ex. `opts` may be NULL. */
int nusht_geometry_for(int lmax, int mmax, double eps, int dtype, const nusht_plan_opts* opts,
                   nusht_geometry* out);

/* Build a plan for `npts` points (theta in [0, pi], phi any finite value, taken mod 2 pi),
   both device arrays of float64 that the plan copies (the caller may free them afterwards).
   0 <= mmax <= lmax <= 16383, 1 <= npts < 2^31, 1e-14 <= eps <= 1e-1.
   Planning (the point binning of the nuFFT, Sec. III) is done here, once, and synchronises
   `stream`.  NUSHT_EINVAL also reports a theta outside [0, pi] or a non-finite coordinate,
   found by a device check.  On success *out owns all device scratch until nusht_destroy. */
int nusht_plan(int lmax, int mmax, int64_t npts, const double* theta, const double* phi,
               double eps, int dtype, nusht_plan_t* out);
int nusht_plan_ex(int lmax, int mmax, int64_t npts, const double* theta, const double* phi,
                  double eps, int dtype, const nusht_plan_opts* opts, void* stream,
                  nusht_plan_t* out);

/* Fills *out with the plan's sizes. */
int nusht_plan_info(nusht_plan_t plan, nusht_geometry* out);

/* Device-side status of the plan's execution calls so far: waits for the plan's device to
   finish its work, then returns NUSHT_EDEVICE (with nusht_last_error naming the kernel) if a
   kernel has flagged a failure it could not report through its own return value -- the
   bounded cross-wave wait of the Legendre adjoint (Eq. 6, S^H) giving up -- and NUSHT_OK
   otherwise.  The flag stays set until nusht_destroy.  nusht_solve and nusht_stage_stats
   check it as well. */
int nusht_plan_status(nusht_plan_t plan);

/* Type 2 (synthesis), Eq. (3): map[b][i] = sum_lm a_lm Y_lm(theta_i, phi_i), to accuracy eps.
   alm: [nmaps][nalm] complex128, map: [nmaps][npts] float64, nmaps >= 1.
   Scratch grows on the first call with a larger nmaps than before (that call allocates). */
int nusht_synthesis(nusht_plan_t plan, const double* alm, double* map, int nmaps, void* stream);

/* Type 1 (adjoint), Eq. (2): alm[b][lm] = sum_i map[b][i] conj(Y_lm(theta_i, phi_i)),
   0 <= m <= mmax.  No quadrature weights: this is the adjoint, not an inverse (Sec. II.A). */
int nusht_adjoint(nusht_plan_t plan, const double* map, double* alm, int nmaps, void* stream);

/* Spin-weighted transforms (the spin-n extension of Sec. V: Wigner's d in place of the
   Legendre functions in S; D, F and N are the spin-0 ones run on two real maps per field).
   Definitions: sY_lm(theta, phi) = slam_lm(theta) e^{i m phi} with
     slam_lm = (-1)^s sqrt((2l+1)/4pi) d^l_{m,-s}(theta)  (Wigner's d; the spin-raising ladder
     from the Y_lm above: (s+1)Y = eth(sY) / sqrt((l-s)(l+s+1)),
     eth = -sin^s(theta) (d/dtheta + i/sin(theta) d/dphi) sin^-s(theta)).
   A field of spin s >= 1 is a pair of real maps (Q, U) with Q + iU = sum_lm sa_lm sY_lm and
   gradient / curl coefficients G, C: sa_lm = -(G_lm + i C_lm), (-s)a_lm = -(-1)^s (G_lm - i C_lm);
   G and C of a real pair obey G_{l,-m} = (-1)^m conj(G_lm), so only m >= 0 is stored, as for
   spin 0.  Coefficients with l < s do not exist: they are ignored on input and written as 0.
   Layout: alm [nfields][2][nalm] complex128 (G, then C, of every field); map
   [nfields][2][npts] float64 (Q, then U).  For spin 1 and G = -sqrt(l(l+1)) a_lm, C = 0 the
   map is (Q, U) = -(d f/d theta, (d f/d phi)/sin theta) of the spin-0 map f of a_lm.
   The adjoint is the transpose under <.,.>_m above, applied to G and C alike.
   Plans: either DFS mode, 1 <= spin <= min(lmax, NUSHT_MAX_SPIN), and
   2 spin log2(1/tan(theta_1/2)) <= 800 with theta_1 = pi/(N_r - 1) the ring next to a pole
   (the two Wigner-d functions of a ring share one exponent; spin <= 35 at lmax 4095,
   <= 32 up to lmax 9000) -- NUSHT_EINVAL otherwise;
   the first call with a spin builds its recurrence table (32 bytes per coefficient, kept
   until the spin changes or the plan is destroyed, so that call synchronises and
   allocates).  The adjoint adds the sums of its waves with device atomics, so its results
   can differ between runs by rounding; on a deterministic plan it writes per-wave partial
   sums instead (16 bytes x 2 nfields x nalm per wave of one m, about 11 waves at lmax 4095,
   as plan scratch grown on demand like the batch scratch) and adds them in a fixed order: bit-identical repeats. */
#define NUSHT_MAX_SPIN 64
int nusht_synthesis_spin(nusht_plan_t plan, int spin, const double* alm, double* map,
                         int nfields, void* stream);
int nusht_adjoint_spin(nusht_plan_t plan, int spin, const double* map, double* alm, int nfields,
                       void* stream);
/* Spin-weighted synthesis plus the derivatives of Q and U with respect to the point
   coordinates (the component functions in the local basis, differentiated as functions of
   (theta, phi)): map, dtheta, dphi [nfields][2][npts].  FP64 plans only (NUSHT_EPRECISION
   otherwise); the same plan conditions as nusht_synthesis_spin. */
int nusht_synthesis_spin_deriv(nusht_plan_t plan, int spin, const double* alm, double* map,
                               double* dtheta, double* dphi, int nfields, void* stream);

/* Synthesis plus the derivatives of the map with respect to the point coordinates:
   dtheta[b][i] = d map[b][i] / d theta_i, dphi[b][i] = d map[b][i] / d phi_i.  FP64 plans only
   (NUSHT_EPRECISION otherwise).  Used for gradients with respect to lensing deflections. */
int nusht_synthesis_deriv(nusht_plan_t plan, const double* alm, double* map, double* dtheta,
                          double* dphi, int nmaps, void* stream);

/* Lensing pointing (App. C): the deflected angles of the plan's points under the lensing
   potential Phi with coefficients dlm (complex128 [nalm], same layout as alm).  The
   deflection is the gradient of Phi (Eq. C2): alpha_theta = dPhi/dtheta and
   alpha_phi = (dPhi/dphi) / sin(theta) (0 at an exact pole), from nusht_synthesis_deriv; each
   point then moves a distance alpha = |alpha| along the great circle in the direction
   (alpha_theta, alpha_phi) (Eq. C1).  theta_out, phi_out: float64 [npts], caller's point
   order, theta' in [0, pi], phi' in [0, 2 pi).  FP64 plans only (NUSHT_EPRECISION
   otherwise); the accuracy of alpha is the plan's eps.  Enqueues only. */
int nusht_pointing(nusht_plan_t plan, const double* dlm, double* theta_out, double* phi_out,
                   void* stream);

/* Eq. (C1) alone, for given deflection components: theta_out, phi_out [npts] are the angles
   of n' = cos(a) n + sin(a)/a (alpha_theta e_theta + alpha_phi e_phi), a = |alpha|, with
   n, e_theta, e_phi the right-handed basis at (theta, phi).  All arrays float64 device
   pointers [npts]; the outputs may alias the inputs.  Enqueues only. */
int nusht_deflect(const double* theta, const double* phi, const double* alpha_theta,
                  const double* alpha_phi, int64_t npts, double* theta_out, double* phi_out,
                  void* stream);

/* Gradients of a loss L(map) through the synthesis, given g = dL/dmap [nmaps][npts]:
   nusht_vjp_alm writes dL/dRe a + i dL/dIm a [nmaps][nalm], i.e. the adjoint Y^H g (Eq. 2)
   scaled by 2 for m > 0 (a_{l,-m} = (-1)^m conj(a_lm) carries the other half) and real for
   m = 0.  nusht_vjp_points writes grad_theta[i] = sum_b g[b][i] dtheta[b][i] and likewise
   for phi (dtheta, dphi from nusht_synthesis_deriv); either output may be NULL, not both. */
int nusht_vjp_alm(nusht_plan_t plan, const double* grad_map, double* grad_alm, int nmaps,
                  void* stream);
int nusht_vjp_points(const double* grad_map, const double* dtheta, const double* dphi,
                     double* grad_theta, double* grad_phi, int nmaps, int64_t npts, void* stream);
/* The same coefficient gradient for the spin-weighted synthesis: grad_map [nfields][2][npts]
   (dL/dQ, dL/dU) -> grad_alm [nfields][2][nalm] (dL/dRe + i dL/dIm of G and C): the spin
   adjoint scaled by 2 for m > 0 and real for m = 0.  Same plan conditions as
   nusht_adjoint_spin. */
int nusht_vjp_alm_spin(nusht_plan_t plan, int spin, const double* grad_map, double* grad_alm,
                       int nfields, void* stream);

/* Iso-latitude parts on their own (the S operator of Eq. 5 and its adjoint) on the plan's
   CC grid: ring[b][j][k] = map at (theta_j = j pi/(N_r-1), phi_k = 2 pi k / N_phi).
   ring: [nmaps][N_r][N_phi] float64.  The adjoint returns sum_jk ring[b][j][k] Y*_lm. */
int nusht_ring_synthesis(nusht_plan_t plan, const double* alm, double* ring, int nmaps,
                         void* stream);
int nusht_ring_adjoint(nusht_plan_t plan, const double* ring, double* alm, int nmaps,
                       void* stream);

/* Least-squares inverse (Sec. I: iterative inverse algorithms call the
   transforms repeatedly).  CGLS on min || W^(1/2) (S a - d) ||_2 in the <.,.>_m geometry:
   each iteration runs one synthesis and one adjoint plus FP64 device reductions.
   map: d [npts] (one map); alm: in = initial iterate x0 [nalm], out = solution;
   weights: [npts] float32 row weights W (NULL = all ones).  Iterates while the recurred
   ||d - S a|| / ||d|| is above tol, checked every iteration through one 8-byte device-to-host
   read; it then recomputes the true residual, and if that is still above tol restarts CGLS
   from the current iterate with the true residual (at most 4 restarts, within maxiter).
   *iters (iterations in total) and *relres (true residual of the returned iterate) are
   written.  Returns NUSHT_OK only when the true residual is <= tol, NUSHT_ENOCONV otherwise
   (the iterate is still written).  Synchronises. */
int nusht_solve(nusht_plan_t plan, const double* map, double* alm, const float* weights,
                double tol, int maxiter, int* iters, double* relres, void* stream);

/* nusht_solve that also records the recurred relative residual ||d - S a_k|| / ||d|| after
   each iteration k = 0..iters into `history`, a HOST array of at least maxiter + 1 doubles
   (NULL: not recorded).  The values are the ones the stopping test reads, so recording
   costs nothing extra. */
int nusht_solve_ex(nusht_plan_t plan, const double* map, double* alm, const float* weights,
                   double tol, int maxiter, int* iters, double* relres, double* history,
                   void* stream);

/* Spin-s least-squares inverse of nusht_synthesis_spin for one field: minimises
   ||W^(1/2) (S_s a - d)||_2 over its gradient and curl coefficients a by the CGLS iteration of
   nusht_solve_ex (same stopping test, restarts, status codes and history), with S_s^H
   = nusht_adjoint_spin, the transpose of S_s in <.,.>_m summed over the G and C triangles.
   spin: 1 <= spin <= min(lmax, NUSHT_MAX_SPIN), within the ring-grid limit of
   nusht_synthesis_spin.  map: FP64 [2][npts] (Q then U), device.  alm: complex FP64
   [2][nalm] (G then C), device, in/out: the initial iterate on entry (zeros for a cold
   start), the solution on return.  weights: FP32 [npts] > 0, device, or NULL; point i's
   weight multiplies its Q and its U residual.  Entries with l < spin stay as given (no
   harmonic reaches them).  Synchronises. */
int nusht_solve_spin(nusht_plan_t plan, int spin, const double* map, double* alm,
                     const float* weights, double tol, int maxiter, int* iters, double* relres,
                     double* history, void* stream);

/* ---------------------------------------------------------------------------------------
 * Learned quadrature weights for the weighted least-squares inverse.
 *
 * The paper has no such component; it uses the transforms as the inner loop of an
 * iterative inverse (Sec. I), and these calls build a preconditioner for nusht_solve: a
 * small network maps density features of each point to a positive weight w_i, trained so
 * that S^H W d approximates the least-squares solution.  All arrays are device pointers;
 * FP32 unless stated.  Calls only enqueue work (except nusht_weight_loss_grad).
 * ------------------------------------------------------------------------------------- */

/* Number of FP32 parameters of the 12 -> 128 -> 128 -> 128 -> 1 network (tanh hidden
   layers, softplus output).  Layout: for each layer its transposed weight [in][out]
   row-major, then its bias [out]. */
int64_t nusht_mlp_param_count(void);

/* density[ntheta][nphi] = (count of points in equal-angle cell) / (npts * cell area / 4 pi),
   cell (a, b) holding theta in [pi a / ntheta, pi (a+1) / ntheta) and phi mod 2 pi in
   [2 pi b / nphi, 2 pi (b+1) / nphi), indices clamped.  Uniform points give ~1.
   theta, phi: FP64 [npts].  ntheta * nphi <= 2^24.  Allocates a stream-ordered count
   buffer. */
int nusht_density_map(const double* theta, const double* phi, int64_t npts, int ntheta,
                      int nphi, float* density, void* stream);

/* nusht_density_map for callers that cannot allocate device memory (code under HIP graph
   capture, tight serving loops, harnesses that forbid hipMalloc): the same result, with the
   cell counts kept in a fixed device array of 65536 counts (256 KiB per GPU, held until the
   process ends) instead of a stream-ordered allocation.  No hipMalloc, hipFree or other
   allocating call is made.  ntheta * nphi > 65536 returns NUSHT_EINVAL.  Every call on one GPU
   shares that GPU's array: calls that overlap on one GPU (different streams, or host threads)
   race and must be serialised by the caller. */
int nusht_density_map_noalloc(const double* theta, const double* phi, int64_t npts, int ntheta,
                              int nphi, float* density, void* stream);

/* features[npts][12]: log density bilinearly interpolated between cell centres at the
   point; log density of the 3 x 3 cells around the point's cell (theta clamped, phi
   periodic, row-major); cos theta; sin theta.  log density is floored at log 1e-3. */
int nusht_point_features(const double* theta, const double* phi, int64_t npts,
                         const float* density, int ntheta, int nphi, float* features,
                         void* stream);

/* weights[i] = softplus(net(features[i])) * scale. */
int nusht_mlp_forward(const float* params, const float* features, int64_t npts, float scale,
                      float* weights, void* stream);

/* grad_params = d/dparams sum_i grad_weights[i] * weights[i], deterministic for a given npts
   (fixed per-block partial sums reduced in block order).  Allocates a stream-ordered
   partial buffer of at most 512 * nusht_mlp_param_count() floats. */
int nusht_mlp_backward(const float* params, const float* features, const float* grad_weights,
                       int64_t npts, float scale, float* grad_params, void* stream);

/* One Adam update of params[n] in place with first/second moments m, v (start at 0) and
   step >= 1 (bias corrections 1 - beta^step). */
int nusht_adam_step(float* params, const float* grad, float* m, float* v, int64_t n, float lr,
                    float beta1, float beta2, float eps, int step, void* stream);

/* alm = S^H (W d): the adjoint (Eq. 2) of the weighted map, i.e. the quadrature estimate of
   the coefficients and the initial iterate of a weighted nusht_solve.  d: FP64 [npts];
   weights: FP32 [npts]; alm: complex128 [nalm].  Allocates a stream-ordered [npts] buffer. */
int nusht_weighted_adjoint(nusht_plan_t plan, const double* d, const float* weights,
                           double* alm, void* stream);

/* Training loss of the weights for one point set: with r = S^H (W d) - astar (Eq. 2 applied
   to the weighted map), *loss = <r, r>_m / <astar, astar>_m (host double), and, if
   grad_weights != NULL, grad_weights[i] = 2 d_i (S r)_i / <astar, astar>_m (one synthesis).
   d: FP64 [npts] in the plan's point order; astar: complex128 [nalm]; weights: FP32 [npts].
   Synchronises (reads the loss). */
int nusht_weight_loss_grad(nusht_plan_t plan, const double* d, const double* astar,
                           const float* weights, float* grad_weights, double* loss,
                           void* stream);

/* Per-stage device times (ms) of the last execution call when the plan was built with
   opts.timing != 0 (HIP events recorded on the call's stream around each stage).
   Synchronises on the plan's last event.  Writes up to maxn values to ms and the stage
   names (static strings) to names (may be NULL); returns the count. */
int nusht_stage_times(nusht_plan_t plan, double* ms, const char** names, int maxn);

/* Kinds of execution call, for nusht_stage_stats. */
enum { NUSHT_CALL_SYNTHESIS = 0, NUSHT_CALL_ADJOINT = 1, NUSHT_CALL_SYNTHESIS_DERIV = 2,
       NUSHT_CALL_RING = 3, NUSHT_CALL_SPIN_SYNTHESIS = 4, NUSHT_CALL_SPIN_ADJOINT = 5 };

/* Mean per-stage device time (ms) over the calls of one kind made since the plan was built
   or since nusht_stage_reset (the most recent 64 calls of the plan count at most); ncalls
   (may be NULL) receives the number of calls averaged per stage.  Same output convention as
   nusht_stage_times; returns the number of stages written.  Synchronises. */
int nusht_stage_stats(nusht_plan_t plan, int kind, double* ms, int* ncalls, const char** names,
                      int maxn);

/* Forget the recorded calls (timing plans only; the events themselves are reused). */
void nusht_stage_reset(nusht_plan_t plan);

/* Frees everything the plan owns.  NULL is a no-op. */
void nusht_destroy(nusht_plan_t plan);

/* Static description of a status code. */
const char* nusht_strerror(int status);

/* Text naming the first failing check or HIP/rocFFT call of the calling thread's last failed
   call (empty if none).  Valid until the next failing call on the same thread. */
const char* nusht_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* NUSHT_H */
