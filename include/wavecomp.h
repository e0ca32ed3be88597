/*
 * wavecomp.h - C ABI of the MI355X (gfx950) library for the autoencoder-
 * compressed adjoint gradient and Gauss-Newton Hessian-vector product of
 * the acoustic velocity-strain inverse problem.
 *
 * Method: Wittmer, Badger, Sundar, Bui-Thanh, "An Autoencoder Compression
 * Approach for Accelerating Large-scale Inverse Problems" (arXiv 2304.04781).
 *   - forward model: Sec. 2, Eq. (model) with density 1: dv/dt = grad(c^2 e) + b,
 *     de/dt = div v, zero initial state, traction-free top surface;
 *   - parameter-to-observable map F = B A, B samples the vertical velocity at
 *     receivers (Sec. 2);
 *   - misfit J = 1/2 ||F(c) - d||^2 weighted by the noise covariance sigma^2 I
 *     (Sec. 2, MAP objective), time quadrature dt * sum over steps 1..T;
 *   - gradient by the adjoint method and Hv by incremental forward +
 *     incremental adjoint solves (Sec. 1 and Sec. 4); the adjoint is the
 *     exact transpose of the discrete forward map;
 *   - every forward state is stored compressed by a dense autoencoder and
 *     decompressed in the time-reversed solves (Sec. 3, 3.1, 3.3); states
 *     are normalised per vector by r = max(max - min, beta) (Sec. 3.3.1).
 *
 * Discretisation: cells (k, j, i) with k the depth index (k = 0 at the free
 * surface), x fastest. e at cell centres; v_z[k] on the face between cells
 * k-1 and k (v_y, v_x likewise). One step n -> n+1:
 *     v_a <- S_va (v_a + dt G_a(c^2 e) + dt b_a^n),   e <- S_e (e + dt D v),
 * G_a q[i] = (q[i]-q[i-1])/dx with q[-1] = 0; D v[i] = sum_a (v_a[i+1]-v_a[i])/dx
 * with v_a[n_a] = 0; S = exp(-dt * sum of absorbing profiles) (quadratic
 * profile over `sponge` cells on the bottom and the four sides, strength
 * 3 c_ref ln(1e3) / (2 sponge dx)); p^{n+1}_r = v_z at receiver face r.
 *
 * Conventions for every entry point:
 *   - Pointers are DEVICE pointers unless their name starts with h_ (host).
 *     The caller owns all argument buffers; the library never frees them.
 *   - State arrays are float32 [S][4][nz][ny][nx], field order (e, v_z, v_y, v_x),
 *     S = number of sources (one wavefield per source).
 *   - Traces, observations and residuals are float32 [S][T][R]; index n holds
 *     time level n+1.
 *   - Work is enqueued on the context's (or the given) HIP stream. Calls that
 *     return a host scalar (h_misfit, h_loss) synchronise that stream.
 *   - Return value: WV_OK (0) or WV_OK_FALLBACK (1) on success, a negative
 *     WV_E* code on failure; wv_last_error() then describes it (thread-local
 *     message). No C++ exception crosses this interface.
 *   - A wv_ctx is bound to one device and one stream and is not thread-safe.
 */
#ifndef WAVECOMP_H
#define WAVECOMP_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define WV_OK            0
#define WV_OK_FALLBACK   1   /* compressed result rejected by the accuracy guard;
                                checkpointed result returned instead */
#define WV_EINVAL      (-1)  /* bad argument (null pointer, size, NaN/negative speed) */
#define WV_ENOMEM      (-2)  /* device allocation failed or exceeds the memory budget */
#define WV_EDEVICE     (-3)  /* a HIP runtime call failed */
#define WV_ESTATE      (-4)  /* call order violated (e.g. hessvec without a matching forward) */
#define WV_EUNSTABLE   (-5)  /* c_max dt / dx >= 1/sqrt(dims): leapfrog unstable */
#define WV_ESHAPE      (-6)  /* grid not divisible into 8^3 patches for autoencoder storage */

/* Storage of the forward history consumed by the reverse-time solves. */
#define WV_STORE_NONE        0  /* forward only; adjoint calls fail with WV_ESTATE */
#define WV_STORE_FULL        1  /* every e^n, n = 1..T-1, in float32 (small problems) */
#define WV_STORE_CHECKPOINT  2  /* optimal binomial checkpointing ("revolve") with
                                   n_checkpoints state slots, the zero initial
                                   state counted as one (Sec. 1 checkpointing) */
#define WV_STORE_AE_BF16     3  /* autoencoder latents in bfloat16 (Sec. 3.1 space
                                   compression, 8^3-cell x 4-field patches) */
#define WV_STORE_AE_FP8      4  /* autoencoder latents in OCP FP8 E4M3FN with one
                                   float32 scale per patch */
#define WV_STORE_AE_TIME     5  /* time compression (Sec. 3.2): e only, 4^3 cells x 32
                                   consecutive levels per vector, bfloat16 latents;
                                   the reverse solves decode a whole window at once.
                                   Needs nz, ny, nx divisible by 4. Exception vectors:
                                   the K (wv_set_ae_exceptions) largest-range vectors
                                   of each window and source are kept exactly. No
                                   guard or fallback (space modes only) */

/* Latent formats of ae_encode / ae_decode. */
#define AE_LATENT_BF16  0
#define AE_LATENT_FP8   1

/* Fallback policy of wv_set_storage. */
#define WV_FALLBACK_NONE        0  /* report guard failures only through the guard error */
#define WV_FALLBACK_CHECKPOINT  1  /* recompute with checkpointing when the guard trips */

typedef struct wv_grid {
    int32_t nz, ny, nx;   /* cells; ny == 1 selects the 2D (z, x) mode (no y terms) */
    double dx;            /* cell size [m] */
    double dt;            /* time step [s] */
    int32_t nt;           /* number of time steps T (states 1..T, traces 1..T) */
    int32_t sponge;       /* absorbing layer width in cells (0 = none) */
    double c_ref;         /* speed setting the absorbing strength (e.g. max of the
                             true model); fixed so the layer does not depend on c */
    int32_t nsrc;         /* S: sources = independent wavefields (>= 1) */
    int32_t nrec;         /* R: receivers (>= 0) */
} wv_grid;

typedef struct wv_ctx wv_ctx;  /* opaque: grid, stream, history store, work buffers */
typedef struct ae_net ae_net;  /* opaque: autoencoder weights, Adam moments, scales */

typedef struct ae_train_cfg {
    int32_t epochs;        /* passes over the samples */
    int32_t batch;         /* samples per Adam step; a last partial batch is dropped */
    double lr;             /* initial learning rate */
    int32_t decay_every;   /* the rate is multiplied by decay_factor every this many epochs */
    double decay_factor;
    double beta1, beta2, eps;  /* Adam constants */
    int32_t weighting;     /* 0: plain mean squared error over the normalised
                              vectors (Sec. 3.3.1); 1: each (sample, field)
                              weighted by (r / beta_f)^2, i.e. the squared error
                              in the field's physical scale (needs meta) */
} ae_train_cfg;

/* ---- context --------------------------------------------------------------------- */

/* Create a solver context on the current device. h_src: [nsrc][3] (k, j, i) of
 * the v_z face carrying each source's vertical point force; h_rec: [nrec][3]
 * (k, j, i) of the sampled v_z faces (shared by all sources). stream: a
 * hipStream_t (NULL = default stream) that runs the stencil steps; the
 * compression, decompression and exception work of the autoencoder modes runs on
 * three non-blocking side streams at the default priority, created with the first
 * context on a device and shared by every context on it (calls on different
 * contexts of one device are serialised there, and events order them with each
 * context's stream). Fails with WV_EINVAL for indices outside the grid or a (y, x)
 * plane of 2^30 cells or more, WV_ENOMEM when work buffers cannot be allocated. */
int wv_create(const wv_grid* grid, const int32_t* h_src, const int32_t* h_rec,
              void* stream, wv_ctx** out);

/* Spatial shape of every source (paper Sec. 4.1: the Ricker force is smoothed
 * by a narrow Gaussian in space). The force density on the v_z faces is
 * wavelet[s][n] * w[dk][(dj)][di] at offsets |dk|, |dj|, |di| <= radius from the
 * source face (dk slowest; no dj in 2D), truncated at the grid boundary.
 * h_weights: host float32 [(2 radius + 1)^dims]. Default: radius 0, weight 1
 * (a point force). Invalidates the stored history. */
int wv_set_source_stencil(wv_ctx* ctx, int32_t radius, const float* h_weights);

/* Free every buffer the context owns. Safe on NULL. */
int wv_destroy(wv_ctx* ctx);

/* Choose how wave_forward keeps the history (WV_STORE_*). n_checkpoints is used
 * by WV_STORE_CHECKPOINT and by the fallback; ae must be non-NULL for the AE
 * modes (the context keeps a reference; the net must outlive it).
 * mem_budget_bytes > 0 caps the history allocation (WV_ENOMEM beyond it).
 * guard_tol > 0 enables the accuracy guard of the AE modes: during each forward
 * solve, 16 stored states spread evenly over it (every ceil((T-1)/16)-th state)
 * and the last one are decoded as the reverse solves read them (exception patches
 * exact) and their e compared with the true e while the solve still holds it
 * (one e field of scratch per source). The guard error is, per source, the
 * largest L2 error of a checked state over the largest L2 norm of the checked
 * states' e (so an early state that holds little of the wavefield does not
 * magnify the decoder's noise floor); its worst over sources above guard_tol
 * marks the store degraded, and with
 * fallback_policy WV_FALLBACK_CHECKPOINT gradient/hessvec then recompute with
 * checkpointing and return WV_OK_FALLBACK. Allocation happens here; the previous
 * store is freed first. Errors: WV_EINVAL (unknown mode or policy, missing net,
 * n_checkpoints < 1 where slots are needed), WV_ESHAPE (an AE mode on a grid that is
 * not 3D or not divisible into 8^3 patches, 4^3 blocks for WV_STORE_AE_TIME),
 * WV_ENOMEM (budget or device memory). An unknown mode or policy is rejected before
 * anything changes; after any other error the previous store is gone and the context
 * stores nothing (as WV_STORE_NONE): gradient and hessvec return WV_ESTATE until a
 * mode is set. */
int wv_set_storage(wv_ctx* ctx, int mode, int32_t n_checkpoints, ae_net* ae,
                   int64_t mem_budget_bytes, double guard_tol, int fallback_policy);

/* Error bounding for the AE modes: after compressing a state, the k_per_step
 * patches with the largest e-field range r also keep their e values exactly
 * (float32), and decompression of e restores them. Ranges are compared at a
 * resolution of 2^-5 relative (the top 14 bits of the float); within the bin of
 * the k-th largest range, lower patch indices come first.
 * In the time-compression mode k_per_step counts e-only vectors (4^3 cells x 32
 * levels) kept per window and source, chosen the same way.
 * 0 (default) stores latents only, as in the paper; the paper mentions storing
 * residuals to bound the error (Sec. 1, Sec. 3.3). Takes effect at the next
 * wv_set_storage. */
int wv_set_ae_exceptions(wv_ctx* ctx, int32_t k_per_step);

/* Precision of the per-patch normalisation metadata (lo, r) of the space-compressed
 * stores (Sec. 3.3.1 keeps an offset and a scale per vector): bits = 32 (default)
 * stores float32 pairs, 32 B per patch; bits = 16 stores bfloat16 pairs, 16 B per
 * patch, with lo rounded down and r rounded up to bfloat16 before the encoder
 * normalises, so lo <= min, lo + r >= max and the decoder reads exactly the values
 * the encoder used (no inconsistency; a patch whose offset dwarfs its range loses
 * up to 8 bits of its normalised resolution). This is what lets the 8-source FP8
 * workload keep 4000 steps of latents within one GPU. Needs the fused network
 * shape (hidden 512, latent 32). Applies to the incremental store too; takes
 * effect at the next wv_set_storage. WV_EINVAL for other bit counts. */
int wv_set_ae_metadata(wv_ctx* ctx, int32_t bits);

/* Compression of the incremental forward states (AE modes). The paper notes
 * that the incremental forward states can be compressed as well (Sec. 4); the
 * 384^3 Hessian-vector configuration stores both histories. With enable = 1,
 * every hessvec / wave_inc_forward of an AE mode also compresses each incremental
 * state dx_n (n = 1..T-1, every source, all four fields) through the same
 * autoencoder into a second latent store of the same format, with its own
 * exception patches; it is allocated at the first such call, within the memory
 * budget together with the forward store (WV_ENOMEM beyond it). The Gauss-Newton
 * product itself does not read these states (wv_decode_delta returns them).
 * enable = 0 frees the store. In WV_STORE_AE_TIME the same setting keeps de_n
 * (e only) in an incremental time store of the forward store's layout; the
 * full-Newton product fills that store in any case, and enable = 0 frees it too.
 * Other modes ignore the setting. */
int wv_set_delta_storage(wv_ctx* ctx, int32_t enable);

/* Decompress the stored incremental state dx_n (1 <= n <= T-1) of every source
 * into state [S][4][N] (device): the fields whose bit is set in field_mask (bit f
 * = field f: e, v_z, v_y, v_x; others untouched), the exception patches of e
 * exact. In WV_STORE_AE_TIME only e is stored (field_mask must be 1): its window
 * is decompressed whole, the exception vectors exact. WV_ESTATE when the last
 * incremental forward stored none (or a forward solve ran since); WV_EINVAL for a
 * bad mask, a level outside [1, T-1] (time store) or NULL state. */
int wv_decode_delta(wv_ctx* ctx, int32_t n, uint32_t field_mask, float* state);

/* Bytes of history storage the current mode holds (after wv_set_storage), plus
 * the incremental store once allocated. */
int wv_storage_bytes(const wv_ctx* ctx, int64_t* h_bytes);

/* ---- wave solves (paper Sec. 2; Sec. 1 and 4 for the adjoint solves) ------------- */

/* Forward solve from the zero state over T steps at wave speed c [nz*ny*nx] for
 * every source; wavelet [S][T] is the force density b^n (already divided by
 * dx^dims). Writes traces [S][T][R]; final_state [S][4][N] if non-NULL. Fills the
 * history store of the current mode (compressing each state for the AE modes).
 * capture (if non-NULL) receives raw float32 states [ncap][S][4][N] of steps
 * n = capture_every, 2 capture_every, ... (ncap = floor((T-1)/capture_every)):
 * the training snapshots of the learned compressor. */
int wave_forward(wv_ctx* ctx, const float* c, const float* wavelet, float* traces,
                 float* final_state, float* capture, int32_t capture_every);

/* wave_forward that also copies e^n of every source at the nsteps listed levels
 * h_steps[q] (host, distinct, each in [1, T]) into e_out [nsteps][S][N] in list
 * order (the training levels of the time-compression network); no traces out. */
int wave_forward_e(wv_ctx* ctx, const float* c, const float* wavelet, const int32_t* h_steps,
                   int32_t nsteps, float* e_out);

/* e^n [S][N] (1 <= n <= T-1) as the reverse solves read it from the store of the
 * last forward solve: the float32 copy (full storage), the decoded state with its
 * exact patches (AE modes) or the decoded window level (time compression).
 * WV_ESTATE without such a store (checkpointing included). Synchronises. */
int wv_load_e(wv_ctx* ctx, int32_t n, float* out);

/* Reverse-time adjoint solve consuming the store of the last wave_forward at the
 * same c: returns g = J_F^T w, i.e. g = -2 dt c * sum_n e^n * q^n for the adjoint
 * source w = residual [S][T][R] (pass dt/sigma^2 (p - d) for the misfit
 * gradient). g is summed over sources. WV_ESTATE if no store is available
 * (checkpoint slots are consumed by one reverse sweep). */
int wave_adjoint(wv_ctx* ctx, const float* c, const float* residual, float* g);

/* Misfit gradient: forward solve (filling the store), J = dt/(2 sigma^2)
 * sum (p - d)^2 in float64, residual dt/sigma^2 (p - d), adjoint solve.
 * d_obs [S][T][R]; g [N]; *h_misfit receives J. */
int gradient(wv_ctx* ctx, const float* c, const float* wavelet, const float* d_obs,
             double sigma, float* g, double* h_misfit);

/* Hessian-vector product at the c of the last gradient() (sigma taken from that
 * call), reading the forward history (decompressed again for the AE modes:
 * compress once, decompress in every Hv).
 * gauss_newton = 1: Hdc = J_F^T (dt/sigma^2) J_F dc: incremental forward with
 * source dm e^n (dm = 2 c dc), then the incremental adjoint (Sec. 4).
 * gauss_newton = 0: the full-Newton product, the derivative of the gradient along
 * dc, Hdc = -2 dt (dc * sum_n e^n q^n + c * sum_n (de^n q^n + e^n dq^n)): the
 * incremental forward keeps de^n (full storage; compressed into the incremental
 * latent store in the AE modes; in WV_STORE_AE_TIME into a second time store of
 * the same layout and exception count, allocated at the first such call within
 * the memory budget together with the forward store), then the adjoint mu of the
 * last gradient's residual and the incremental adjoint dmu (residual dt/sigma^2
 * dp, and -dt dm q in its eta equation) step together in reverse time. Needs the
 * full, an AE or the time store (WV_ESTATE for checkpointing or after a fallback).
 * WV_ESTATE when c differs from the last gradient's c or no store exists. */
int hessvec(wv_ctx* ctx, const float* c, const float* dc, float* Hdc, int gauss_newton);

/* Incremental forward only: dp [S][T][R] = J_F dc (uses the stored history). */
int wave_inc_forward(wv_ctx* ctx, const float* c, const float* dc, float* dtraces);

/* ---- MAP point: BiLaplacian prior (paper Sec. 2) and Newton-CG (Sec. 4) ----------- */

/* Prior term of the MAP objective, 1/2 ||c - c0||^2 weighted by the inverse prior
 * covariance, with the BiLaplacian prior of Sec. 2: the inverse covariance is the
 * square of the elliptic operator
 *     A u = alpha (u - div(Theta grad u)),   zero normal flux of Theta grad u
 * on the boundary, Theta = diag(theta_z, theta_y, theta_x) [m^2]. On the grid:
 * (A u)_i = alpha (u_i - sum over the faces of cell i shared with a neighbour nb
 * of theta_a (u_nb - u_i) / dx^2) (boundary faces carry no flux), and with the
 * lumped mass dx^dims I (dims = 2 when ny == 1, whose y term vanishes)
 *     R(c) = 1/2 dx^dims ||A (c - c0)||^2,   grad R = dx^dims A A (c - c0),
 *     Hess R = dx^dims A A.
 * wv_set_prior copies c0 [N] (device) into the context; alpha = 0 removes the
 * prior (c0 may then be NULL). WV_EINVAL for negative or non-finite alpha or
 * theta. */
int wv_set_prior(wv_ctx* ctx, double alpha, const double* h_theta, const float* c0);

/* R(c) into *h_cost (may be NULL), and g += grad R when g is non-NULL. Both are
 * zero without a prior. Synchronises the context's stream when h_cost is set. */
int wv_prior(wv_ctx* ctx, const float* c, float* g, double* h_cost);

/* Hdc += dx^dims A A dc (nothing without a prior). */
int wv_prior_hessvec(wv_ctx* ctx, const float* dc, float* Hdc);

/* A draw from the prior N(c0, (dx^dims A A)^-1) (Sec. 3.3.1, Algorithm 1: the
 * compressor's training states come from forward solves at prior draws):
 * out = c0 + x with A x = w / sqrt(dx^dims), for white noise w [N] (device, drawn
 * by the caller). x is found by conjugate gradients from 0 (A is symmetric
 * positive definite) until |r| <= rtol |w / sqrt(dx^dims)| or maxit iterations;
 * *h_iters and *h_relres (may be NULL) report the iterations and the final
 * relative residual. WV_ESTATE without a prior. Uses the Newton-CG work vectors. */
int wv_prior_sample(wv_ctx* ctx, const float* w, float* out, double rtol, int32_t maxit, int32_t* h_iters,
                    double* h_relres);

typedef struct wv_newton_cfg {
    int32_t max_newton;     /* Newton iterations (>= 0) */
    int32_t max_cg;         /* conjugate-gradient iterations per Newton step (>= 1) */
    double eta_max;         /* cap of the forcing eta = min(eta_max, sqrt(|g| / |g_0|)), in (0, 1) */
    double rel_tol;         /* stop once |g| <= rel_tol |g_0| (>= 0) */
    double c_armijo;        /* sufficient decrease J(c + a p) <= J + c_armijo a g.p, in (0, 1) */
    int32_t max_backtrack;  /* halvings of the step length before the line search fails (>= 0) */
    int32_t gauss_newton;   /* 1: Gauss-Newton misfit Hessian, 0: full Newton (full, AE or time store) */
    int32_t precondition;   /* 1: CG preconditioned by the prior covariance (dx^dims A A)^-1, each
                               application two elliptic solves by CG to 1e-6 relative residual;
                               0: none. 1 needs a prior (WV_ESTATE otherwise) */
} wv_newton_cfg;

typedef struct wv_newton_rec {
    double cost;        /* J = misfit + prior at the iterate */
    double misfit;
    double prior;
    double gnorm;       /* |g|, g = gradient of J */
    double step;        /* accepted step length (0 for the last iterate) */
    double cg_rel_res;  /* |r|_M / |g|_M of the CG recurrence when CG stopped (r = -g - H p) */
    int32_t cg_iters;   /* Hessian actions spent on the step from this iterate */
    int32_t neg_curv;   /* CG stopped at non-positive curvature */
    int32_t backtracks; /* step halvings (max_backtrack + 1: line search failed) */
    int32_t status;     /* return code of the gradient at the iterate (WV_OK or WV_OK_FALLBACK) */
} wv_newton_rec;

/* Inexact Newton-CG for the MAP point (Sec. 4; the paper's references on
 * Newton-CG for wave inversion): from c (device [N], updated in place), repeat
 *   1. J, g at the iterate: gradient() plus the prior term (for later iterates
 *      the accepted trial of the line search already computed them);
 *   2. stop if |g| <= rel_tol |g_0|;
 *   3. conjugate gradients on H p = -g from p = 0, H = hessvec() + prior Hessian
 *      (each iteration one Hessian action, which decompresses the stored forward
 *      history again in the AE modes), optionally preconditioned by the prior
 *      covariance M, until |r|_M <= eta |g|_M (|r|_M = sqrt(r.Mr), M = I without
 *      preconditioning) with eta = min(eta_max, sqrt(|g| / |g_0|)), max_cg
 *      iterations, or non-positive curvature d.Hd <= 0 (then the iterate so far
 *      is kept, or p = d = -M g at the first iteration);
 *   4. Armijo backtracking from the step length 1, halving; every trial runs a
 *      gradient (forward with storage + adjoint), so an accepted trial leaves its
 *      store for the next Hessian actions. A trial speed outside the stable,
 *      positive range is rejected like an increase of J.
 * Vector updates are float32, dot products float64.
 * h_log: host array of max_newton + 1 records (iterates 0 .. *h_iters);
 * *h_iters: Newton steps taken; *h_reason: 0 iteration limit, 1 gradient
 * tolerance, 2 line search failed (c then holds the last accepted iterate and the
 * store belongs to the last trial). Needs a storage mode other than WV_STORE_NONE. */
int wv_newton_cg(wv_ctx* ctx, float* c, const float* wavelet, const float* d_obs, double sigma,
                 const wv_newton_cfg* cfg, wv_newton_rec* h_log, int32_t* h_iters, int32_t* h_reason);

/* ---- autoencoder (paper Sec. 3.3 architecture, Eq. (single_layer); Sec. 3.3.1) --- */

/* Create a dense autoencoder in_dim -> hidden -> latent -> hidden -> in_dim with
 * GELU on the hidden layers (in_dim must be 2048 = 4 fields x 8^3, hidden a
 * multiple of 64, latent a multiple of 16). h_init: host float32 parameters in
 * the order W1 [in][hid], b1 [hid], W2 [hid][lat], b2 [lat], W3 [lat][hid],
 * b3 [hid], W4 [hid][in], b4 [in] (input-major weights, y W + b). The library
 * keeps float32 master weights, bfloat16 copies and Adam moments on the device.
 * h_beta: per-field normalisation floors beta_f [4] (NULL = 1e-7 each). */
int ae_create(int32_t in_dim, int32_t hidden, int32_t latent, const float* h_init,
              const double* h_beta, ae_net** out);
void ae_destroy(ae_net* net);

/* Number of float32 parameters (layout as h_init). */
int ae_param_count(const ae_net* net, int64_t* h_count);
/* Copy the float32 master parameters to / from host memory (layout as h_init). */
int ae_get_params(const ae_net* net, float* h_out);
int ae_set_params(ae_net* net, const float* h_in);
/* Set / get the per-field floors beta_f. */
int ae_set_beta(ae_net* net, const double* h_beta);
int ae_get_beta(const ae_net* net, double* h_beta);
/* Set beta_f = rel * max |x_f| over nstates raw states [nstates][4][N]
 * (field-wise maxima; the paper's beta = 1e-7 taken relative to each
 * field's scale). */
int ae_fit_beta(ae_net* net, const wv_grid* grid, const float* states, int64_t nstates,
                double rel, void* stream);
/* Save / load weights, biases, Adam moments, step count and floors (binary file). */
int ae_save(const ae_net* net, const char* path);
int ae_load(const char* path, ae_net** out);

/* Normalise one state [4][N] into the network input layout: y [P][2048] bfloat16
 * (bit patterns, patch p = (pz*Py + py)*Px + px, entry f*512 + lz*64 + ly*8 + lx),
 * meta [P][4][2] = (min, r) per patch and field with r = max(max - min, beta_f). */
int ae_normalize(const ae_net* net, const wv_grid* grid, const float* state, uint16_t* y,
                 float* meta, void* stream);

/* The rows of ae_normalize for the listed patches only: row q of y [nrows][2048]
 * and meta [nrows][4][2] is patch rows[q] (device int32, each in [0, P), checked
 * before launch: WV_EINVAL otherwise). Keeping a random subset of the patch
 * vectors of each state is the write-or-discard step of the training-data
 * generation (Sec. 3.3.1, Algorithm 1). */
int ae_normalize_rows(const ae_net* net, const wv_grid* grid, const float* state, const int32_t* rows,
                      int32_t nrows, uint16_t* y, float* meta, void* stream);

/* ---- time compression (paper Sec. 3.2) ---------------------------------------------
 * A vector holds one field, e (the only one the reverse solves read), on a 4^3
 * block of cells over a window of 32 consecutive time levels: entry
 * t*64 + lz*16 + ly*4 + lx, vector s*B + b for source s (grid->nsrc sources) and
 * block b = (bz*By + by)*Bx + bx, B = (nz/4)(ny/4)(nx/4). A window buffer e_win
 * holds levels [32][S][N] (or [nvalid][S][N]); a window of nvalid < 32 levels
 * (the last of a solve) is completed by repeating its last level. Each vector is
 * normalised as a whole, r = max(max - min, beta_e) (Sec. 3.3.1, beta_e = the
 * net's first floor). The net must have in_dim 2048. WV_ESHAPE unless the grid is
 * 3D with nz, ny, nx divisible by 4; WV_EINVAL for nvalid outside [1, 32]. */

/* beta_e = rel * max |e| over nlevels levels e [nlevels][S][N]. */
int ae_time_fit_beta(ae_net* net, const wv_grid* grid, const float* e, int64_t nlevels, double rel,
                     void* stream);
/* Normalised vectors y [n][2048] (bfloat16 bits) and meta [n][2] = (lo, r) of the
 * vectors rows[0..nrows) (device int32 in [0, S*B), checked before launch), or of
 * all S*B vectors in order when rows is NULL (n = S*B). */
int ae_time_normalize(const ae_net* net, const wv_grid* grid, const float* e_win, int32_t nvalid,
                      const int32_t* rows, int32_t nrows, uint16_t* y, float* meta, void* stream);
/* Compress a window: latent [S*B][latent] bfloat16, meta [S*B][2]. */
int ae_time_encode(const ae_net* net, const wv_grid* grid, const float* e_win, int32_t nvalid,
                   uint16_t* latent, float* meta, void* stream);
/* Decompress into levels 0..nvalid-1 of the window buffer e_win. */
int ae_time_decode(const ae_net* net, const wv_grid* grid, const uint16_t* latent, const float* meta,
                   int32_t nvalid, float* e_win, void* stream);

/* Compress one state [4][N]: per-patch normalisation, encoder, latent store.
 * latent: [P][latent] bfloat16 (AE_LATENT_BF16) or e4m3 bytes (AE_LATENT_FP8);
 * qscale [P] float32 scales (FP8 only, else may be NULL); meta [P][4][2]. */
int ae_encode(const ae_net* net, const wv_grid* grid, const float* state, int latent_fmt,
              void* latent, float* meta, float* qscale, void* stream);

/* ae_encode for callers that cannot allocate device memory (code under HIP graph
 * capture, serving loops, harnesses that forbid hipMalloc): the same kernels and
 * results as ae_encode, bit for bit, but no allocation of any kind. The float32
 * latents of an FP8 encode are staged in a static device array of 16 MiB that the
 * library holds on each device it runs on until the process ends (its address is
 * looked up at the first FP8 call on a device); bfloat16 latents need no staging.
 * Limits: the fused network shape (hidden 512, latent 32, else WV_EINVAL) and, for
 * AE_LATENT_FP8, P * latent * 4 <= 16 MiB, i.e. at most 131072 patches (WV_EINVAL
 * beyond, before any work is queued). Every call on one device shares that
 * device's array and nothing in it needs to start at zero; calls that overlap in
 * time on one device (two streams, or two threads) race on it. */
int ae_encode_noalloc(const ae_net* net, const wv_grid* grid, const float* state, int latent_fmt,
                      void* latent, float* meta, float* qscale, void* stream);

/* Decompress into state [4][N]: decoder, de-normalisation x = min + r y. Only
 * the fields whose bit is set in field_mask (bit f = field f) are computed and
 * written (the gradient needs only e, mask 1). */
int ae_decode(const ae_net* net, const wv_grid* grid, const void* latent, const float* meta,
              const float* qscale, int latent_fmt, uint32_t field_mask, float* state,
              void* stream);

/* Train on nsamples normalised vectors y [nsamples][2048] (bfloat16 bits, e.g.
 * from ae_normalize) by minimising the (optionally weighted) mean squared
 * reconstruction error with Adam (Sec. 3.3.1 loss, Table 2 schedule).
 * meta: [nsamples][4][2] from ae_normalize (required when h_cfg->weighting = 1,
 * else may be NULL). perm: device int32 [epochs][nsamples] visiting order per
 * epoch (NULL = in order). h_loss_per_epoch (host, may be NULL) receives the
 * mean batch loss per epoch. The batch must be a multiple of 32. */
int ae_train(ae_net* net, const uint16_t* y, const float* meta, int64_t nsamples,
             const ae_train_cfg* h_cfg, const int32_t* perm, float* h_loss_per_epoch,
             void* stream);

/* One training step on a batch given explicitly (rows idx[0..batch) of y and
 * meta) and, if h_grads is non-NULL, the float32 parameter gradients of that
 * step (layout as h_init) copied to the host before the Adam update. Returns
 * the batch loss. */
int ae_train_step(ae_net* net, const uint16_t* y, const float* meta, const int32_t* idx,
                  int32_t batch, double lr, const ae_train_cfg* h_cfg, float* h_grads,
                  double* h_loss, void* stream);

/* ---- host-only helpers ---------------------------------------------------------- */

/* Optimal checkpoint schedule for reversing nsteps steps with nslots slots (the
 * slot of the zero initial state included). Actions are int32 triples
 * (kind, a, b): kind 0 = advance from state a by b steps, 1 = store the current
 * state (step a) in slot b, 2 = restore slot b (step a), 3 = deliver state a to
 * the adjoint. Writes at most cap triples to h_actions and the count to
 * *h_count; *h_forward_steps = number of step evaluations. Runs on the host. */
int wv_revolve_schedule(int32_t nsteps, int32_t nslots, int32_t* h_actions, int64_t cap,
                        int64_t* h_count, int64_t* h_forward_steps);

/* Diagnostics of the last solve: step evaluations of the forward model (sweep
 * plus checkpoint recomputation), the guard error of the accuracy guard (the
 * largest L2 error of e among its checked states over their largest e norm, worst
 * source; -1 if not run) and whether it tripped.
 * Any pointer may be NULL. */
int wv_stats(const wv_ctx* ctx, int64_t* h_forward_steps, double* h_guard_err, int* h_degraded);

/* Kernel timing. every > 0: every every-th launch of each timed class is
 * bracketed by HIP events recorded on the stream that runs it: the context's
 * stream for the stencil steps; in the autoencoder modes the device's side
 * streams for the compression (forward sweep), the exception selection and copy
 * (forward sweep) and the decompressions of the reverse and incremental sweeps,
 * which run beside the stencil steps. every = 0 switches timing off. Either call
 * clears the totals. */
int wv_set_timing(wv_ctx* ctx, int32_t every);

/* Mean duration in microseconds and number of timed launches since the last
 * wv_set_timing, for one class: 0 forward stencil step, 1 adjoint stencil step,
 * 2 incremental-forward stencil step, 3 compression of one state (all sources),
 * 4 decompression of one e field (with its exception patches written exactly),
 * 5 selection of the exception patches of one state, 6 a separate exception
 * restore (not launched: the decompression writes those patches), 7 copy of the
 * exception patches of one state. In the time-compression mode classes 3 and 4
 * time the compression and decompression of one window of 32 levels, on the
 * context's stream. Waits for the timed work. NULL outputs are skipped;
 * WV_EINVAL for an unknown class. */
int wv_kernel_time(wv_ctx* ctx, int32_t cls, double* h_mean_us, int64_t* h_count);

/* Number of consecutive adjoint steps whose gradient terms e^k q^k are summed in
 * float32 before the sum is added to the compensated (Kahan) accumulator (Sec. 2,
 * the time integral of the gradient): the adjoint step reads and writes the
 * float32 partial every step and the compensated pair once per block. */
int wv_accumulation_block(void);

/* Measurement aid, no part of the solves: the HBM rate of a plain streaming kernel
 * with the stencils' array mix, the practical ceiling they are compared with next
 * to the published peak. in: n_in arrays [n_in][n], out: n_out arrays [n_out][n]
 * (device float32, n a positive multiple of 4); every element of every array is
 * read or written once per launch (float4 per thread, non-temporal). Mixes
 * (n_in, n_out): (1, 1) copy, (5, 4) the forward step's, (7, 5) the adjoint
 * step's. Runs one warm-up and reps timed launches on stream (HIP events) and
 * returns the mean duration in microseconds in *h_us; synchronises. WV_EINVAL for
 * another mix, reps < 1 or a bad n. */
int wv_stream_probe(const float* in, float* out, int32_t n_in, int32_t n_out, int64_t n, int32_t reps,
                    void* stream, double* h_us);

const char* wv_last_error(void);
const char* wv_version(void);

#ifdef __cplusplus
}
#endif
#endif /* WAVECOMP_H */
