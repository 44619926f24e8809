/*
 * lbm.h -- C ABI of the MI355X (gfx950) fused lattice-Boltzmann LES
 * forest-canopy step.
 *
 * The method is that of Shao et al., "Near-wall approximations to speed up
 * simulations for atmosphere boundary layers in the presence of forests using
 * lattice Boltzmann method on GPU" (arXiv 2206.15454): D3Q19 BGK lattice
 * Boltzmann with Guo forcing (Sec. 2.1), Smagorinsky eddy viscosity
 * (Sec. 2.2), forest drag injected as a body force with a leaf-area-density
 * profile (Sec. 2.3), in the per-step order of Algorithm 1 (Sec. 3).
 *
 * Conventions (every entry point):
 *  - Lattice units: dx = dt = 1, c_s^2 = 1/3.  x is streamwise, y wall-normal,
 *    z spanwise.  Cell (i,j,k) has centre height y_j = j + 1/2; the walls are
 *    the planes y = 0 and y = ny.  x and z are periodic.
 *  - Arrays are C order [component][z][y][x], x fastest.  Populations are
 *    [19][z][y][x] in the direction order of lbm_lattice().
 *  - Every call returns an lbm_status; no C++ exception crosses the ABI.
 *    lbm_last_error() gives a message for the last failed call on a context.
 *  - A context is used by one host thread at a time.  Work is enqueued on the
 *    context's HIP stream; only lbm_moments, lbm_stats(READ) and lbm_get_f
 *    synchronise that stream.
 *  - "on_device" pointers are device pointers on the context's device;
 *    otherwise host pointers.  The caller keeps ownership of every array it
 *    passes; the library copies what it needs before returning.
 */
#ifndef LBM_H
#define LBM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct lbm_ctx lbm_ctx; /* opaque, owned by the library */

typedef enum {
    LBM_OK = 0,
    LBM_EINVAL = 1,    /* invalid argument (value, size, NULL, blob shape) */
    LBM_ENOMEM = 2,    /* device or host allocation failed, or dev_bytes too small */
    LBM_EDEVICE = 3,   /* a HIP call failed; the message holds hipGetErrorString */
    LBM_ESTATE = 4,    /* call not valid in the current state (e.g. step before init) */
    LBM_EUNSTABLE = 5  /* non-finite moments or max |u| > 0.35 were found */
} lbm_status;

/* Population storage.  The "S" types store the shifted value f_i - w_i
 * (w_i the lattice weight) so that the small deviations from rest keep their
 * digits; F32 storage is shifted as well, F64 stores the same shifted value in
 * double.  Arithmetic is FP64 for LBM_F64 and FP32 for the others.
 * Rounding into storage is round-to-nearest-even, except LBM_BF16SR: BF16
 * with stochastic rounding (rounds up with probability equal to the dropped
 * fraction; the random bits are a hash of the step, the cell and the
 * direction, so runs are reproducible).  Initial and imported states are
 * rounded to nearest. */
typedef enum { LBM_F64 = 0, LBM_F32 = 1, LBM_F16S = 2, LBM_BF16S = 3, LBM_BF16SR = 4 } lbm_storage;

/* Wall-normal (y) boundaries.  BOUNCEBACK is the halfway no-slip wall;
 * FREESLIP is specular reflection (a symmetry plane); EQUILIBRIUM is the
 * forced-equilibrium boundary of Sec. 5.1 (the upper boundary "moves with the
 * free-stream velocity"): every population entering through it is
 * feq(1, u_wall), populations leaving through it are lost; PERIODIC must be
 * set on both ends or neither. */
typedef enum {
    LBM_BC_PERIODIC = 0,
    LBM_BC_BOUNCEBACK = 1,
    LBM_BC_FREESLIP = 2,
    LBM_BC_EQUILIBRIUM = 3
} lbm_bc;

typedef enum { LBM_CLOSURE_SMAG = 0, LBM_CLOSURE_MLP = 1 } lbm_closure;

typedef struct lbm_params {
    int32_t nx, ny, nz;  /* cells, each >= 1; nx*ny*nz < 2^31 */
    int32_t storage;     /* lbm_storage */
    double tau0;         /* molecular relaxation time, > 0.5 (nu0 = (tau0 - 1/2)/3) */
    double c_smag;       /* Smagorinsky constant C_smag of Sec. 2.2 (= Cs^2), >= 0; 0 = off */
    double g[3];         /* driving acceleration; force density rho*g (Sec. 4, Eq. Body_force) */
    int32_t bc_ylo;      /* lbm_bc at y = 0  */
    int32_t bc_yhi;      /* lbm_bc at y = ny */
    void *stream;        /* hipStream_t to enqueue on; NULL = the null stream */
    double u_wall[3];    /* velocity of an LBM_BC_EQUILIBRIUM boundary (finite) */
    int32_t forest_map;  /* != 0: reserve device memory for a heterogeneous forest
                            (lbm_set_forest): 2 bytes per cell + a 768 KiB table */
} lbm_params;

typedef struct lbm_diag {
    double mass;         /* sum of rho over cells, FP64 */
    double mom[3];       /* sum of rho u (force-corrected velocity), FP64 */
    double impulse[3];   /* sum over all steps and cells of the body force F, FP64 */
    double max_u;        /* max |u| over cells */
    int64_t t;           /* steps done since lbm_init */
    int64_t nonfinite;   /* cells whose rho, u or nu_t is not finite */
    int64_t mlp_fallback;/* cells where the learned closure fell back to Smagorinsky
                            in its last evaluation (0 with the Smagorinsky closure) */
} lbm_diag;

/* D3Q19 direction table: rest; +x,-x,+y,-y,+z,-z; then the twelve edge
 * vectors, each followed by its opposite (q odd and q+1 are opposite):
 * (1,1,0) (-1,-1,0) (1,-1,0) (-1,1,0) (1,0,1) (-1,0,-1) (1,0,-1) (-1,0,1)
 * (0,1,1) (0,-1,-1) (0,1,-1) (0,-1,1).  Weights 1/3, 1/18 (axis), 1/36
 * (edge).  c: [19][3], w: [19] (either may be NULL).  Returns 19. */
int32_t lbm_lattice(int32_t *c, double *w);

/* Device bytes one context needs (populations, moments, partial sums; the
 * population rows padded to whole 128-byte lines, see lbm_create).
 * Returns 0 for invalid parameters. */
size_t lbm_required_bytes(const lbm_params *p);

/* Create a context on the current HIP device.  dev_buf == NULL: the library
 * allocates; otherwise dev_buf is a caller-owned device buffer of dev_bytes
 * >= lbm_required_bytes(p), 256-byte aligned, that must outlive the context.
 * EINVAL for bad parameters (tau0 <= 0.5, a dimension < 1, periodic on one
 * end only, unknown storage); ENOMEM if the buffer is too small or the
 * allocation fails.  *out is NULL on failure.
 *
 * Launch choices are made here from the grid and storage type; environment
 * variables read at this call override them (for tests and tuning; the
 * populations are bit-identical under every choice, FP64 diagnostic sums
 * may differ in their last bits through the summation order):
 *   LBMX_BX=64|128|256      tile width in x (default: the widest of 256, 128,
 *                           64 that pads a row least)
 *   LBMX_ZALIGN=bytes       population z-layers (px ny cells) rounded up to a
 *   LBMX_ZPAD=bytes         multiple of, or widened by, this many bytes (a
 *                           multiple of 128; default: neither)
 *   LBMX_QPAD=bytes         pad between population planes (default 2048 for
 *                           the 16-bit types, 1024 otherwise)
 *   LBMX_XCD_REMAP=0|1      one contiguous tile range per XCD (default 1;
 *                           0: blocks go to the XCDs round robin)
 *   LBMX_XCD_RUN=tiles      the XCDs take turns in runs of this many tiles
 *                           (default: 2 for the step of FP32 and 4 for FP64
 *                           arrays above 256 MiB; the learned-closure
 *                           kernel keeps one range per XCD)
 *   LBMX_WIDE=0|1           64-bit population addresses (default: only when
 *                           buffer resources cannot address the array)
 *   LBMX_STREAMING=0|1      non-temporal population accesses (default: when
 *                           the population array exceeds 256 MiB and a row
 *                           is a whole number of 128-byte lines)
 *   LBMX_TILE_ORDER=0|1     row-major or memory-order tile numbering (default:
 *                           memory order for FP32 and FP64 arrays above
 *                           256 MiB, otherwise unless rows stream and a plane
 *                           is at most 96 MiB)
 *   LBMX_FX=0|1             kernels that leave out the y and z force terms
 *                           when g_y = g_z = 0 and the drag is x-only
 *                           (default 1)
 *   LBMX_MLP_SPLIT=0|1      a step that evaluates the learned closure runs
 *                           the network's kernel on the rows whose y/h lies
 *                           in the closure's range and the plain step on the
 *                           others, whose cells all fall back (default 1;
 *                           0: the network's kernel on every row)
 *   LBMX_MLP_OVERLAP=N      with that split, the plain rows run on a second
 *                           stream of the library's beside the network's
 *                           kernel, which takes N blocks per CU (default 2;
 *                           0: one stream, the launches in turn).  The
 *                           caller's stream waits for both; results are the
 *                           same bit for bit
 *   LBMX_PITCH=0|1          population rows padded to whole 128-byte lines
 *                           (default: for population arrays above 256 MiB,
 *                           rows of nx cells that are not whole lines get a
 *                           pitch of the next whole number of lines; the
 *                           step writes values of no meaning to the pad
 *                           cells, so that every line is written whole, and
 *                           no cell of the grid reads them) */
lbm_status lbm_create(const lbm_params *p, void *dev_buf, size_t dev_bytes, lbm_ctx **out);

/* Release the context (and its device memory if the library allocated it). */
lbm_status lbm_destroy(lbm_ctx *ctx);

/* Message of the last failed call on ctx ("" if none; a static message for
 * ctx == NULL). */
const char *lbm_last_error(const lbm_ctx *ctx);

/* Change the stream later work is enqueued on. */
lbm_status lbm_set_stream(lbm_ctx *ctx, void *stream);

/* Forest canopy (Sec. 2.3, Eq. forestForce; Algorithm 1): drag acceleration
 * a_d = -cd * lad[j] * |u*| * u*_x added to the x component of the body
 * force in every cell of row j with lad[j] > 0, where u* is the velocity with
 * the driving force only; vector_drag != 0 applies -cd*lad*|u*|*u* to all
 * three components.  lad: host array of ny values (1/cell), ny must equal
 * the context's ny.  Copied.  EINVAL for ny mismatch, NULL lad or a negative
 * or non-finite value. */
lbm_status lbm_set_canopy(lbm_ctx *ctx, double cd, const double *lad, int32_t ny,
                          int32_t vector_drag);

/* Heterogeneous forest (Sec. 3, the forest description before Algorithm 1,
 * alg:forestGASCANS, and that algorithm's set-up steps).  Forest code of a
 * cell (uint32, 0 = not forest):
 *   bits  0-9   h   height of the cell's forest object in cells (1..1023),
 *                   the rows spanned by its bounding box;
 *   bits 10-19  y   row of the cell minus the object's lowest row (< h);
 *   bits 20-31  q_m height of the LAD maximum, y_m = h * q_m / 4096.
 * Its LAD is afm * r^n * exp(n (1 - r)) of Eq. (af_theory) at y + 1/2, with
 * r = (h - y_m)/(h - y - 1/2), n = 6 below y_m and 1/2 above; constant_lad
 * != 0 gives afm in every forest cell (the constant-LAD case of Table
 * tab:forest_cases).
 *
 * lbm_forest_codes (host only): codes [nz][ny][nx] from a point cloud
 * points [npoints][3] (x, y, z in cell units, the domain is [0,nx) x [0,ny)
 * x [0,nz)).  A cell holding at least one point is a forest cell; an object
 * is a set of forest cells connected through faces, periodic in x and z;
 * q_m = round(4096 ym_frac).  nobjects (may be NULL) receives the object
 * count.  EINVAL for a point outside the domain or not finite, ym_frac
 * outside [0, 4095.5/4096), an object taller than 1023 rows, or NULL codes. */
lbm_status lbm_forest_codes(const double *points, int64_t npoints, int32_t nx, int32_t ny,
                            int32_t nz, double ym_frac, uint32_t *codes, int64_t *nobjects);

/* Use per-cell forest codes (host array [nz][ny][nx], copied) instead of the
 * per-row LAD of lbm_set_canopy, until the next lbm_set_canopy.  The drag is
 * that of lbm_set_canopy with the cell's LAD.  The library keeps a table of
 * the distinct codes' LAD (FP64) and a 16-bit table index per cell.  ESTATE if
 * the context was created without forest_map; EINVAL for NULL codes, a code
 * with y >= h, more than 65535 distinct codes, or a non-finite cd or afm. */
lbm_status lbm_set_forest(lbm_ctx *ctx, double cd, double afm, int32_t constant_lad,
                          const uint32_t *codes, int32_t vector_drag);

/* Eddy-viscosity closure.  LBM_CLOSURE_SMAG (blob ignored) restores Sec. 2.2.
 * LBM_CLOSURE_MLP loads a learned closure blob (host memory, nbytes == 10184,
 * format below) that replaces nu_t of Sec. 2.2 where its 9 input features lie
 * inside the stored ranges, and falls back to the Smagorinsky value elsewhere
 * (and in a cell whose hidden activations leave the FP16 range, |x| > 65504:
 * the device evaluates layer 1 with BF16 operands, the activations and
 * layer 2 in FP16, all accumulations in FP32).
 * EINVAL for a bad magic, version, shape or size.
 *
 * Blob (little-endian):
 *     0 char magic[4] "LBMC"; 4 u32 version 1; 8 u32 n_in 9, n_h1 64, n_h2 64, 0
 *    24 f32 mean[9], std[9], lo[9], hi[9]
 *   168 f32 out_scale s, canopy height h (cells), 0, 0
 *   184 f32 b1[64], b2[64], b3, 0, 0, 0
 *   712 bf16 W1[64][9], W2[64][64], w3[64]
 * Network: z = (x - mean)/std; h1 = gelu(W1 z + b1); h2 = gelu(W2 h1 + b2);
 * nu_t = s * softplus(w3.h2 + b3), gelu the tanh form.  Features, with
 * P = Pi_neq/(rho/3) and n = e_y: tr P, tr P^2, tr P^3, n.P.n, n.P^2.n,
 * sqrt(tr P^2), y_j/h, lad[j] (the cell's LAD with lbm_set_forest), 1.  Then
 * tau = tau0 + 3 nu_t. */
lbm_status lbm_set_closure(lbm_ctx *ctx, int32_t closure, const void *blob, size_t nbytes);

/* Evaluate the learned closure only on every `every`-th step (1 <= every <=
 * 1024; default 1 = every step) and let the steps in between reuse, cell by
 * cell, the nu_t of the last evaluation (kept in the context's moments
 * buffer).  A cost saving of this library, not of the paper: the steps in
 * between run at the speed of the Smagorinsky step.  The first step after
 * this call, lbm_set_closure, lbm_init or lbm_set_f evaluates.  The
 * diagnostics' mlp_fallback is the count of the last evaluation.  No effect
 * with the Smagorinsky closure.  EINVAL for every out of range. */
lbm_status lbm_set_closure_interval(lbm_ctx *ctx, int32_t every);

/* Initial state: f = feq(rho, u) (Sec. 2.1, Eq. local_eq) taken as the
 * post-collision populations at t = 0; resets t, the impulse and the
 * statistics.  rho: [nz][ny][nx], u: [3][nz][ny][nx], FP64.  The moments
 * read back before the first step are rho, u and nu_t = 0.  EINVAL for NULL. */
lbm_status lbm_init(lbm_ctx *ctx, const double *rho, const double *u, int32_t on_device);

/* Enqueue n >= 0 time steps, one fused kernel launch each, asynchronously
 * on the context's stream (a step that evaluates a learned closure whose y/h
 * range leaves out rows takes two or three launches, the rows outside it on
 * a second stream of the library's that the context's stream waits for; see
 * LBMX_MLP_SPLIT and LBMX_MLP_OVERLAP).
 * One step is the time loop body of Algorithm 1 (alg:forestGASCANS): stream
 * (Sec. 2.1, Eq. lbe; walls of Sec. 4 and Sec. 5.1), velocity (Eqs. density,
 * momentum), forest force and corrected velocity (Sec. 2.3, Eq.
 * forestForce), eddy viscosity (Sec. 2.2, Eqs. nu_t, strain and tau_total),
 * and the forced BGK collision (Eqs. bgk, local_eq, bodyforce), stored in
 * place.  The last step of the call also writes the moments (rho, u, nu_t)
 * and the per-wavefront FP64 diagnostics read by lbm_moments.  ESTATE before
 * lbm_init or after an instability was reported; EINVAL for n < 0. */
lbm_status lbm_step(lbm_ctx *ctx, int64_t n);

/* Synchronise the stream, then copy the moments of the latest step (FP64,
 * rho [N], u [3][N], nu_t [N]; any pointer may be NULL) and, if d != NULL,
 * the FP64 diagnostics (deterministic two-pass reductions).  rho and u are
 * the density and force-corrected velocity of Sec. 2.1 (Eqs. density,
 * momentum), nu_t the eddy viscosity of the step's closure (Sec. 2.2); the
 * mass and momentum are their FP64 sums over the cells.  EUNSTABLE (with
 * the outputs still written) if a non-finite value or max |u| > 0.35 is
 * found; later steps then return ESTATE until lbm_init or lbm_set_f. */
lbm_status lbm_moments(lbm_ctx *ctx, double *rho, double *u, double *nu_t, int32_t on_device,
                       lbm_diag *d);

/* Plane statistics (time and x-z averages, Sec. 4 and Sec. 5.2).
 * op 0 RESET: zero the sums.  op 1 ENABLE: sample after every step whose
 * new t is a multiple of every (every = 0 disables).  op 2 READ: synchronise
 * and write prof [ny][10] = means over samples and x-z of
 * u, v, w, uu, vv, ww, uv, uw, vw, nu_t.  nsamples (may be NULL) receives
 * the sample count. */
lbm_status lbm_stats(lbm_ctx *ctx, int32_t op, int32_t every, double *prof, int64_t *nsamples);

/* Overwrite the state with post-collision populations f [19][N] (FP64,
 * rounded into the storage type), stored in the slots the next step reads
 * (the in-place buffer's layout alternates between steps; t and that
 * alternation are unchanged, so a state saved with lbm_get_f and restored
 * continues bit for bit).  Clears an instability.  The moments read by
 * lbm_moments stay those of the latest step. */
lbm_status lbm_set_f(lbm_ctx *ctx, const double *f, int32_t on_device);

/* Read the current post-collision populations (decoded to FP64) [19][N];
 * synchronises the stream. */
lbm_status lbm_get_f(lbm_ctx *ctx, double *f, int32_t on_device);

/* Leaf-area density of Eq. (af_theory) at cell centres y_j = j + 1/2:
 * a(y) = afm * r^n * exp(n (1 - r)), r = (h - ym)/(h - y), n = 6 for y < ym,
 * 1/2 for ym <= y < h, 0 for y >= h.  With lai > 0 the profile is rescaled so
 * that sum_j a_j = lai (afm ignored).  Host only; out: ny values.  EINVAL for
 * h <= 0, ym outside [0, h), ny < 1 or NULL out. */
lbm_status lbm_lad_lalic(double h, double ym, double afm, double lai, int32_t ny, double *out);

/* ------------------------------------------------------------------------
 * Learned closure: training data and training (design of this library; the
 * paper names other SGS models as future work, Sec. 6).
 * ---------------------------------------------------------------------- */

/* Training samples from a run at twice the resolution.  `fine` must have
 * even nx, ny, nz and hold the moments of its latest step (lbm_step called).
 * The coarse grid is (nx/2, ny/2, nz/2).  For every coarse cell (FP32):
 *   - box-filtered velocity ub and the subfilter stress
 *     tau = box(u u) - ub ub + box(-2 nu_t^f S^f), S^f the fine strain rate by
 *     central differences of the fine velocity (one-sided next to y walls,
 *     periodic in x and z), in coarse lattice units (velocity unchanged);
 *   - the coarse strain Sb of ub by central differences on the coarse grid;
 *   - the target nu_t* = max(0, -tau_dev : Sb / (2 Sb : Sb)) (0 where Sb = 0);
 *   - the 9 closure features of the stress a coarse LBM would carry,
 *     P = -2 (tau0_coarse + 3 nu_t*) Sb: tr P, tr P^2, tr P^3, P_yy, (P^2)_yy,
 *     sqrt(tr P^2), (j + 1/2)/canopy_h, lad_coarse[j], 1.
 * X: device [nc][9], y: device [nc], nc = (nx/2)(ny/2)(nz/2) (cell order
 * [z][y][x]).  lad_coarse: host, ny/2 values.  EINVAL for odd dimensions, NULL
 * pointers or nc mismatch; ESTATE before lbm_init. */
lbm_status lbm_closure_samples(lbm_ctx *fine, double tau0_coarse, double canopy_h,
                               const double *lad_coarse, float *X, float *y, int64_t nc);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same
 * samples as lbm_closure_samples, bit for bit, with the work area (the
 * filtered velocity and subfilter stress, 9 FP32 per coarse cell, and the
 * coarse LAD) taken from a fixed device array of the library instead of
 * allocated per call.  That array holds LBM_NOALLOC_MAX_COARSE coarse cells
 * and LBM_NOALLOC_MAX_LAD coarse rows (about 9 MiB); each device the library
 * runs on keeps its own copy until the process ends.  The call allocates
 * nothing and does not synchronise: it enqueues a copy of lad_coarse (host,
 * ny/2 values, free to reuse on return) and two kernels on the context's
 * stream; X and y are ready when that stream is.  Every call on one device
 * shares the array, so calls that may overlap on one device (different
 * streams, host threads) race; calls on one stream are ordered.  Nothing in
 * the array needs clearing between calls.  Errors as lbm_closure_samples,
 * and EINVAL when the coarse grid exceeds either limit. */
#define LBM_NOALLOC_MAX_COARSE 262144
#define LBM_NOALLOC_MAX_LAD 4096
lbm_status lbm_closure_samples_noalloc(lbm_ctx *fine, double tau0_coarse, double canopy_h,
                                       const double *lad_coarse, float *X, float *y, int64_t nc);

typedef struct lbm_trainer lbm_trainer; /* opaque */

typedef struct lbm_train_params {
    float mean[9], std[9];   /* feature standardisation z = (x - mean)/std, std > 0 */
    float out_scale;         /* s: the network's softplus output is nu_t / s */
    float lr, beta1, beta2, eps; /* Adam */
    int32_t max_batch;       /* largest batch passed to lbm_train_step */
    void *stream;            /* hipStream_t or NULL */
} lbm_train_params;

/* A trainer for the 9-64-64-1 closure network: FP32 master parameters
 * (flat order W1[64][9], b1[64], W2[64][64], b2[64], w3[64], b3; 4865 values,
 * host array `params`, copied), Adam moments, BF16 MFMA fragments. */
lbm_status lbm_train_create(const lbm_train_params *prm, const float *params, lbm_trainer **out);

/* Gradient of L = (1/n) sum (softplus(o) - y/s)^2 over one batch (device X
 * [n][9] raw features, device y [n] target nu_t) with BF16 operands and FP32
 * accumulation on the matrix cores; with update != 0 one Adam step follows.
 * loss_out (host, may be NULL; synchronises) receives L.  EINVAL for n < 1 or
 * n > max_batch. */
lbm_status lbm_train_step(lbm_trainer *tr, const float *X, const float *y, int64_t n,
                          int32_t update, float *loss_out);

/* Copy the FP32 master parameters and/or the last gradient (host, 4865
 * values each; either may be NULL).  Synchronises. */
lbm_status lbm_train_get(lbm_trainer *tr, float *params, float *grad);

lbm_status lbm_train_destroy(lbm_trainer *tr);
const char *lbm_train_last_error(const lbm_trainer *tr);

#ifdef __cplusplus
}
#endif

#endif /* LBM_H */
