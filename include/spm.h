/*
 * spm.h - C ABI of the MI355X periodic Stokes mobility solver.
 *
 * Method: Wang, Nazockdast & Barnett, "An integral equation method for the
 * simulation of doubly-periodic suspensions of rigid bodies in a shearing viscous
 * flow" (arXiv:1912.04501). The library solves the quasi-static mobility problem
 * of Sec. 3 for rigid ellipses and smooth star-shaped particles in a sheared,
 * skewed unit cell through the completed second-kind BIE of Sec. 5 (eq. BIEPerturbed):
 *
 *     (1/2 I + K + L) sigma = -T(u0, p0) = -mu gamma (n_2, n_1),
 *
 * where K is the traction of the periodic single-layer potential, applied as a
 * 3x3 near-image sum (direct, or by a fast multipole method) + exterior barycentric
 * close correction + proxy-Stokeslet periodizing correction (Sec. 4.2, Sec. 6.1-6.3),
 * with the pressure pin of the Sec. 6.2 remark, and L the rigid-mode completion of Sec. 5.
 *
 * Conventions (all calls):
 *  - Lattice e1 = (1, 0), e2 = (s, 1) (Sec. 2, Sec. 7); the skew s is reduced to
 *    [-1/2, 1/2) internally (same lattice); the cell centre is c_U.
 *  - Angles are radians, counter-clockwise. Ellipse i is
 *    x(t) = c_i + R(theta_i) (a_i cos t, b_i sin t), nodes t_k = 2 pi k / N_i,
 *    particle-major: the nodes of particle 0 first.
 *  - Densities and node-vectors are SoA FP64: v[0..N-1] first components,
 *    v[N..2N-1] second components.
 *  - Background flow u0 = (gamma x_2, 0). Velocities are defined up to one constant
 *    per cell; they are reported in the gauge where the area-weighted mean of
 *    v_i - u0(c_i) over the cell's particles is zero (see spm_velocities); omega is
 *    gauge-free.
 *
 * Memory and streams: every array argument is a DEVICE pointer on the handle's
 * stream unless its name ends in _host. The caller owns all arrays; the library
 * only borrows them for the duration of the call and never frees them. The
 * handle owns its device workspace, which it obtains through the allocator
 * callbacks given to spm_create (or hipMalloc/hipFree when they are NULL). All
 * kernels run on the stream given to spm_create; calls return after that stream
 * has finished the call's work (so outputs are ready). A handle is not
 * thread-safe; distinct handles are independent.
 *
 * Errors: every call returns 0 on success or a negative SPM_E* code;
 * spm_last_error() returns a message for the last failure on that handle.
 * On error no output is guaranteed except where stated (SPM_ENOCONV).
 */
#ifndef SPM_H
#define SPM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define SPM_OK 0
#define SPM_EINVAL (-1)    /* bad argument (null pointer, size out of range, call order) */
#define SPM_EOVERLAP (-2)  /* particles overlap or come closer than cfg.min_gap */
#define SPM_ENOCONV (-3)   /* GMRES hit max_iter; outputs hold the last iterate */
#define SPM_EHIP (-4)      /* a HIP runtime call failed; message carries the HIP error */
#define SPM_ENOMEM (-5)    /* the allocator returned NULL */
#define SPM_ESTATE (-6)    /* call made before the lattice/particles were set */

#define SPM_FP64 0         /* every sum in FP64 */
#define SPM_FP32 1         /* near-image sum in FP32 with FP32 accumulation; the rest FP64 */
#define SPM_FP32_IR 2      /* solve: FP64 iterative refinement around FP32-near-sum GMRES */
#define SPM_FP32_RELAXED 3 /* solve: one FP64 GMRES whose operator products switch to the FP32
                              near sum once the residual estimate is below cfg.relax_tol */

#define SPM_X0_ZERO 0      /* initial guess of a solve without sigma0: zero */
#define SPM_X0_PREVIOUS 1  /* spm_step: the previous step's density (first step: zero) */
#define SPM_X0_NETWORK 2   /* the learned warm start of the network set by spm_set_network */

#define SPM_SHAPE_ELLIPSE 0  /* params (a, b, -, -): x(t) = (a cos t, b sin t) */
#define SPM_SHAPE_STAR 1     /* params (s, A, omega, phi): x(t) = r(t) (cos t, sin t),
                                r(t) = s (1 + A cos(omega t + phi)), |A| < 1, integer omega >= 0
                                (the smooth star-shaped curves of Sec. 8 Examples 2 and 4) */

#define SPM_NEAR_DIRECT 0  /* near-image sum: tiled direct N-body kernels (FP64 or FP32) */
#define SPM_NEAR_FMM 1     /* near-image sum: fast multipole method in FP64 (Sec. 6.2 remark: the
                              paper evaluates this sum with an FMM); single-cell handles, SPM_FP64 */

#define SPM_NEAR_SET_3X3 0      /* near images: the 3x3 lattice images of every whole particle (centres
                                   wrapped into the cell); proxies on a circle of radius R_proxy */
#define SPM_NEAR_SET_DILATED 1  /* the near set of Sec. 4.2 (definition of G_near): every node wrapped into the
                                   cell on its own, its images inside the dilated cell U~ (same centre,
                                   twice the side: four images per node); proxies on U~'s walls (Sec. 6.1
                                   remark), M/4 per side (M a multiple of 4). Direct near sums only;
                                   particles must stay within lattice distance 1/2 of their close
                                   neighbourhood (SPM_EINVAL at set-up otherwise); no contour mu_eff and no
                                   field evaluation */

#define SPM_PRECOND_NONE 0
#define SPM_PRECOND_BLOCK 1  /* right preconditioner blockdiag(B_q)^-1 of isolated-body self blocks
                                (particles of at most 512 nodes; SPM_EINVAL at the solve otherwise) */

typedef struct spm_handle spm_handle;
typedef struct spm_mlp spm_mlp;

/* Solver configuration; spm_default_config() fills the values in brackets. */
typedef struct {
  double mu;            /* viscosity [1] */
  double gamma;         /* shear rate [1] */
  int32_t M;            /* proxy Stokeslets on a circle about c_U [32] (Sec. 6.1) */
  double R_proxy;       /* proxy circle radius [1.5] */
  int32_t m_wall;       /* Gauss-Legendre collocation points per wall [24] (Sec. 6.1) */
  double close_factor;  /* close-evaluation threshold in node spacings [10] (Sec. 6.3 remark) */
  double tol;           /* relative residual of the solve [1e-10] */
  int32_t max_iter;     /* GMRES iteration cap per Krylov solve [500] */
  int32_t precision;    /* SPM_FP64, SPM_FP32_IR or SPM_FP32_RELAXED for spm_solve [SPM_FP64] */
  double inner_tol;     /* SPM_FP32_IR: relative tolerance of the first inner solve; 0 = 3e-3 with
                           the block preconditioner, 1e-4 without [0] */
  double min_gap;       /* reject geometries with a periodic boundary gap below this [0] */
  double rcond;         /* proxy pseudo-inverse relative cutoff [1e-14] */
  int32_t use_graph;    /* replay one captured GMRES iteration as a HIP graph [1] */
  int32_t poll_every;   /* GMRES iterations between convergence checks on the host [2] */
  int32_t x0;           /* SPM_X0_* initial guess when no sigma0 is given [SPM_X0_ZERO] */
  int32_t precond;      /* SPM_PRECOND_* [SPM_PRECOND_NONE] */
  int32_t learned_max_iter; /* iteration cap of a warm-started or preconditioned attempt before
                               the plain-GMRES fallback; 0 = max_iter [0] */
  double relax_tol;     /* SPM_FP32_RELAXED: residual estimate below which products use the FP32
                           near sum; 0 = adaptive: relax_safety * tol / delta32, delta32 the
                           relative error of the FP32 operator measured once per geometry (two
                           operator products), kept within [10 tol, 1e-2] [0] */
  int32_t near_method;  /* SPM_NEAR_DIRECT or SPM_NEAR_FMM [SPM_NEAR_DIRECT]; SPM_NEAR_FMM needs
                           precision SPM_FP64 (SPM_EINVAL at spm_create) and one cell (SPM_EINVAL
                           when more cells are set) */
  int32_t fmm_order;    /* SPM_NEAR_FMM: terms of each multipole and local expansion, 8..64;
                           0 = 40 (relative error of the near sum about 1e-14) [0] */
  double node_spacing;  /* node spacing h of the perimeter rule used when node counts are not
                           given: N_i = clamp(8 ceil(P_i / (8 h)), 64, 256), P_i the perimeter
                           [2.170590708293102e-3: about 5,000 nodes for 25 ellipses of aspect
                           ratio 1.5-3 at area fraction 0.3] */
  double relax_safety;  /* margin theta of the adaptive relaxed switch point, 0 < theta <= 1 [0.01] */
  double learned_accept;/* SPM_X0_NETWORK: a cell whose fitted network guess leaves a relative residual
                           above this starts from zero instead (acceptance test of the guess) [0.5] */
  int32_t near_set;     /* SPM_NEAR_SET_3X3 or SPM_NEAR_SET_DILATED [SPM_NEAR_SET_3X3]; with the dilated
                           set, M = 64, m_wall = 24 and rcond = 1e-8 are the measured choices */
} spm_config;

typedef struct {
  int32_t status;          /* 0 or SPM_ENOCONV */
  int32_t iterations;      /* total GMRES iterations (all inner solves for FP32_IR) */
  int32_t fp64_matvecs;
  int32_t fp32_matvecs;
  int32_t n_close_pairs;   /* (target, source image) pairs given the close correction */
  int32_t refinements;     /* outer iterations of FP32_IR (0 for FP64) */
  double rel_residual;     /* final ||b - A sigma|| / ||b|| with the FP64 operator */
  double seconds_setup;    /* geometry, proxy pseudo-inverse, close pairs */
  double seconds_solve;
  double seconds_readout;
  int32_t fallback;        /* 1 if the warm-started/preconditioned attempt failed and plain
                              GMRES (zero guess, no preconditioner) produced the result */
  int32_t first_iterations;/* iterations of that failed attempt (0 without fallback) */
  double min_gap;          /* smallest distance between nodes of different particles (any
                              images, every cell of the handle): the boundary gap to within
                              the node spacing; 1e300 when no two particles come within the
                              close-evaluation reach */
  int32_t guess_rejected;  /* SPM_X0_NETWORK: 1 if the fitted network guess left a residual above
                              cfg.learned_accept and the solve started from zero */
} spm_solve_info;

typedef void* (*spm_alloc_fn)(size_t bytes, void* stream, void* ctx);
typedef void (*spm_free_fn)(void* ptr, void* stream, void* ctx);

/* Fill cfg with the defaults listed in spm_config. */
void spm_default_config(spm_config* cfg);

/* Create a handle. stream: a hipStream_t (NULL = the null stream). alloc/free may
 * both be NULL (hipMalloc/hipFree). The config is copied. */
int spm_create(spm_handle** h, const spm_config* cfg, void* hip_stream,
               spm_alloc_fn alloc, spm_free_fn free_fn, void* alloc_ctx);
void spm_destroy(spm_handle* h);
const char* spm_last_error(const spm_handle* h);

/* Lattice (Sec. 2): e1 must be (1, 0) and e2 = (s, 1); s is reduced to
 * [-1/2, 1/2) (the nearest-integer shift of Sec. 7). center = c_U (may be NULL:
 * origin). Host pointers. Invalidates particles set before. */
int spm_set_lattice(spm_handle* h, const double e1_host[2], const double e2_host[2],
                    const double center_host[2]);

/* Ellipses (Sec. 2 geometry; Sec. 6 periodic trapezoid rule). Host arrays of
 * length n: centres [2n] (x0, y0, x1, y1, ...), theta, semi-axes a and b, node
 * counts (even, 8 <= N_i <= 4096; NULL: the perimeter rule of cfg.node_spacing).
 * Centres are wrapped into the cell. Builds
 * the nodes, the proxy pseudo-inverse and the close-pair list. Returns
 * SPM_EOVERLAP if two boundaries (any images) come within cfg.min_gap or
 * overlap. */
int spm_set_ellipses(spm_handle* h, int32_t n, const double* centers_host, const double* theta_host,
                     const double* a_host, const double* b_host, const int32_t* n_nodes_host);

int spm_num_nodes(const spm_handle* h, int64_t* N);
int spm_num_particles(const spm_handle* h, int32_t* n);

/* Node data (device arrays of length N each; any may be NULL). */
int spm_get_nodes(spm_handle* h, double* x, double* y, double* nx, double* ny, double* w);

/* Wrapped particle centres (host [2n]). */
int spm_get_centers(spm_handle* h, double* centers_host);

/* y = (1/2 I + K + L) sigma with the pressure pin (Sec. 5 eq. BIEPerturbed,
 * Sec. 6.2 pin). precision: SPM_FP64 or SPM_FP32 (near sum only). sigma, out: [2N]. */
int spm_apply(spm_handle* h, const double* sigma, double* out, int32_t precision);

/* Right-hand side b = -mu gamma (n_2, n_1) (Sec. 3, u0 = (gamma x_2, 0)). out [2N]. */
int spm_rhs(spm_handle* h, double* out);

/* Solve the completed BIE by GMRES (cfg.precision selects FP64 or FP32_IR) and
 * read out particle velocities vel [2n] (v_x0, v_y0, ...), angular velocities
 * omega [n] and mu_eff (device, one value per cell) - any of the three may be NULL.
 * sigma0 (may be NULL) is the initial guess; sigma [2N] receives the density.
 * info (host, may be NULL). Returns SPM_ENOCONV with the last iterate if GMRES
 * does not reach cfg.tol in cfg.max_iter iterations. */
int spm_solve(spm_handle* h, const double* sigma0, double* sigma, double* vel, double* omega,
              double* mu_eff, spm_solve_info* info_host);

/* Velocities and angular velocities of the rigid particles for a given density
 * (Sec. 3 eq. RigidBodyMotion, read at the centroids). vel [2n], omega [n]. The
 * velocity is defined up to one constant per cell; it is fixed so that the
 * area-weighted mean of v_i - u0(c_i) over the cell's particles is zero (a gauge that
 * does not depend on where the particles sit in the cell). */
int spm_velocities(spm_handle* h, const double* sigma, double* vel, double* omega);

/* Flow velocity and pressure at points x (Sec. 3; Sec. 5 representations of u and p; the
 * quasi-static solver of Sec. 7 returns u(x) and p(x)). sigma [2N] (device): a solved
 * density. xt, yt [n_targets] (device): any points (the disturbance is periodic; the
 * total velocity includes u0 = (gamma x_2, 0)). u [2 n_targets] (device): u_1 of every
 * target, then u_2, in the velocity gauge of spm_velocities. p [n_targets] (device): the
 * pressure of the representation (defined up to one constant), NaN inside particles,
 * where u is the particle's rigid motion. Points within close_factor * h of a curve use
 * the Laplace decomposition of the single layer with the barycentric rule of Sec. 6.3
 * (no slip is met to the discretisation error however close). With SPM_NEAR_FMM the
 * near-image sums at the points (and at the particle centres for the readout) come from
 * the FMM's quadtree instead of a direct sum over all images. Single-cell handles;
 * 0 <= n_targets <= 2^28. */
int spm_eval_field(spm_handle* h, const double* sigma, int64_t n_targets, const double* xt, const double* yt,
                   double* u, double* p);

/* Effective viscosity (Sec. 3 eq. mueff, evaluated by the particle-stresslet
 * identity; valid whether or not particles cross the wall D). mu_eff: device, one
 * value per cell. */
int spm_effective_viscosity(spm_handle* h, const double* sigma, double* mu_eff);

/* Effective viscosity by contour deformation (Sec. 7, efficient evaluation of the
 * effective viscosity), derived for this library's 3x3 near set: the shear force of
 * eq. mueff is carried from D to straight lines and segments that are about half a cell
 * or more from every source curve (D - e2, D + 2 e2 and four lattice-edge segments three
 * cells apart), plus the smooth proxy correction on D; valid whether or not particles
 * cross D. Gauss-Legendre with m nodes per cell edge (m = 0 selects 16; 4 <= m <= 128,
 * else SPM_EINVAL). sigma: device [2N] (SoA). mu_eff: device, one value per cell. */
int spm_effective_viscosity_contour(spm_handle* h, const double* sigma, int32_t m, double* mu_eff);

/* Forward Euler time stepping (Sec. 7) of a single-cell handle. t_inout (host): time on entry/exit;
 * the skew follows s(t) = s(0) + gamma t from the lattice set last plus the
 * elapsed time. centers_inout [2n], theta_inout [n] (host) hold the state;
 * mu_eff_series_host [n_steps] receives mu_eff(t_k); infos_host [n_steps] may be NULL.
 * The initial guess of every solve follows cfg.x0 (SPM_X0_PREVIOUS: the previous step's
 * density). If a step fails (SPM_EOVERLAP when particles collide or come closer than
 * cfg.min_gap, SPM_ENOCONV when GMRES does not converge), the state and *t_inout hold the
 * state that step was solving: (t_out - t_in) / dt steps were completed, their series
 * entries are set, and infos_host of the failing step holds its info after a solve. The
 * handle is then left without particles (SPM_ESTATE until particles and lattice are
 * given again). */
int spm_step(spm_handle* h, double dt, int32_t n_steps, double* t_inout, double* centers_inout_host,
             double* theta_inout_host, double* mu_eff_series_host, spm_solve_info* infos_host);

/* ---- stage entry points (each one step of the matvec, for checking) ---- */

/* Near-image traction sum T_near(x_i) = sum_j sum_{s in S9} G^t(x_i, y_j + s; n_i) w_j sigma_j,
 * self pair skipped (Sec. 4.2 G_near; 3x3 images per particle). out [2N]. */
int spm_near_traction(spm_handle* h, const double* sigma, double* out, int32_t precision);

/* With SPM_NEAR_FMM: the quadtree of the current geometry (levels below the root box, expansion
 * terms) and the work of one near sum (direct pairs of neighbouring leaves, multipole-to-local
 * translations). Host outputs, any may be NULL. SPM_ESTATE without an FMM plan. */
int spm_fmm_stats(spm_handle* h, int32_t* levels, int32_t* order, double* p2p_pairs, double* m2l_translations);

/* Close-evaluation correction Delta T (Sec. 6.3): barycentric traction minus the
 * plain near-sum terms over each close (target, source image) pair. out [2N].
 * precision selects which plain terms are subtracted (those of the FP64 or the
 * FP32 near sum). For SPM_FP32 it also holds the own-curve correction: the terms
 * between a target and the nodes of its own curve (zero shift) in FP64 minus the FP32
 * near sum's (FP32 coordinates cannot resolve those short, nearly tangent chords). */
int spm_close_correction(spm_handle* h, const double* sigma, double* out, int32_t precision);

/* Proxy strengths xi = Q^+ (g0 - g) (Sec. 6.2 steps 2-3). xi [2M] (device),
 * ordered all first components then all second components. */
int spm_proxy_strengths(spm_handle* h, const double* sigma, double* xi);

/* ---- allocation-free near sum ---- */

#define SPM_NOALLOC_MAX_N 131072   /* largest node count of spm_near_traction_noalloc */

/* For callers that cannot allocate device memory (code under HIP graph capture, serving loops
 * and harnesses that forbid hipMalloc): the near-image traction sum of spm_near_traction for
 * one cell given by its node arrays, with no handle and no allocation. Its forces, FP32 copies,
 * work plan and partial sums live in one file-scope device array of the library (about 16 MB
 * per GPU, kept until the process ends; its address is looked up once per device on the
 * first call, with that device current). Every call on a GPU shares that array: calls that
 * overlap on one GPU (other streams or threads) race and must be serialised by the caller.
 * Inputs (device, on hip_stream, NULL = the null stream): x, y, nx, ny, w [n] (nodes, outward
 * unit normals, quadrature weights, particle-major as spm_get_nodes returns them), sigma [2n]
 * (SoA density); skew: e2 = (skew, 1) of the cell (reduced to [-1/2, 1/2)); every node's 3x3
 * images m e1 + n e2 are sources, and only the node's own unshifted image is skipped (the
 * node list must hold each particle whole, centres wrapped as the handle wraps them).
 * precision SPM_FP64 or SPM_FP32 (FP32 pair sums, FP64 accumulation of the tiles). out [2n]
 * (device): T_near, SoA. Returns after the stream has finished. Errors (no message):
 * SPM_EINVAL for n < 1, n > SPM_NOALLOC_MAX_N, a NULL pointer, a non-finite skew or another
 * precision; SPM_EHIP when a HIP call fails. */
int spm_near_traction_noalloc(void* hip_stream, int64_t n, double skew, const double* x, const double* y,
                              const double* nx, const double* ny, const double* w, const double* sigma,
                              int32_t precision, double* out);

/* ---- ensembles of independent cells ---- */

/* Replace the contents of the handle by n_cells independent unit cells, solved
 * together (every kernel covers all cells; GMRES runs the cells in lockstep and
 * freezes each one at its own convergence). skews_host [n_cells]: e2 = (s_c, 1) of
 * each cell (reduced to [-1/2, 1/2)); part_offsets_host [n_cells + 1]: particles of
 * cell c are part_offsets[c] .. part_offsets[c+1]-1 of the particle arrays (as in
 * spm_set_ellipses; n_nodes_host may be NULL: the perimeter rule of cfg.node_spacing); every
 * cell is centred at the origin. 1 <= n_cells <= 1024. */
int spm_set_cells(spm_handle* h, int32_t n_cells, const double* skews_host, const int32_t* part_offsets_host,
                  const double* centers_host, const double* theta_host, const double* a_host,
                  const double* b_host, const int32_t* n_nodes_host);

/* As spm_set_cells for particles of any supported shape: kind_host [n] (SPM_SHAPE_*),
 * params_host [4n] (see SPM_SHAPE_*); the curve of particle i is c_i + R(theta_i) x(t),
 * t_k = 2 pi k / N_i, and its reference point c_i (inside the curve) carries the rigid
 * motion (velocity and angular velocity are read there). The largest radius must stay
 * below 0.45 (3x3 image rule). n_nodes_host may be NULL (the perimeter rule). */
int spm_set_cells_shapes(spm_handle* h, int32_t n_cells, const double* skews_host, const int32_t* part_offsets_host,
                         const double* centers_host, const double* theta_host, const int32_t* kind_host,
                         const double* params_host, const int32_t* n_nodes_host);

int spm_num_cells(const spm_handle* h, int32_t* n_cells);

/* Solve every cell set by spm_set_cells / spm_set_cells_shapes (as spm_solve). mu_eff:
 * device [n_cells]; infos_host [n_cells] (may be NULL); cell_latency_s_host [n_cells] (may
 * be NULL): seconds from the start of the solve to the moment the cell met the tolerance,
 * from the device wall clock. spm_solve on a handle with several cells behaves the same
 * without latencies. */
int spm_solve_cells(spm_handle* h, const double* sigma0, double* sigma, double* vel, double* omega, double* mu_eff,
                    spm_solve_info* infos_host, double* cell_latency_s_host);

/* One call for an ensemble of independent cells of ellipses (Sec. 3 problem per cell; the
 * quasi-static solver of Sec. 7 takes mu, gamma, e1, e2 and the boundaries and returns the
 * rigid motions): sets the cells (replacing the handle's contents, as spm_set_cells) and
 * solves them together in lockstep (as spm_solve_cells, zero initial guess or cfg.x0).
 * Host inputs: lattices_host [6 n_cells] = e1 (2), e2 (2), cell centre c_U (2) per cell, with
 * e1 = (1, 0) and e2 = (s, 1) (else SPM_EINVAL); part_offsets_host [n_cells + 1] (CSR:
 * particles of cell c are part_offsets[c] .. part_offsets[c+1]-1); centers_host [2n],
 * theta_host, semi_a_host, semi_b_host [n]; n_nodes_host [n] or NULL (the perimeter rule of
 * cfg.node_spacing). Device outputs (any may be NULL): vel [2n] (velocities of the wrapped
 * centres in the gauge of spm_velocities, u0 = (gamma x_2, 0) of the absolute position),
 * omega [n], mu_eff [n_cells]. Host outputs: infos_host [n_cells], cell_latency_s_host
 * [n_cells] (may be NULL). 1 <= n_cells <= 1024. The densities stay in the handle. */
int spm_solve_batch(spm_handle* h, int32_t n_cells, const double* lattices_host, const int32_t* part_offsets_host,
                    const double* centers_host, const double* theta_host, const double* semi_a_host,
                    const double* semi_b_host, const int32_t* n_nodes_host, double* vel, double* omega,
                    double* mu_eff, spm_solve_info* infos_host, double* cell_latency_s_host);

/* Number of close (target, source particle, shift) triples, and the triples
 * themselves (host arrays of length count, sorted by target, particle, shift;
 * shift index = 3 (m + 1) + (n + 1) for the image m e1 + n e2). */
int spm_close_pairs(spm_handle* h, int64_t* count, int32_t* target_host, int32_t* particle_host,
                    int32_t* shift_host, int64_t capacity);

/* The proxy least-squares pseudo-inverse Q^+ (host [n_cells * 2M * 8m], row-major per cell). */
int spm_proxy_pinv(spm_handle* h, double* pinv_host);

/* The proxy matrix Q (host [n_cells * 8m * 2M], row-major per cell), the singular
 * values of its Jacobi SVD (host [n_cells * 2M], unsorted, may be NULL) and the number
 * of Jacobi sweeps used (host [n_cells], may be NULL). */
int spm_proxy_svd(spm_handle* h, double* Q_host, double* s_host, int32_t* sweeps_host);

/* ---- launch shape of the near-image sum ---- */

/* Time candidate launch shapes of the persistent near-sum kernel (block 64/128/256
 * threads, 1/2/4 targets per lane, 128/256/512 sources per LDS tile) on the handle's
 * current geometry (all cells), for FP64 and FP32, and keep the fastest. cache_path (may
 * be NULL): text file of earlier results keyed by device, node count, cell count, pair work
 * and precision; a hit skips the timing, a miss appends. best_ms_host [2] (may be NULL):
 * the winning per-launch time (0 on a cache hit). The shape stays until the node count
 * changes. SPM_ESTATE on an SPM_NEAR_FMM handle, which plans no direct near-sum launches. */
int spm_autotune(spm_handle* h, const char* cache_path, double* best_ms_host);

/* Current near-sum launch shape {block, targets per lane, tile, workgroups per compute unit}
 * for precision SPM_FP64 or SPM_FP32 (host [4]). The kernel is persistent: its grid is
 * (workgroups per compute unit) x (compute units), where 0 selects the occupancy limit; the
 * work (target blocks of block x targets-per-lane nodes against source tiles of the same
 * cell) is divided evenly over that grid. spm_set_launch overrides it (SPM_EINVAL for an
 * unsupported shape: block 64, 128 or 256; 1, 2 or 4 targets per lane; 16 <= tile <= 1024;
 * 0 <= workgroups per compute unit <= 32). */
int spm_get_launch(spm_handle* h, int32_t precision, int32_t* cfg_host);
int spm_set_launch(spm_handle* h, int32_t precision, const int32_t* cfg_host);

/* ---- measurement ---- */

/* Enable (1) or disable (0) timing of the near-sum kernels with HIP events recorded
 * on the handle's stream around every launch; resets the counters. */
int spm_profile(spm_handle* h, int32_t enable);

/* Totals since spm_profile(h, 1): kernel 0 = FP64 near sum, 1 = FP32 near sum (pairs: node-image
 * pair evaluations, 9 N^2 per launch); with SPM_NEAR_FMM, 2 = the FMM's target evaluation kernel
 * (local expansions and the direct pairs of neighbouring leaves; pairs: those direct pairs) and
 * 3 = its multipole-to-local kernel (pairs: translations). total_ms: summed launch durations;
 * launches: number of launches. Any output may be NULL. Synchronises. */
int spm_profile_read(spm_handle* h, int32_t kernel, double* total_ms, int64_t* launches, double* pairs);

/* ---- block preconditioner ---- */

/* out = P^{-1} v with P = blockdiag(B_q): B_q is particle q's completed operator alone in
 * free space (sigma/2 + its own traction single layer with the smooth diagonal limit of
 * Sec. 6 + the rigid-mode completion L of Sec. 5; no pin, no images, no other particles).
 * The blocks are built and inverted (FP64 Gauss-Jordan, stored FP32) once per particle
 * shape (a, b, N_i) in the body frame and kept for later geometries with the same
 * shapes; each application rotates into the body frame and back. v, out [2N]. */
int spm_precond_apply(spm_handle* h, const double* v, double* out);

/* ---- learned warm start ---- */

#define SPM_MLP_IN 33          /* features per particle */
#define SPM_MLP_HIDDEN 256     /* width of the three hidden layers */
#define SPM_MLP_OUT 128        /* body-frame Fourier coefficients per particle (64 complex) */
#define SPM_MLP_NPARAMS 173184 /* W0[256x33] b0 W1[256x256] b1 W2[256x256] b2 W3[128x256] b3 */
#define SPM_MLP_BF16 0         /* matrix-core products in bfloat16, FP32 accumulation */
#define SPM_MLP_FP32 1         /* matrix-core products in FP32 (checking mode) */

/* Per-particle network inputs [n x 33] (device, bfloat16 bit patterns, nearest-even rounding
 * of the FP32 values of spm_features_f32; the network's first layer rounds its input to
 * bfloat16 in either form, so widening these to FP32 feeds spm_mlp_forward the same numbers). */
int spm_features(spm_handle* h, uint16_t* feat_bf16);

/* Per-particle features [n x 33] (FP32, device): for the 8 nearest other particle images
 * (3x3 images of the particle's own cell, its own images included, ordered by squared
 * centre distance, then particle, then shift index) the centre offset in the particle's
 * body frame divided by its semi-major axis and (cos, sin) of twice the angle
 * difference; then a/b. */
int spm_features_f32(spm_handle* h, float* features);

/* Training targets [n x 128] (FP32, device) of a density sigma [2N]: sigma minus its
 * cell-wide normal component beta* n (beta* = <sigma, n>/<n, n> per cell), rotated into
 * each particle's body frame, divided by mu gamma, as the discrete Fourier
 * coefficients c_m, m = -32..31 (real parts, then imaginary parts). Particles of at
 * most 512 nodes (SPM_EINVAL otherwise). */
int spm_density_modes(spm_handle* h, const double* sigma, float* modes);

/* Warm start from coefficients [n x 128] (device FP32): decode to the nodes (g), then per
 * cell sigma0 = alpha g + beta n with (alpha, beta) minimising |b - alpha A g - beta n/2|
 * (the completed operator maps n to n/2), so the guess never has a larger residual than
 * zero. sigma0 [2N] (device). One FP64 operator application. */
int spm_warm_start(spm_handle* h, const float* modes, double* sigma0);

/* Attach a network (borrowed: it must outlive its use; NULL detaches) for SPM_X0_NETWORK. */
int spm_set_network(spm_handle* h, spm_mlp* net);

/* features -> network (BF16) -> spm_warm_start. sigma0 [2N] (device). */
int spm_learned_guess(spm_handle* h, double* sigma0);

/* Forward Euler as spm_step, also recording for every step k the features and the
 * training targets of the solved density (device, [n_steps x n x 33] and
 * [n_steps x n x 128]; either may be NULL). */
int spm_step_record(spm_handle* h, double dt, int32_t n_steps, double* t_inout, double* centers_inout_host,
                    double* theta_inout_host, double* mu_eff_series_host, spm_solve_info* infos_host,
                    float* features, float* targets);

/* Network object (its own stream and allocator, as spm_create). Parameters start at zero;
 * set them with spm_mlp_set_params (which also resets the Adam state). */
int spm_mlp_create(spm_mlp** net, void* hip_stream, spm_alloc_fn alloc, spm_free_fn free_fn, void* alloc_ctx);
void spm_mlp_destroy(spm_mlp* net);
const char* spm_mlp_last_error(const spm_mlp* net);
int spm_mlp_set_params(spm_mlp* net, const float* params);   /* device [SPM_MLP_NPARAMS] */

/* Weights as a bfloat16 copy and/or an FP32 master copy (device, n_params == SPM_MLP_NPARAMS,
 * packed as for spm_mlp_set_params). The network keeps the FP32 master (Adam updates it);
 * in SPM_MLP_BF16 mode every layer product rounds its operands to bfloat16 (nearest even), so
 * the bfloat16 weights it multiplies are the rounding of the master (biases are added in FP32). master_fp32 NULL: the
 * master is params_bf16 widened (exact). Both given: params_bf16 must be the rounding of
 * master_fp32 (SPM_EINVAL otherwise). Resets the Adam moments. */
int spm_mlp_set_weights(spm_mlp* net, const uint16_t* params_bf16, const float* master_fp32, int64_t n_params);
int spm_mlp_get_params(spm_mlp* net, float* params);         /* device [SPM_MLP_NPARAMS] */

/* y [batch x 128] = MLP(x [batch x 33]) (device FP32, row-major). */
int spm_mlp_forward(spm_mlp* net, const float* x, int64_t batch, float* y, int32_t mode);

/* Loss (1/(2 batch)) sum |y - t|^2 (host) and its gradient with respect to the packed
 * parameters (device [SPM_MLP_NPARAMS], may be NULL). */
int spm_mlp_loss_grad(spm_mlp* net, const float* x, const float* t, int64_t batch, int32_t mode, float* grads,
                      double* loss_host);

/* Back-propagation of an upstream gradient: forward pass of x [batch x 33] (device FP32) in
 * mode, then grad [SPM_MLP_NPARAMS] (device, packed as the parameters) = d(sum_b dy_b . y_b)/d
 * params for dy [batch x 128] (device FP32) = dL/dy of the caller's loss. dy is only read. */
int spm_mlp_backward(spm_mlp* net, const float* x, const float* dy, int64_t batch, float* grad, int32_t mode);

/* One Adam step with bias correction on the FP32 master parameters: m <- beta1 m + (1 - beta1) g,
 * v <- beta2 v + (1 - beta2) g^2, p <- p - lr (m / (1 - beta1^step)) / (sqrt(v / (1 - beta2^step)) + eps).
 * grad [SPM_MLP_NPARAMS] (device). step >= 1 numbers the steps since the last set_params /
 * set_weights (which zero m and v); 0 <= beta < 1, lr > 0, eps > 0 (else SPM_EINVAL). */
int spm_mlp_adam_step(spm_mlp* net, const float* grad, float lr, float beta1, float beta2, float eps, int32_t step);

/* n_batches Adam steps (beta1 0.9, beta2 0.999, eps 1e-8, bias-corrected) on minibatches
 * of the n_samples rows of x [n_samples x 33] and t [n_samples x 128]: batch k uses the
 * rows idx[k batch .. (k+1) batch) (device int32; SPM_EINVAL if any is out of range).
 * losses (device [n_batches], may be NULL) receives each minibatch loss before its step. */
int spm_mlp_train(spm_mlp* net, const float* x, const float* t, int64_t n_samples, const int32_t* idx,
                  int32_t n_batches, int32_t batch, float lr, int32_t mode, float* losses);

#ifdef __cplusplus
}
#endif

#endif /* SPM_H */
