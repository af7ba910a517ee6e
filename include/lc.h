/*
 * lc.h -- C ABI of the MI355X (gfx950) long-characteristics transport sweep.
 *
 * The library computes the high-order transport step of the multilevel
 * quasidiffusion method with the method of long characteristics (Coale &
 * Anistratov, "Multilevel method for thermal radiative transfer problems with
 * method of long characteristics for the Boltzmann transport equation"):
 *   - the characteristic grid over a 2D orthogonal material grid
 *     (section "Method of Long Characteristics / Ray-Tracing Scheme":
 *     characteristic coordinates, segments between cell-boundary crossings,
 *     widths w_k, and the vertex-avoiding, width-halving construction given
 *     after eq. (16));
 *   - the backward-Euler sweep along every characteristic, eq. (10)-(13);
 *   - the cell-average moments E, F and Eddington tensor, eq. (7), (14)-(15),
 *     and boundary-face factors, eq. (16) and the "other linear-fractional
 *     factors" of the method section.
 *
 * Conventions used by every entry point
 * -------------------------------------
 * Material grid: nx x ny uniform cells on [0,lx] x [0,ly]; cell i = iy*nx+ix.
 * Boundary faces (nb = 2(nx+ny)): [0,ny) x=0 (row iy), [ny,2ny) x=lx,
 *   [2ny,2ny+nx) y=0 (column ix), [2ny+nx,nb) y=ly.
 * Quadrature: n_az azimuths phi[a] (n_az even, phi[a+n_az/2] = phi[a] + pi),
 *   n_pol polar cosines mu[p] (|mu| < 1), weights omega[m], direction
 *   m = a*n_pol + p, Omega_m = (sqrt(1-mu^2) cos phi, sqrt(1-mu^2) sin phi, mu).
 *   No azimuth may be parallel to a grid axis.
 * Azimuth pairs: pair a < n_az/2 holds azimuth a (d = 0, forward) and
 *   a + n_az/2 (d = 1, reverse); both share one family of characteristics.
 * Characteristics of pair a are ordered by v = -x sin(phi_a) + y cos(phi_a)
 *   ascending; global ray index k runs over pairs then rays; segments are
 *   stored in forward order; global segment index j runs over pairs, rays,
 *   segments.  Segment length l is the in-plane length; the path length in
 *   direction m is l / sqrt(1 - mu_p^2).
 * Groups: G >= 1; every [G][cells] input array is group-major; the moment
 *   outputs of lc_moments and lc_step are cell-major (group fastest).
 * Per-segment state (the previous step's segment-average intensities
 *   I_bar^{n-1}): an opaque caller-owned device buffer of lc_state_bytes()
 *   bytes; lc_state_export() gives it in the canonical order
 *   [j][d][p][g] as float64.
 * Exit intensities I_exit: float64 [n_rays][2][n_pol][G] (d = 0 leaves the
 *   forward traversal's end, d = 1 the reverse traversal's end).
 * Incoming boundary intensities I_in: float64 [nb][M][G]; only entries with
 *   Omega_m . n_b < 0 are read.
 *
 * Memory and errors
 * -----------------
 * Unless stated otherwise, array pointers are DEVICE pointers owned by the
 * caller; "stream" is a hipStream_t (NULL = default stream).  The library
 * owns only its opaque handles (and their device geometry and workspaces),
 * released by the matching *_free call.  lc_sweep, lc_moments and lc_step
 * allocate nothing and never synchronise the stream, so a caller may capture
 * them in a HIP graph.  Every entry point validates its arguments on the host
 * before launching anything and returns a status; no exception or abort
 * crosses the ABI.  lc_last_error() returns a thread-local description of the
 * last failure.  A device fault surfaces as LC_ERR_HIP from a later call.
 * Results are deterministic: no floating-point atomics are used.
 */
#ifndef LC_H
#define LC_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    LC_OK = 0,
    LC_ERR_ARG = 1,          /* invalid argument (null, size, range, layout) */
    LC_ERR_ALLOC = 2,        /* device or host allocation failed */
    LC_ERR_HIP = 3,          /* a HIP runtime call failed */
    LC_ERR_STATE = 4,        /* invalid handle or inconsistent internal state */
    LC_ERR_UNSUPPORTED = 5   /* valid request outside what this build supports */
} lc_status;

typedef enum { LC_RAYS_UNIFORM = 0, LC_RAYS_TUBES = 1 } lc_ray_mode;
typedef enum { LC_F64 = 0, LC_F32 = 1 } lc_prec;

typedef struct { int32_t nx, ny; double lx, ly; } lc_grid;

/* Host arrays: phi[n_az], mu[n_pol], omega[n_az*n_pol]. */
typedef struct {
    int32_t n_az, n_pol;
    const double* phi;
    const double* mu;
    const double* omega;
} lc_quad;

typedef struct {
    int64_t n_rays;          /* characteristics over all azimuth pairs */
    int64_t n_segments;      /* stored segments (each serves d = 0 and d = 1) */
    int32_t n_pairs, n_az, n_pol, n_cells, n_faces;
    int32_t max_seg_per_ray;
    int32_t mode;            /* lc_ray_mode */
    double h_moc;
} lc_rays_info_t;

typedef struct lc_rays_s* lc_rays_t;
typedef struct lc_plan_s* lc_plan_t;
typedef struct lc_batch_s* lc_batch_t;

/* Library version (major*10000 + minor*100 + patch). */
int32_t lc_version(void);

/* Thread-local text describing the last non-OK status returned on this
 * thread ("" if none).  Valid until the next failing call on the thread. */
const char* lc_last_error(void);

/*
 * Process-wide settings for testing and debugging.
 *
 * lc_set_alloc_limit -- every later device allocation of the library larger
 * than `bytes` fails (0: no limit, the default) as if the device were out of
 * memory: the call that needed it returns LC_ERR_ALLOC and frees whatever it
 * had allocated, so that error paths can be exercised on any GPU.
 *
 * lc_set_validation -- with enable != 0, lc_sweep, lc_sweep_points,
 * lc_sweep_noalloc and lc_step first check kappa, planck (all the steps'
 * values for lc_step) and I_in on the device for values that are not finite
 * or are negative, and return LC_ERR_ARG naming the array and the first such
 * index; this synchronises the stream.  Off by default (the checks cost a
 * pass over the inputs).  The batched calls are not checked.
 */
lc_status lc_set_alloc_limit(uint64_t bytes);
lc_status lc_set_validation(int32_t enable);

/*
 * lc_build_rays -- characteristic grid for every azimuth pair.
 * Paper: characteristic coordinates and segment lengths (section on the
 * method of long characteristics), segment area eq. (14), the construction of
 * the grid of characteristics after eq. (16), and the sets C(i,m) and F(f,m)
 * of eq. (15)-(16).
 *   mode LC_RAYS_UNIFORM: K = ceil(W/h_moc) characteristics of equal width
 *     delta = W/K tiling the projected width W, centrelines at
 *     v_min + (k+1/2) delta.
 *   mode LC_RAYS_TUBES: the paper's construction -- the gaps between the
 *     sorted projections of all grid vertices (no centreline crosses a
 *     vertex), each halved until no width exceeds h_moc.
 * Segments are cut at every grid-line crossing; crossings closer than
 * 1e-12*min(hx,hy) are merged (no zero-length segments).  A characteristic
 * entering or leaving through a domain corner belongs to the x = const face.
 * The device geometry (segments, cell-major segment lists with area weights,
 * boundary exit maps) lives in the returned handle; building synchronises
 * `stream`.  Errors: LC_ERR_ARG for null pointers, nx/ny < 1, non-positive
 * sizes or h_moc, odd n_az, unpaired azimuths, |mu| >= 1, axis-parallel
 * azimuths, or a spacing so coarse that some cell is crossed by no
 * characteristic of some direction; LC_ERR_ALLOC; LC_ERR_HIP.
 */
lc_status lc_build_rays(const lc_grid* grid, const lc_quad* quad, double h_moc,
                        int32_t mode, void* stream, lc_rays_t* out);
lc_status lc_rays_free(lc_rays_t rays);
lc_status lc_rays_info(lc_rays_t rays, lc_rays_info_t* info);

/*
 * lc_rays_export -- copy the geometry to HOST arrays (any may be NULL):
 * ray_off[n_pairs+1] (first global ray of each pair), seg_off[n_rays+1]
 * (first global segment of each ray), cell[n_segments], len[n_segments],
 * width[n_rays], face[n_rays][2] (entry and exit face of the forward
 * traversal).  Synchronous.
 */
lc_status lc_rays_export(lc_rays_t rays, int32_t* ray_off, int32_t* seg_off,
                         int32_t* cell, double* len, double* width, int32_t* face);

/*
 * lc_plan_create -- per-(geometry, G, precision) workspace: the cell
 * coefficient table (modified opacity kappa_t = kappa + 1/(c dt), emission
 * kappa B / kappa_t, and 1/(c dt kappa_t) of eq. (11)) and, for LC_F32, the
 * per-group power-of-two scale of the stored intensities.  prec LC_F64 sweeps
 * and stores in float64; LC_F32 sweeps and stores in float32 with
 * compensated float32 moment sums and float64 division and boundary factors.
 * The plan keeps a reference to `rays`, which must outlive it.  Errors:
 * LC_ERR_ARG for G outside 1..4096 or an unknown precision; LC_ERR_UNSUPPORTED
 * when the state would hold 2^32 or more lane records (a lane record is the
 * n_pol values of one (segment, traversal, group)), the limit of the moment
 * gather's 32-bit offsets; LC_ERR_ALLOC; LC_ERR_HIP.
 */
lc_status lc_plan_create(lc_rays_t rays, int32_t G, int32_t prec, lc_plan_t* out);
lc_status lc_plan_free(lc_plan_t plan);

/* Bytes of one per-segment state buffer of `plan` (a 256-byte header, then
 * n_segments*2*n_pol*G values of the plan's precision). */
size_t lc_state_bytes(lc_plan_t plan);

/*
 * lc_state_fill -- initial condition of eq. (2) for the state: every segment
 * and direction takes the value of the cell field it lies in,
 * state[j][d][p][g] = field[g][cell(j)].  field: float64 [G][cells].
 */
lc_status lc_state_fill(lc_plan_t plan, const double* field, void* state, void* stream);

/* lc_state_export -- state in canonical order, float64 [n_segments][2][n_pol][G]. */
lc_status lc_state_export(lc_plan_t plan, const void* state, double* out, void* stream);

/*
 * lc_state_import -- the inverse of lc_state_export: fill a state buffer
 * from finite float64 values in the canonical order [n_segments][2][n_pol][G]
 * (resuming a run from an exported state, or moving a state between
 * precisions).  LC_F64 plans store the values as they are; LC_F32 plans
 * take each group's power-of-two scale from its largest magnitude and store
 * the exactly rescaled values rounded to float32.  Uses the plan's
 * group-maximum workspace, so order it with the plan's sweeps on one stream.
 * Errors: LC_ERR_ARG (NULL), LC_ERR_UNSUPPORTED (more than 2^31 x 1024
 * value rows), LC_ERR_HIP.
 */
lc_status lc_state_import(lc_plan_t plan, const double* in, void* state, void* stream);

/*
 * lc_sweep -- one backward-Euler transport sweep, eq. (10)-(13), over every
 * characteristic, direction and group:
 *   kappa_t = kappa + 1/(c dt),  Q = kappa B + I_bar^{n-1}/(c dt),
 *   tau = kappa_t l / sin(zeta),  I_out = I e^{-tau} + (Q/kappa_t)(1 - e^{-tau}),
 *   alpha = 1/tau - e^{-tau}/(1 - e^{-tau}),  I_bar = alpha I + (1 - alpha) I_out.
 * kappa, planck: float64 [G][cells] (kappa > 0 or 0, planck >= 0, finite);
 * c_dt > 0; state_prev -> state_new (distinct buffers of lc_state_bytes);
 * I_in: float64 [nb][M][G]; I_exit: float64 [n_rays][2][n_pol][G] or NULL.
 * The intensity entering a characteristic is I_in of the face it enters
 * through.  Errors: LC_ERR_ARG (null or aliased buffers, c_dt <= 0),
 * LC_ERR_HIP.
 */
lc_status lc_sweep(lc_plan_t plan, const double* kappa, const double* planck, double c_dt,
                   const void* state_prev, void* state_new, const double* I_in,
                   double* I_exit, void* stream);

/*
 * lc_sweep_noalloc -- lc_sweep for callers that cannot allocate device memory
 * while they sweep: code under HIP graph capture, tight serving loops,
 * harnesses that forbid hipMalloc.  Same arguments, results (bit for bit)
 * and errors as lc_sweep, except that
 *   - the sweep's scratch -- the cell coefficient table (cells x G records
 *     of 8 bytes for LC_F32 or 16 for LC_F64, rounded up to 256 bytes) and
 *     the float32 per-group maxima (2 G values of 8 bytes) -- lives in a
 *     static device array of 64 MiB, which the library holds on every device
 *     it runs on until the process ends, instead of the plan's workspace;
 *   - it always sweeps whole traversals (a plan's split setting is not
 *     used) and records no timing events;
 *   - it calls no allocating routine (the first call on a device looks up
 *     the array's address there).
 * Every call on a device shares that device's array, and each call
 * rewrites (and clears) what it reads, so calls ordered on one stream are
 * safe; calls that overlap on one device (other streams, other threads)
 * race and must not be made.  Errors: as lc_sweep, plus LC_ERR_ARG when the
 * plan's scratch exceeds the array (256^2 cells x 51 groups fit in either
 * precision, 512^2 x 51 does not), LC_ERR_HIP when the address lookup fails.
 */
lc_status lc_sweep_noalloc(lc_plan_t plan, const double* kappa, const double* planck, double c_dt,
                           const void* state_prev, void* state_new, const double* I_in,
                           double* I_exit, void* stream);

/*
 * lc_moments -- cell and boundary moments of a swept state, eq. (7),
 * (14)-(16).  For each cell i and direction m the area-weighted mean
 *   I_{i,m} = sum_{C(i,m)} A I_bar / sum_{C(i,m)} A,  A = l w,
 * then Phi = sum_m omega_m I_{i,m}, E = Phi/c, F = sum_m omega_m Omega_m I_{i,m},
 * f = sum_m omega_m Omega_m Omega_m I_{i,m} / Phi (f := 1/3 on the diagonal
 * where Phi = 0).  Outputs (float64, any may be NULL):
 *   E[cells][G], F[cells][2][G] (x, y), f[cells][4][G] (xx, xy, yy, zz),
 *   bnd[G][nb][8] = Phi+, J+, Phi-, J-, C = J+/Phi+, f_xx, f_xy, f_yy of the
 *   boundary face (outgoing: width-weighted mean exit intensity of the
 *   characteristics leaving through the face, or of the one leaving nearest
 *   its centre if none does; incoming: I_in).  bnd needs I_exit and I_in.
 * c > 0 is the speed of light in the caller's units.  Errors: LC_ERR_ARG
 * (null state, c not finite or <= 0, bnd without I_exit and I_in),
 * LC_ERR_HIP.
 */
lc_status lc_moments(lc_plan_t plan, const void* state, const double* I_exit,
                     const double* I_in, double c, double* E, double* F, double* f,
                     double* bnd, void* stream);

/*
 * Interior faces, eq. (16): the face-average moments on every interior face
 * of the material grid, from the intensities at the faces' crossings with
 * the characteristics (I_{k,s} at the upwind face of each segment).
 *
 * lc_plan_enable_faces -- build the interior-face crossing lists F(f, m)
 * (kept with the characteristic grid, shared by its plans) and this plan's
 * records of them.  Allocates; synchronises `stream`.  A crossing is where
 * two consecutive segments lie in cells that share a face; a passage
 * through a vertex (diagonal neighbours) crosses no face interior and is
 * left out.  Faces: x-faces (x = ix hx, 1 <= ix < nx) of row iy are numbered
 * iy (nx - 1) + ix - 1, then y-faces (y = iy hy, 1 <= iy < ny) of column ix
 * follow at (nx - 1) ny + (iy - 1) nx + ix.  Errors: LC_ERR_ALLOC,
 * LC_ERR_STATE (crossings that do not form contiguous runs), LC_ERR_HIP.
 *
 * lc_sweep_points -- lc_sweep that also stores, in `points` (a buffer of
 * lc_state_bytes, same layout as the state), the intensity entering every
 * segment in each traversal.  Same results in state_new and I_exit as
 * lc_sweep.  Errors as lc_sweep, and LC_ERR_ARG for a NULL or aliased
 * points buffer.
 *
 * lc_face_moments -- per interior face f and group: the width-weighted mean
 * of the crossing intensities of each direction, I_{f,m} = sum w_k I / sum
 * w_k over F(f, m) (read per direction, as for the boundary faces; a
 * direction with no crossing contributes nothing), then E_f = sum_m omega_m
 * I_{f,m} / c, F_f = sum_m omega_m Omega_m I_{f,m}, f_f = sum_m omega_m
 * Omega_m Omega_m I_{f,m} / (c E_f) (1/3 on the diagonal where E_f = 0).
 * points: as written by lc_sweep_points; state: the state_new of that sweep
 * (its header holds the scale of the stored values).  Outputs (float64, any
 * may be NULL), face-major like lc_moments: E[faces][G], F[faces][2][G],
 * f[faces][4][G], faces = (nx - 1) ny + nx (ny - 1).  Needs
 * lc_plan_enable_faces (LC_ERR_STATE otherwise); LC_ERR_ARG for NULL
 * points/state or c <= 0.
 */
lc_status lc_plan_enable_faces(lc_plan_t plan, void* stream);
lc_status lc_sweep_points(lc_plan_t plan, const double* kappa, const double* planck, double c_dt,
                          const void* state_prev, void* state_new, const double* I_in, double* I_exit,
                          void* points, void* stream);
lc_status lc_face_moments(lc_plan_t plan, const void* points, const void* state, double c, double* E, double* F,
                          double* f, void* stream);

/*
 * lc_grey_closures -- cell-local closures of the effective grey problem,
 * eq. (8)-(9), from the multigroup cell moments of this plan (as written by
 * lc_moments or lc_step) and the opacity and Planck source of the step:
 *   out[13][cells] = E, F_x, F_y (sums over the groups), <kappa>_E,
 *   <kappa>_B, K_R,xx = <kappa>_|F_x|, K_R,yy = <kappa>_|F_y|, eta_x, eta_y,
 *   <f>_E (xx, xy, yy, zz), where
 *   <u>_E = sum_g u_g E_g / sum_g E_g,  <u>_B = sum_g u_g B_g / sum_g B_g
 *   (the mean that closes the emission term of eq. (5a) when a_R T^4 is read
 *   as (4 pi / c) sum_g B_g), <u>_|F_a| = sum_g u_g |F_a,g| / sum_g |F_a,g|,
 *   eta_a = sum_g (kappa_g - K_R,aa) F_a,g / sum_g E_g, <f>_E =
 *   sum_g f_g E_g / sum_g E_g; the group sums are deterministic (a fixed
 *   order over the groups, the same in every call).
 *   A zero denominator takes a fallback: <kappa>_E -> <kappa>_B -> the mean
 *   of kappa_g over the groups; <kappa>_B and <kappa>_|F_a| -> <kappa>_E;
 *   with sum E = 0, eta = 0 and <f>_E = 1/3 on the diagonal.
 * E, F, f: float64 in the cell-major layout of lc_moments; kappa, planck:
 * float64 [G][cells]; out: float64, caller-owned.  Allocates nothing.
 * Errors: LC_ERR_ARG (null pointer), LC_ERR_HIP.
 */
lc_status lc_grey_closures(lc_plan_t plan, const double* E, const double* F, const double* f,
                           const double* kappa, const double* planck, double* out, void* stream);
/* The same with explicit sizes, for moments gathered from several plans (for
 * instance groups swept on characteristic grids of their own): E, F, f in the
 * cell-major layout of lc_moments over all G groups.  LC_ERR_ARG for cells or
 * G < 1 or a NULL pointer. */
lc_status lc_grey_closures_dims(int32_t cells, int32_t G, const double* E, const double* F, const double* f,
                                const double* kappa, const double* planck, double* out, void* stream);

/*
 * Low-order quasidiffusion (LOQD) equations.  Multigroup, eq. (4), for one
 * backward-Euler time step on the material grid, closed by the Eddington
 * tensors of the transport sweep (cells: eq. (7), (15); faces: eq. (16))
 * and its half-range boundary factors.  Time-discrete, with
 * kappa_t = kappa + 1/(c dt):
 *   c kappa_t E + div F = 4 pi kappa B + E^{n-1}/dt,
 *   kappa_t F + c div(f E) = F^{n-1}/(c dt).
 * The paper cites its second-order finite-volume scheme without printing
 * it; the scheme here: unknowns are the cell averages E_i and the face
 * averages E_f of every group; the balance is integrated over each cell;
 * the first moment over each half cell next to a face, with kappa_t F taken
 * at the face, the cell tensor times E_i at the centre, the face tensor
 * times E_f on the face and the cell's transverse face averages for the
 * mixed term; an interior face has one normal flux; a boundary face closes
 * with n.F = C (c E_f - Phi^-) - J^- (C, Phi^-, J^- from the boundary
 * factors).  Faces are numbered as for lc_face_moments (interior x-faces,
 * then interior y-faces), followed by the boundary faces in their own order
 * (nf = (nx-1) ny + nx (ny-1) + 2 (nx + ny)); normal fluxes are the x
 * component on x-faces and the y component on y-faces.
 *
 * lc_loqd_create -- solver handle for an nx x ny grid on [0,lx] x [0,ly]
 * and G groups; holds the face structure and the solver's workspace
 * (about (22 G + 11) nf + (6 G + 4) nx ny doubles).  Errors: LC_ERR_ARG,
 * LC_ERR_ALLOC, LC_ERR_HIP.
 *
 * lc_loqd_solve -- one step for every group.  Inputs (device, float64):
 * kappa, planck, E_prev [G][cells]; F_prev [G][nf]; f_cell [cells][4][G]
 * (the layout lc_moments writes); f_face [interior faces][4][G] (the layout
 * lc_face_moments writes; may be NULL on a grid without interior faces);
 * bnd [G][nb][8] (the layout lc_moments writes: C in column 4, Phi^- in 2,
 * J^- in 3, the face tensor in 5-7).  Outputs: E_cell [G][cells], E_face
 * [G][nf], F_face [G][nf].  The cell unknowns are eliminated exactly (the
 * mixed terms cancel in each cell balance, so a cell row holds its own four
 * faces only) and the face system of every group is solved by BiCGSTAB
 * with a Jacobi preconditioner, all groups at once, to a relative residual
 * rtol of the face system (its true residual is checked when the recursive
 * one reaches rtol, up to three times); inner products are fixed-order
 * reductions, so results are deterministic.  Face systems of up to 16384
 * faces run the whole iteration in one launch, one workgroup per group;
 * larger ones one launch per vector operation (lc_loqd_set_solver chooses
 * explicitly).  The iteration starts from zero, or from E_face's contents
 * after lc_loqd_set_warm_start.  iters (host, may be NULL) receives the
 * iterations run (the most of any group); resid (host [G], may be NULL)
 * each group's final relative residual.
 * Synchronises `stream` (convergence checks), so it cannot be captured in a
 * graph.  Errors: LC_ERR_ARG (NULL inputs or outputs, c or c_dt not finite
 * or <= 0, rtol outside (0, 1), max_iter < 1), LC_ERR_STATE (invalid
 * handle), LC_ERR_UNSUPPORTED (some group above rtol after max_iter
 * iterations; the outputs then hold the last iterate), LC_ERR_HIP.
 */
typedef struct lc_loqd_s* lc_loqd_t;
lc_status lc_loqd_create(int32_t nx, int32_t ny, double lx, double ly, int32_t G, lc_loqd_t* out);
lc_status lc_loqd_free(lc_loqd_t loqd);
lc_status lc_loqd_solve(lc_loqd_t loqd, double c, double c_dt, const double* kappa, const double* planck,
                        const double* E_prev, const double* F_prev, const double* f_cell,
                        const double* f_face, const double* bnd, double* E_cell, double* E_face,
                        double* F_face, double rtol, int32_t max_iter, int32_t* iters, double* resid,
                        void* stream);

/*
 * The same scheme in general form, for the effective grey equations of
 * eq. (5) (and any system of this shape): per group (G of the handle),
 *   sigma_i E_i + (F_R - F_L)/hx + (F_T - F_B)/hy = source_i,
 *   k (h/2) F_f = -c ((f E)_high - (f E)_low) - c h/(2 h_t) (mixed term)
 *                 - (h/2) eta E_f + (h/2) F^{n-1}_f / (c dt)
 * on each half cell, with k and eta given per cell and side.  Eq. (4) is
 * sigma = c kappa_t, source = 4 pi kappa B + c E^{n-1}/(c dt), k = kappa_t,
 * eta = 0.
 *
 * lc_loqd_solve_general -- inputs (device, float64): sigma, source
 * [G][cells]; k_side, eta_side [G][4][cells] (sides L, R, B, T of each
 * cell); F_prev [G][nf]; f_cell [G][3][cells] and f_face [G][3][nf]
 * (xx, xy, yy); bc [G][nb][3] (C, Phi^-, J^-).  Outputs, solver, iters,
 * resid, synchronisation and errors as lc_loqd_solve.
 *
 * lc_loqd_grey_coefficients -- the grey equations' coefficients (G = 1
 * arrays of the general form, and E^{n-1} = sum_g E^{n-1}_g) from a
 * multigroup solution on the handle's grid (the handle's G groups): the
 * multigroup inputs of lc_loqd_solve and its outputs E_cell, E_face,
 * F_face.  Paper: eq. (5) closed by the spectrum averages of eq. (8)-(9),
 * taken where the scheme uses them so that the two schemes are
 * algebraically consistent (summed over the groups, the multigroup
 * equations are the grey ones, and the grey solution is the sum of the
 * group solutions):
 *   sigma = c (<kappa>_E + 1/(c dt)), source = 4 pi <kappa>_B sum_g B_g +
 *     c E^{n-1}/(c dt) (a_R T^4 read as (4 pi / c) sum_g B_g) per cell;
 *   per cell side: K_R = sum_g kappa_g |F_g,f| / sum_g |F_g,f| (normal face
 *     fluxes), k = K_R + 1/(c dt), eta = sum_g (kappa_g - K_R) F_g,f / E_f
 *     with the face's grey E;
 *   <f>_E of cells with cell energies, of faces with face energies;
 *   boundary: C = sum_g C_g E_g,f / E_f, Phi^- = 0,
 *     J^- = sum_g (C_g Phi^-_g + J^-_g).
 * Zero denominators: <kappa>_E -> <kappa>_B -> mean kappa_g; K_R ->
 * <kappa>_E; eta = 0; <f> = 1/3 on the diagonal; C -> mean C_g.  Sums over
 * the groups run in a fixed order.  Outputs (device, float64): sigma,
 * source, E_prev_grey [cells]; k_side, eta_side [4][cells]; F_prev_grey
 * [nf]; f_cell_grey [3][cells]; f_face_grey [3][nf]; bc_grey [nb][3];
 * kappa_E, kappa_B [cells] (<kappa>_E and <kappa>_B, the inputs of
 * lc_loqd_grey_meb; either may be NULL).
 * Allocates and synchronises nothing.  Errors: LC_ERR_ARG (NULL, c or c_dt
 * not finite or <= 0), LC_ERR_STATE, LC_ERR_HIP.
 */
lc_status lc_loqd_solve_general(lc_loqd_t loqd, double c, double c_dt, const double* sigma,
                                const double* source, const double* k_side, const double* eta_side,
                                const double* F_prev, const double* f_cell, const double* f_face,
                                const double* bc, double* E_cell, double* E_face, double* F_face,
                                double rtol, int32_t max_iter, int32_t* iters, double* resid,
                                void* stream);
lc_status lc_loqd_grey_coefficients(lc_loqd_t loqd, double c, double c_dt, const double* kappa,
                                    const double* planck, const double* E_prev, const double* F_prev,
                                    const double* f_cell, const double* f_face, const double* bnd,
                                    const double* E_cell, const double* E_face, const double* F_face,
                                    double* sigma, double* source, double* k_side, double* eta_side,
                                    double* F_prev_grey, double* f_cell_grey, double* f_face_grey,
                                    double* bc_grey, double* E_prev_grey, double* kappa_E,
                                    double* kappa_B, void* stream);

/*
 * lc_loqd_grey_meb -- the effective grey problem of one backward-Euler step:
 * the grey equations, eq. (5), coupled to the grey material energy balance,
 * eq. (6), with material energy eps = c_v T (the paper's test material),
 *   c_v (T - T^{n-1}) / dt = c <kappa>_E E - c <kappa>_B a_R T^4,
 *   c (<kappa>_E + 1/(c dt)) E + div F = c <kappa>_B a_R T^4 + E^{n-1}/dt,
 * with the spectrum averages and the other grey coefficients held fixed
 * (the outputs of lc_loqd_grey_coefficients).  Newton iteration on T:
 * a_R T^4 is linearised about the iterate T_k, the energy balance then gives
 * T = alpha + beta E per cell, the grey equations with the resulting
 * absorption and source are solved as lc_loqd_solve_general does, and T is
 * updated, until max over cells of |T_{k+1} - T_k| / |T_{k+1}| <= newton_tol.
 * The handle's G is the number of independent grey problems (normally 1);
 * every array carries a leading [G] axis over the layouts of
 * lc_loqd_solve_general: kappa_E, kappa_B, E_prev, T_prev [G][cells];
 * k_side, eta_side [G][4][cells]; F_prev [G][nf]; f_cell [G][3][cells];
 * f_face [G][3][nf]; bc [G][nb][3] (device, float64).  T [G][cells]
 * (device, in/out): the first iterate on entry (T_prev is the usual
 * choice), the converged temperature on return.  Outputs E_cell [G][cells],
 * E_face, F_face [G][nf] as lc_loqd_solve_general.  c_v (energy per volume
 * and temperature) and a_R > 0 in the units of E and T.  Each inner solve
 * runs to rtol within max_iter iterations; newton_iters (may be NULL)
 * receives the Newton iterations, iters (may be NULL) the BiCGSTAB
 * iterations summed over them, resid (may be NULL, [G]) the last inner
 * solve's relative residuals.  Uses the handle's coefficient buffers
 * (sigma, source) and synchronises the stream every iteration.  Errors:
 * LC_ERR_ARG (NULL, c, c_dt, c_v or a_R not finite or <= 0, newton_tol < 0,
 * max_newton or max_iter < 1, rtol outside (0, 1)), LC_ERR_STATE,
 * LC_ERR_UNSUPPORTED (an inner solve or the Newton iteration did not
 * converge; the outputs then hold the last iterate), LC_ERR_HIP.
 */
lc_status lc_loqd_grey_meb(lc_loqd_t loqd, double c, double c_dt, const double* kappa_E,
                           const double* kappa_B, const double* E_prev, const double* k_side,
                           const double* eta_side, const double* F_prev, const double* f_cell,
                           const double* f_face, const double* bc, const double* T_prev, double c_v,
                           double a_R, double* T, double* E_cell, double* E_face, double* F_face,
                           double newton_tol, int32_t max_newton, double rtol, int32_t max_iter,
                           int32_t* newton_iters, int32_t* iters, double* resid, void* stream);

/*
 * lc_loqd_set_warm_start -- with enable != 0, every later solve on the
 * handle (lc_loqd_solve, lc_loqd_solve_general and each Newton iteration
 * of lc_loqd_grey_meb) starts BiCGSTAB from the current contents of its
 * E_face output (which must then hold finite values) instead of zero; the
 * solution is the same within rtol, reached in fewer iterations when the
 * system changed little since the last solve.  Errors: LC_ERR_STATE.
 */
lc_status lc_loqd_set_warm_start(lc_loqd_t loqd, int32_t enable);

/*
 * lc_loqd_set_solver -- how the handle's BiCGSTAB runs: 0 (default) by
 * size, 1 one workgroup per group running the whole iteration in one
 * launch (face systems up to 16384 faces, the default there: no host round
 * trips; larger systems run as 2), 2 grids of blocks per vector operation
 * with the host testing convergence every 8 iterations (the default above
 * 16384 faces).  The two
 * iterate alike and differ only in the order of their sums, so their
 * solutions agree within rtol.  Errors: LC_ERR_ARG, LC_ERR_STATE.
 */
lc_status lc_loqd_set_solver(lc_loqd_t loqd, int32_t mode);

/*
 * Multilevel quasidiffusion (MLQD) time steps on the Fleck-Cummings test
 * material of the paper's results section: opacity 27/nu^3 (1 - e^(-nu/T))
 * at each group's representative frequency nu_g, material energy
 * eps = c_v T.  One step composes the paper's three levels:
 *   1. the transport sweep (eq. (10)-(13)) from the state of step n-1 with
 *      kappa_g, B_g of the current temperature, giving the cell and face
 *      Eddington tensors and the boundary factors;
 *   2. the multigroup LOQD equations, eq. (4), closed by them;
 *   3. the effective grey problem, eq. (5)-(6), closed by the spectrum
 *      averages of eq. (8)-(9),
 * iterated: an outer (transport) iteration s forms the closures with the
 * material of T^(s); inner (low-order) iterations, closures fixed,
 * evaluate kappa_g, B_g at the temperature T and solve 2. then 3. for
 * Phi(T), until max_i |Phi(T)_i - T_i| / Phi(T)_i <= eps or max_inner
 * passes, the next T from Anderson mixing of the last passes on log T
 * (depth set by lc_mlqd_set_acceleration, default 3; it changes the
 * iteration's speed, not its fixed point); the step ends when, between
 * transport sweeps, the
 * temperature changes by at most eps (relative, every cell) and the grey
 * cell energy by at most eps (max |dE| / max |E|).  T^(0) = T^{n-1}.
 * B_g(T) = (a_R c T^4 / 4 pi)(15/pi^4) int over [nu_{g-1}/T, nu_g/T] of
 * x^3/(e^x - 1) dx (per steradian, the 4 pi kappa B of eq. (4a)).
 *
 * lc_mlqd_create -- for a float64 plan (its grid, quadrature,
 * characteristic grid and G; interior-face lists are enabled on it, as
 * lc_plan_enable_faces; a float32 plan is refused with LC_ERR_UNSUPPORTED,
 * since the iterations converge far below the float32 sweep's rounding):
 * nu [G] (host, keV, > 0) the opacity frequencies; edges [G + 1] (host,
 * keV, increasing, edges[0] >= 0, only edges[G] may be +infinity: with 0
 * and infinity the groups sum to a_R c T^4 / 4 pi); c, c_v, a_R > 0 in the
 * units of the rest (c_v: energy per volume and temperature).  Allocates
 * the step's work buffers (a state-sized buffer for the face crossings,
 * the closures, two LOQD handles with warm starts, the grey coefficients)
 * and synchronises the device.  Errors: LC_ERR_ARG, LC_ERR_STATE,
 * LC_ERR_ALLOC, LC_ERR_HIP.
 *
 * lc_mlqd_set_acceleration -- Anderson depth of the inner iteration,
 * 0 (plain fixed-point passes) to 8.  Errors: LC_ERR_ARG, LC_ERR_STATE.
 *
 * lc_mlqd_material -- kappa_g(T), B_g(T) [G][cells] (device, float64) for
 * T [cells] (device, > 0), as the step evaluates them.  Allocates and
 * synchronises nothing.
 *
 * lc_mlqd_step -- one time step of c_dt (> 0).  Inputs (device): the
 * transport state of step n-1 (state_prev; state_new receives the last
 * sweep's, distinct buffers of lc_state_bytes), I_in [nb][M][G] as for
 * lc_sweep, T_prev [cells], E_prev [G][cells] and F_prev [G][nf] (the
 * multigroup low-order solution of step n-1; face numbering of
 * lc_loqd_solve).  Outputs (device, float64): T [cells]; the multigroup
 * E_cell [G][cells], E_face, F_face [G][nf] of the last inner iteration
 * (the next step's E_prev and F_prev: use other buffers); E_grey [cells]
 * (may be NULL) the grey cell energy.  outer_iters, inner_iters (total),
 * changes [2] (the last dT, dE) may be NULL.  Inner solves: BiCGSTAB to a
 * relative residual of 1e-3 times the last change, within [1e-13, 1e-8]
 * (the pass that ends the inner iteration at 1e-13), Newton to
 * max(min(eps, 1e-11), 1e-13).  eps much below 1e-12 may not be reachable in
 * float64.  The low-order solves of a step start cold and there are no
 * floating-point atomics, so a step's results depend on its arguments alone
 * (the same bits on every call).  Synchronises the stream many times.
 * Errors: LC_ERR_ARG (NULL, aliased states, c_dt or eps not finite or
 * <= 0, max_outer or max_inner < 1), LC_ERR_STATE, LC_ERR_UNSUPPORTED (an
 * inner solve failed, or the step did not converge within max_outer
 * transport iterations: the outputs then hold the last iterates),
 * LC_ERR_HIP.
 */
typedef struct lc_mlqd_s* lc_mlqd_t;
lc_status lc_mlqd_create(lc_plan_t plan, const double* nu, const double* edges, double c, double c_v,
                         double a_R, lc_mlqd_t* out);
lc_status lc_mlqd_free(lc_mlqd_t mlqd);
lc_status lc_mlqd_set_acceleration(lc_mlqd_t mlqd, int32_t depth);
lc_status lc_mlqd_material(lc_mlqd_t mlqd, const double* T, double* kappa, double* planck, void* stream);
lc_status lc_mlqd_step(lc_mlqd_t mlqd, double c_dt, const void* state_prev, void* state_new,
                       const double* I_in, const double* T_prev, const double* E_prev,
                       const double* F_prev, double* T, double* E_cell, double* E_face, double* F_face,
                       double* E_grey, double eps, int32_t max_outer, int32_t max_inner,
                       int32_t* outer_iters, int32_t* inner_iters, double* changes, void* stream);

/*
 * lc_step -- n_steps backward-Euler time steps (sweep, then moments) with the
 * state ping-ponging between state_a and state_b: step t reads the state
 * written by step t-1 (step 0 reads state_a); after an odd number of steps
 * the newest state is in state_b, after an even number in state_a.
 * kappa/planck of step t start at kappa + t*material_stride (elements; 0
 * means the same data every step).  Every step forms its moments (as
 * lc_moments; any output may be NULL); E, F, f, bnd hold those of the last
 * step.  The step sequence is captured once in a HIP graph per argument set
 * and replayed.  Errors: LC_ERR_ARG (n_steps < 1; null kappa, planck, states
 * or I_in; state_a == state_b; material_stride < 0; c_dt or c not finite or
 * <= 0; bnd without I_exit), LC_ERR_ALLOC, LC_ERR_HIP.
 */
lc_status lc_step(lc_plan_t plan, int32_t n_steps, const double* kappa, const double* planck,
                  int64_t material_stride, double c_dt, double c, void* state_a, void* state_b,
                  const double* I_in, double* I_exit, double* E, double* F, double* f,
                  double* bnd, void* stream);

/*
 * Launch tuning of a plan (chosen by the project's autotuner; any value works,
 * results are bit-identical across settings of moments_entries and
 * sweep_unroll).  sweep_unroll: steps of a characteristic whose loads are
 * in flight ahead of the arithmetic, 1, 2, 4, 8 or 16 (16: LC_F32 plans with
 * n_pol <= 4 only); moments_entries: entries of each (cell,
 * azimuth pair) list whose loads go through the moment kernel's pipeline, 1 to
 * 4 (longer lists finish in a plain loop).  Setting the tuning synchronises the
 * device and drops the plan's captured graphs.
 * Errors: LC_ERR_ARG for a null tuning or a value outside those sets (the
 * plan keeps its previous tuning).
 */
typedef struct {
    int32_t sweep_unroll;
    int32_t moments_entries;
} lc_tuning_t;
lc_status lc_plan_set_tuning(lc_plan_t plan, const lc_tuning_t* tuning);
lc_status lc_plan_get_tuning(lc_plan_t plan, lc_tuning_t* tuning);

/*
 * Residency of the whole-traversal sweep of a plan.  capped = 1 (the
 * default): every sweep block reserves a third of a CU's LDS, so at most two
 * blocks (two wavefronts per SIMD) stay resident -- the streams of large
 * problems are served better by the caches that way; capped = 0: residency
 * is set by the kernel's registers alone, which shortens the tail of small
 * problems.  Results are bit-identical either way.  Batches keep the cap.
 * Synchronises the device and drops the plan's captured graphs.  Errors:
 * LC_ERR_ARG for a value other than 0 or 1.
 */
lc_status lc_plan_set_sweep_residency(lc_plan_t plan, int32_t capped);

/*
 * Split sweep (in-ray parallel scan), for problems with few lanes and long
 * characteristics.  The step of eq. (12) is affine in the intensity entering
 * a segment, so a traversal cut into chunks of chunk_steps steps maps the
 * intensity entering each chunk onto the one leaving it as I -> A I + B.
 * With chunk_steps > 0, every following lc_sweep and lc_step of the plan runs
 * three launches: one wavefront per (traversal of a bundle, chunk) forms
 * the chunk's map (the first chunk from the true boundary intensity), a scan
 * composes the maps along each traversal, and one wavefront per chunk sweeps
 * it from its entering intensity, writing the state rows and, at the last
 * chunk, the exit intensities.  The first two chunks of a traversal round
 * exactly as the whole-traversal sweep; later ones differ from it by
 * rounding only.  The plan holds the work lists and a transfer buffer of
 * (chunks - 1 per traversal) * n_pol * 64 value pairs of its precision.
 * chunk_steps = 0 turns it off (the default).  lc_sweep_points and batched
 * steps always sweep whole traversals.  Synchronises the device and drops
 * the plan's captured graphs.  Errors: LC_ERR_ARG for a chunk_steps that is
 * negative, not a multiple of 4 or above 2^24; LC_ERR_UNSUPPORTED for a work
 * list beyond 2^31 blocks; LC_ERR_ALLOC (the plan is then left with the
 * split turned off); LC_ERR_HIP.
 */
lc_status lc_plan_set_split(lc_plan_t plan, int32_t chunk_steps);

/*
 * Gathers split over azimuth pairs, for plans whose (cell, group) lanes are
 * too few to fill the device while every C(i, m) list is long (a fine
 * characteristic grid over a coarse material grid, as in the refinement
 * studies of the numerical-results section).  The moments of eq. (7),
 * (14)-(16) sum, per (cell or interior face, group), the direction averages
 * of every azimuth pair; split, one lane per (pair, cell, group) sums its
 * pair's list and stores the pair's seven partial sums, and a second launch
 * adds them in pair order.  The boundary factors split the same way, one
 * lane per ((pair, traversal), boundary face, group) summing the exit
 * intensities, the combining launch forming the factors.  Both forms add the
 * same terms in the same order, so results are bit-identical either way.
 * mode: 1 splits the cell and face gathers and the boundary factors, 0 runs
 * them whole, -1 (the default at lc_plan_create) chooses per gather: the
 * moments split when the plan's tiles hold fewer than 2048 wavefronts and
 * the lists average at least 8 entries, the boundary factors when
 * nb * G < 16384, or nb * G < 131072 and at least 8 characteristics per
 * (face, pair) exit.  A
 * split plan holds a device buffer of n_pairs * 7 * (its largest gather
 * grid's lanes) values of its precision, or 2 n_pairs (n_pol + 1) nb G
 * doubles if larger.  Batched steps always run whole gathers.
 * lc_plan_get_moment_split returns the forms in use (bit 0: moments, bit 1:
 * boundary factors).  Setting synchronises the device and drops the plan's
 * captured graphs.  Errors: LC_ERR_ARG for a mode outside -1..1;
 * LC_ERR_ALLOC (the plan is then left with whole gathers); LC_ERR_HIP.
 */
lc_status lc_plan_set_moment_split(lc_plan_t plan, int32_t mode);
lc_status lc_plan_get_moment_split(lc_plan_t plan, int32_t* mode);

/*
 * Kernel timers (tracing).  lc_plan_profile(plan, 1) makes every following
 * eager lc_sweep / lc_moments record HIP events around its main kernel on the
 * caller's stream (not inside lc_step graphs; around all three launches of
 * a split sweep); lc_plan_profile_read synchronises those events and
 * returns, in out[4]: total milliseconds and count of the recorded sweeps,
 * then of the cell-moment launches; it also clears the record.
 * lc_plan_profile(plan, 0) stops recording.
 */
lc_status lc_plan_profile(lc_plan_t plan, int32_t enable);
lc_status lc_plan_profile_read(lc_plan_t plan, double* out);

/*
 * Batched form: many independent problems (each its own rays and plan)
 * advanced together.  Problems are grouped by polar bound (the power of two
 * >= n_pol) and by sweep form (mirror-symmetric polar sets of power-of-two
 * size run a sweep without per-angle branches, as in their single-problem
 * runs, so batched results equal those runs bit for bit); per group, the
 * sweep and the cell moments are one launch each
 * over all members, with the launch tuning of the plan of the group's
 * lowest-index member.  lc_batch_create copies the per-problem pointer sets
 * (device arrays as for lc_step) into the handle and builds work lists
 * ordered by decreasing cost; lc_batch_step then runs n_steps time steps of
 * every problem (state ping-pong as lc_step; step t reads material data at
 * kappa + t * material_stride, so with a non-zero stride n_steps must not
 * exceed the steps the caller provides); every step forms each problem's
 * moments, and the outputs hold those of the last step.  The incoming
 * intensities I_in are the same for every step of a call (their float32
 * scale maxima are taken at its first step); they may change between calls.
 * A call whose c differs from the previous call's rewrites the moment and
 * boundary argument records, and first synchronises the device (a step
 * launched earlier may still read them); calls with an unchanged c do not
 * synchronise.  The captured step graph runs the moments of step t on a
 * second stream beside the sweep of step t + 1 and joins it before the call
 * returns its work to the caller's stream.
 * All problems must share one precision.  I_exit is required.  Errors of
 * lc_batch_create:
 * LC_ERR_ARG (no problems; a problem without kappa, planck, states, I_in or
 * I_exit; state_a == state_b; c_dt not finite or <= 0; material_stride < 0;
 * mixed precisions), LC_ERR_STATE (an invalid plan), LC_ERR_UNSUPPORTED
 * (work lists beyond 32-bit indexing), LC_ERR_ALLOC, LC_ERR_HIP.  Errors of
 * lc_batch_step: LC_ERR_ARG (n_steps < 1, c not finite or <= 0),
 * LC_ERR_STATE (a member's plan freed), LC_ERR_HIP.
 */
typedef struct {
    lc_plan_t plan;
    const double* kappa;
    const double* planck;
    int64_t material_stride;
    double c_dt;
    void* state_a;
    void* state_b;
    const double* I_in;
    double* I_exit;          /* required */
    double* E;
    double* F;
    double* f;
    double* bnd;
} lc_problem_t;

lc_status lc_batch_create(int32_t n_problems, const lc_problem_t* problems, lc_batch_t* out);
lc_status lc_batch_step(lc_batch_t batch, int32_t n_steps, double c, void* stream);
lc_status lc_batch_free(lc_batch_t batch);

/* Kernel timers of a batch: with lc_batch_profile(batch, 1), lc_batch_step runs
 * its steps without a graph and records HIP events around the prologue, the
 * sweep launches and the moment launches of each step; lc_batch_profile_read
 * synchronises them and returns out[6] = total ms and launch count of each, in
 * that order, clearing the record. */
lc_status lc_batch_profile(lc_batch_t batch, int32_t enable);
lc_status lc_batch_profile_read(lc_batch_t batch, double* out);

#ifdef __cplusplus
}
#endif
#endif /* LC_H */
