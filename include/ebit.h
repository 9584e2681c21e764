/*
 * ebit.h -- C ABI of the MI355X (gfx950) library for the interface-aware
 * elliptic steps of the EBIT phase-change method (Long, Pan & Zaleski,
 * "A Front-Tracking approach for phase change: the EBIT method").
 *
 * The library implements, on a uniform Cartesian grid (2D or 3D):
 *   ebit_build_coeffs  EBIT edge markers + colour vertices -> interface facets,
 *                      cut fractions theta on grid links, cell flags and the
 *                      multigrid hierarchies of both elliptic operators
 *                      (Sec. 2.1; theta of Eq. ghost_T)
 *   ebit_heat_solve    implicit per-phase diffusion with T = T_sat imposed
 *                      sharply at theta (Eqs. energy_diffusion, ghost_T,
 *                      Txx_ghost), solved by geometric multigrid
 *   ebit_mass_flux     mass flux from one-sided normal temperature gradients
 *                      (Eqs. mass_flux_computation, normal_gradient)
 *   ebit_project       ghost velocities from the mass-flux jump (Eq.
 *                      ghost_velocity), the variable-density Poisson problem
 *                      (Eqs. Poisson_equation, poisson_ghost_fluid) solved by
 *                      geometric multigrid, and the face-velocity update
 *   ebit_ghost_band    the ghost velocities of Eq. ghost_velocity on every
 *                      narrow-band face, from the band-extended mass flux
 *   ebit_volume_fraction
 *                      the liquid volume fraction of every cell from the
 *                      EBIT segments (2D)
 *   ebit_interface_velocity, ebit_advect_markers
 *                      the interfacial velocity (Eq. jump_interfacial_vel)
 *                      and the EBIT marker motion of one time step (Sec. 2.1)
 *   ebit_advect_energy the advection step of the energy equation (Eq.
 *                      energy_advection): explicit Euler, WENO3 derivatives
 *
 * Conventions (all calls):
 *   - Every array argument is a DEVICE pointer owned by the caller, contiguous,
 *     x fastest: cell (i,j,k) is at i + nx*(j + ny*k).  A 2D grid has n[2] = 1.
 *       cells             nx*ny*nz
 *       vertices          (nx+1)*(ny+1)*nvz          nvz = nz+1 (3D), 1 (2D)
 *       axis-a edges      vertex layout with one fewer entry along a
 *                         (edge from vertex v to v + e_a)
 *       axis-a faces      cell layout with one more entry along a
 *                         (face index i_a separates cells i_a - 1 and i_a)
 *   - Colours: 1 = liquid, 0 = vapour.  Markers: fractional position
 *     s in [0, 1] along the edge from its lower vertex; NaN = no marker.
 *   - Domain sides are ordered (-x, +x, -y, +y, -z, +z).
 *   - Work is enqueued on the stream given to ebit_create (a hipStream_t
 *     passed as void*).  Calls that fill an ebit_stats (or return a solver
 *     status) synchronise that stream before returning; ebit_build_coeffs
 *     synchronises to report geometry errors.
 *   - The library never allocates device memory: the caller passes one
 *     workspace of ebit_workspace_bytes() bytes to ebit_create and keeps it
 *     alive until ebit_destroy.  The library never frees caller memory.
 *   - No exception crosses the ABI.  Every call returns an ebit_status;
 *     ebit_status_string() gives a static text; ebit_last_error() gives the
 *     text of the last failure on a context (HIP error strings included).
 *   - Calls on one context must not overlap (one stream, one workspace).
 *   - Environment: EBIT_WIDE_OFFSETS=1, read when a context or batch is
 *     created, makes the outer-loop kernels use 64-bit cell offsets at any
 *     grid size (the form they take from 2^30 cells on); results are the
 *     same bits.  It exists to test that form on small grids.
 *     EBIT_TEST_FP32_STALL=1, read the same way, makes a mixed-precision
 *     context or batch treat every solve still iterating after its first
 *     block of iterations as stalled, to test the FP64 fallback.
 *     EBIT_SOLVE_LOG=<path>, read when a context is created, appends one
 *     JSON line per ebit_heat_solve, ebit_project and ebit_project_one_fluid
 *     call of that context to the file (call, dim, n, precision, and the
 *     fields of ebit_stats); those calls then always wait for the device,
 *     as with a stats argument.  A file that cannot be opened is skipped.
 */
#ifndef EBIT_H
#define EBIT_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define EBIT_MAX_LEVELS 24

typedef enum {
  EBIT_OK = 0,
  EBIT_EINVAL = -1,   /* bad argument; nothing was launched                    */
  EBIT_ENOMEM = -2,   /* workspace smaller than ebit_workspace_bytes()         */
  EBIT_EGEOM = -3,    /* markers inconsistent with colours, or a cut link with
                         no interface cell on either side                      */
  EBIT_ENOCONV = -4,  /* max_iters reached; the best iterate is returned       */
  EBIT_ENAN = -5,     /* NaN/Inf met in a residual norm                        */
  EBIT_EHIP = -6,     /* a HIP call failed (sticky on the context)             */
  EBIT_ESTATE = -7,   /* call order violated (e.g. solve before build_coeffs)  */
  EBIT_EIO = -8       /* the schedule cache file could not be written          */
} ebit_status;

typedef enum { EBIT_BC_NEUMANN = 0, EBIT_BC_DIRICHLET = 1, EBIT_BC_PERIODIC = 2 } ebit_bc;
typedef enum { EBIT_FP64 = 0, EBIT_MIXED = 1 } ebit_precision;
typedef enum { EBIT_OUTER_PCG = 0, EBIT_OUTER_DC = 1 } ebit_outer;
typedef enum { EBIT_SYS_HEAT = 0, EBIT_SYS_PRESSURE = 1 } ebit_system;

/* Grid and boundary conditions.  Periodic sides come in pairs and apply to
 * both T and p; a periodic axis needs n_a = 2^m (the red-black multigrid
 * keeps an even size on every level).  Heat: Dirichlet sides impose T_val
 * through the face ghost 2 T_w - T_c; Neumann sides are insulated.
 * Pressure: Dirichlet (outflow) sides impose p = p_val on the face; Neumann
 * sides are walls (no flux, face velocity left as given). */
typedef struct {
  int dim;          /* 2 or 3                                                */
  int n[3];         /* cells per axis, each >= 3 (n[2] = 1 in 2D)             */
  double h;         /* uniform spacing                                       */
  int T_bc[6];      /* ebit_bc per side                                      */
  double T_val[6];
  int p_bc[6];
  double p_val[6];
} ebit_grid;

/* Phase properties (index l = liquid, v = vapour) and saturation data. */
typedef struct {
  double rho_l, rho_v, lam_l, lam_v, cp_l, cp_v, h_lg, T_sat;
} ebit_props;

/* Solver options; ebit_default_opts() fills the defaults in brackets. */
typedef struct {
  int precision;      /* EBIT_FP64 [default] or EBIT_MIXED (FP32 V-cycles
                         inside the FP64 outer loop; a solve whose V-cycles
                         stop contracting, above the rounding floor and
                         before max_iters, continues in FP64 from its
                         iterate: ebit_stats.fp64_fallback)                   */
  int outer;          /* EBIT_OUTER_PCG [default]: flexible CG preconditioned
                         by one V-cycle; EBIT_OUTER_DC: defect correction
                         x += alpha V(b - A x) with the energy-optimal step
                         alpha = (r.z)/(z.Az)                                 */
  double rtol;        /* relative L2 residual ||b - A x|| / ||b|| [1e-9]; a
                         target below the residual's rounding floor stops
                         at the floor (ebit_stats.res_floor)                  */
  int max_iters;      /* outer iterations [200]                               */
  int nu1, nu2;       /* red-black Gauss-Seidel sweeps before / after the
                         coarse correction, 1..8 each [2, 2]                  */
  double theta_min;   /* lower clamp of theta in the 1/theta terms [1e-3]     */
  int check_every;    /* outer iterations per block between host checks [1]:
                         a block is captured once as a hipGraph and replayed;
                         a case that meets its stop level inside a block
                         skips the rest of it on the device, so results do
                         not depend on this value, only the host round trips.
                         The first block of a solve runs as many iterations
                         as the previous solve of the same system took.     */
  int tail_cells;     /* levels with at most this many cells (and that fit
                         the work-group's LDS) are solved by one work-group
                         kernel; the coarsest level always is [4096]          */
} ebit_opts;

typedef struct {
  int iters;            /* outer iterations                                  */
  int vcycles;          /* V-cycles applied                                   */
  double rel_res;       /* final relative residual (recomputed, not recursive)*/
  double bnorm;         /* ||b||_2                                            */
  double res_floor;     /* rounding floor of rel_res: 4 (dim+1) eps
                           || |b| + |A||x| || / ||b||; a solve also counts as
                           converged once rel_res <= res_floor                */
  double seconds;       /* device time of the call (hipEvent)                 */
  double div_max;       /* ebit_project: max_c |div_c u_{k(c)}| after update  */
  int fallbacks;        /* ebit_mass_flux: first-order gradient fallbacks     */
  int status;           /* ebit_status of the call                            */
  int fp64_fallback;    /* 1 if a mixed-precision solve stalled (its FP32
                           V-cycles stopped contracting the FP64 residual)
                           and was continued in FP64 from its iterate       */
} ebit_stats;

typedef struct ebit_ctx ebit_ctx;

void ebit_default_opts(ebit_opts* opts);
const char* ebit_status_string(ebit_status s);

/* Bytes of device workspace a context on this grid needs.  Returns 0 for an
 * invalid grid. */
size_t ebit_workspace_bytes(const ebit_grid* grid, const ebit_opts* opts);

/* Create a context.  workspace: device memory of at least
 * ebit_workspace_bytes(grid, opts) bytes, 256-byte aligned, owned by the
 * caller.  hip_stream: the hipStream_t all work is enqueued on (NULL = the
 * null stream).  Returns EBIT_EINVAL for a bad grid / props / opts and
 * EBIT_ENOMEM if bytes is too small. */
ebit_status ebit_create(ebit_ctx** ctx, const ebit_grid* grid, const ebit_props* props,
                        const ebit_opts* opts, void* workspace, size_t bytes, void* hip_stream);
ebit_status ebit_destroy(ebit_ctx* ctx);
const char* ebit_last_error(const ebit_ctx* ctx);

/* Sec. 2.1 and Eq. ghost_T.  marker[a] (a < dim): axis-a edge array of s or
 * NaN; vertex_colour, cell_colour: uint8 colours.  Computes each interface
 * cell's facet (centroid = mean of its markers, unit normal from vapour into
 * liquid), theta on every cut link (fraction of the link from its lower cell
 * to the interface), the cell flags, and both multigrid hierarchies for the
 * time step dt.  Returns EBIT_EGEOM if a marker sits on an edge whose end
 * colours agree (or is missing where they differ), a marker is outside
 * [0, 1], periodic seams disagree, or a cut link has no interface cell on
 * either side. */
ebit_status ebit_build_coeffs(ebit_ctx* ctx, const double* const marker[3],
                              const uint8_t* vertex_colour, const uint8_t* cell_colour, double dt);

/* Eqs. energy_diffusion, ghost_T, Txx_ghost: one backward-Euler diffusion
 * step for both phases at once (the cut links decouple them).  T_star: the
 * advected field (cells).  T: output (cells); if use_guess != 0 it also holds
 * the initial guess.  T may alias T_star.  stats may be NULL.  Returns
 * EBIT_ENOCONV / EBIT_ENAN on solver failure (T then holds the last iterate). */
ebit_status ebit_heat_solve(ebit_ctx* ctx, const double* T_star, double* T, int use_guess,
                            ebit_stats* stats);

/* Eqs. mass_flux_computation and normal_gradient.  T: cells, each holding
 * its own phase's temperature.  With stats NULL the call returns without
 * waiting for the device (the work is queued on the context stream); with
 * stats it waits and reports the fallback count.  mdot_cell: output, mdot per cell (0 off the
 * interface), positive for evaporation.  mdot_face[a]: optional outputs
 * (NULL to skip, else all dim non-NULL): mdot on cut faces of axis a (the
 * value of the cell holding the crossing), NaN elsewhere.  The stencil takes
 * two points at h and 2h from the facet centroid along the normal into each
 * phase, tri-/bi-quadratic Lagrange values on the 3^d block around the point
 * (phase cells or one-layer ghost values from Eq. ghost_T). */
ebit_status ebit_mass_flux(ebit_ctx* ctx, const double* T, double* mdot_cell,
                           double* const mdot_face[3], ebit_stats* stats);

/* Eqs. ghost_velocity, Poisson_equation, poisson_ghost_fluid and the
 * face-velocity update.  u_l[a], u_v[a] (a < dim): axis-a face arrays of
 * the liquid and vapour fields; in: u*, out: u^{n+1} (both fields updated on
 * every face; a cut face's non-owning field first receives its ghost value).
 * mdot_cell: from ebit_mass_flux.  p: output pressure (cells); if use_guess
 * != 0 it also holds the initial guess.  stats->div_max reports the discrete
 * divergence after the update. */
ebit_status ebit_project(ebit_ctx* ctx, double* const u_l[3], double* const u_v[3],
                         const double* mdot_cell, double* p, int use_guess, ebit_stats* stats);

/* Sec. 2.4, Eq. extrapolation: `iters` pseudo-time steps of the transport
 * df/dtau + a . grad f = 0 that carries the cell field q across the interface
 * into the narrow band (cells whose 3^d block holds an interface cell), with
 * the geometry of the last ebit_build_coeffs.  a is the band cell's normal
 * (the normalised sum of the facet normals in its 3^d block) pointing away
 * from the interface into the cell's own phase.  mode selects the cells that
 * change (every other cell keeps its value and serves as data):
 *   EBIT_EXT_LIQ_TO_VAP    vapour band cells, from the liquid values;
 *   EBIT_EXT_VAP_TO_LIQ    liquid band cells, from the vapour values;
 *   EBIT_EXT_IFACE_TO_BAND band cells off the interface, from the interface
 *                          cells (the mass flux).
 * Steps: first-order upwind, explicit, dtau = h / dim (monotone), every
 * changing cell from the previous iterate; a term whose upwind cell is beyond
 * a wall or is neither data nor changing drops out.  q: device, cells,
 * updated in place (caller-owned).  iters >= 0.  Asynchronous on the context
 * stream; it reuses the context's solver scratch, so it is not to overlap a
 * solve of the same context.  EBIT_EINVAL for a NULL q, a bad mode or a
 * negative count; EBIT_ESTATE before ebit_build_coeffs. */
typedef enum { EBIT_EXT_LIQ_TO_VAP = 0, EBIT_EXT_VAP_TO_LIQ = 1, EBIT_EXT_IFACE_TO_BAND = 2 } ebit_ext_mode;
ebit_status ebit_extend(ebit_ctx* ctx, double* q, int mode, int iters);

/* Secs. 2.3-2.5, Eq. ghost_velocity over the whole narrow band, from the mass
 * flux carried to the band (step 4 of the time iteration: the mass flux, then
 * the ghost velocities; Sec. 2.4 extends the mass flux to the band for this
 * purpose).  A face gets a ghost when both its cells are band cells (those of
 * ebit_extend), with the geometry of the last ebit_build_coeffs:
 *   - a cut face as in ebit_project (its owner by theta, mdot and n of the
 *     cell holding the crossing; that cell carries a facet, so its band value
 *     is its own mass flux);
 *   - an uncut face belongs to the common phase of its two cells and takes
 *     mdot_f = (mdot_c + mdot_n) / 2 and n_f = (n_c + n_n)_a / 2, the means of
 *     the two cells' band values and unit band normals (0 where the block's
 *     facet normals sum to zero).
 * The other phase's field takes u_vap = u_liq + mdot_f [1/rho] n_f on a
 * liquid face and u_liq = u_vap - mdot_f [1/rho] n_f on a vapour face,
 * [1/rho] = 1/rho_l - 1/rho_v.  Every other face entry is left as it is.
 * u_l[a], u_v[a] (a < dim): axis-a face arrays, updated in place; mdot_band:
 * cells (ebit_mass_flux, then ebit_extend with EBIT_EXT_IFACE_TO_BAND).  All
 * device, caller-owned.  Asynchronous on the context stream; it reuses the
 * context's solver scratch, so it is not to overlap a solve of the same
 * context.  EBIT_EINVAL for a NULL argument; EBIT_ESTATE before
 * ebit_build_coeffs.  ebit_project sets the cut faces again, to the same
 * values when given the same mass flux. */
ebit_status ebit_ghost_band(ebit_ctx* ctx, double* const u_l[3], double* const u_v[3], const double* mdot_band);

/* Secs. 2.2 and 3.1, 2D: the liquid volume fraction of every cell (the
 * integral of H over the cell divided by h^2) from the piecewise-linear EBIT
 * reconstruction: in a cell with two markers, the area of the polygon of its
 * liquid corners and its two markers (the cell on the liquid side of the
 * segment joining them); a cell with no marker takes its corners' colour (1
 * or 0).  marker[0], marker[1]: x- and y-edge arrays of s or NaN;
 * vertex_colour: uint8 colours (the layouts of ebit_build_coeffs);
 * frac: output, cells.  All device, caller-owned.  Needs no
 * ebit_build_coeffs.  Synchronises the context stream to read the status.
 * EBIT_EINVAL for a 3D context or a NULL argument; EBIT_EGEOM if a cell
 * holds other than 0 or 2 markers or its corner colours do not change
 * exactly at its markers (that cell's fraction is NaN, the others are
 * written). */
ebit_status ebit_volume_fraction(ebit_ctx* ctx, const double* const marker[3], const uint8_t* vertex_colour,
                                 double* frac);

/* Sec. 2.3, the one-fluid projection the paper sets against the ghost-fluid
 * one (Eqs. Poisson_equation and pc_source): one face velocity field u (a <
 * dim, axis-a face arrays; in: u*, out: u^{n+1}) and, in each interface
 * cell, the volume source S_pc = mdot S_Gamma / V (1/rho_v - 1/rho_l) on the
 * right-hand side of div u^{n+1} = S_pc, with S_Gamma the area (3D) or
 * length (2D) of the cell's facet plane clipped to the cell and V = h^dim
 * (an evaporating cell is a source).  Face densities, walls and the solve are
 * those of ebit_project.  mdot_cell: from ebit_mass_flux.  p: output
 * pressure (cells); if use_guess != 0 it also holds the initial guess.
 * stats->div_max reports max |div u - S_pc| after the update.  Errors as
 * ebit_project. */
ebit_status ebit_project_one_fluid(ebit_ctx* ctx, double* const u[3], const double* mdot_cell, double* p,
                                   int use_guess, ebit_stats* stats);

/* Sec. 2.3, Eq. jump_interfacial_vel: the interfacial velocity at every cell
 * centre, with the geometry of the last ebit_build_coeffs (2D and 3D).  A
 * cell takes its own phase's velocity (the mean of its two faces per axis
 * in u_l for a liquid cell, in u_v for a vapour cell) plus mdot / rho_k
 * times the band normal n (the normalised sum of the facet normals, vapour
 * -> liquid, of the interface cells in its 3^d block; 0 off that band):
 *   u_gamma = u_k + (mdot / rho_k) n,
 * the paper's relation with its normal pointing into the vapour.  u_l[a],
 * u_v[a] (a < dim): axis-a face arrays; mdot_cell: cells, the mass flux
 * carried into the band (ebit_mass_flux, then ebit_extend with
 * EBIT_EXT_IFACE_TO_BAND); u_gamma[a]: outputs, cells, component a.  All
 * device, caller-owned.  Asynchronous on the context stream.  EBIT_EINVAL
 * for a NULL pointer among the first dim entries; EBIT_ESTATE before
 * ebit_build_coeffs. */
ebit_status ebit_interface_velocity(ebit_ctx* ctx, const double* const u_l[3], const double* const u_v[3],
                                    const double* mdot_cell, double* const u_gamma[3]);

/* Sec. 2.1, Eqs. marker_motion and discrete_marker_motion: one explicit
 * Euler step of the EBIT markers of a 2D grid, split into an x pass and a y
 * pass.  In the pass along axis a every marker moves along a by
 * u_gamma,a dt, bilinear in the four nearest cell centres (the stencil kept
 * inside walls, wrapped on periodic axes; a marker on a wall across a stays
 * on it; the y pass reads the same cell field at the moved positions).
 *   - A marker on a grid line along a (aligned) lands on the edge of its
 *     line that holds its new coordinate (clamped to a wall, wrapped on a
 *     periodic axis); two landings on one edge cancel; the vertices between
 *     the old and the new edge change colour.
 *   - An edge across a (unaligned) then holds a marker exactly when its end
 *     vertices differ in colour.  It sits where the moved interface meets
 *     the edge's line: on each moved segment (a cell's two markers) that
 *     reaches the line, the mean of the points met on the circles through
 *     the segment and the far end of each neighbouring segment (the chord
 *     when the interface ends there); the mean over such segments; the
 *     edge's midpoint if none reaches it.
 *   - Then each cell takes its corners' colour, or for a two-marker cell the
 *     side of its segment's line that the corners mark as liquid (a centre
 *     on the line is liquid).
 * u_gamma[0..1]: cells (ebit_interface_velocity).  marker[0..1]: the x- and
 * y-edge arrays, in/out.  vertex_colour: in/out.  cell_colour: in/out: the
 * cells within 3 cells of a marker (before the step or between its passes)
 * are recomputed, every other cell keeps its colour (in a consistent input
 * that is its corners' colour, which the step leaves unchanged there).  All
 * device, caller-owned; the periodic seams of the input must agree (as
 * ebit_build_coeffs requires).  The work is one scan of the marker arrays,
 * then kernels over the listed markers only.  The call does not need
 * ebit_build_coeffs; it uses the context's scratch, so it must not overlap
 * another call on the context, and it synchronises the context stream to
 * report errors.
 * Errors: EBIT_EINVAL for a 3D grid, fewer than 4 cells on an axis, 2^31
 * edges or more, a NULL
 * pointer, dt negative or not finite, or a marker that would move by more
 * than one cell (h) in a pass or by a non-finite amount; EBIT_EGEOM when a
 * cell holds other than 0 or 2 markers (a saddle) before a pass or after
 * the step, or a marker lies outside [0, 1].  After an error the marker and
 * colour arrays are unspecified. */
ebit_status ebit_advect_markers(ebit_ctx* ctx, const double* const u_gamma[3], double* const marker[3],
                                uint8_t* vertex_colour, uint8_t* cell_colour, double dt);

/* Sec. 2.4, Eq. energy_advection: the intermediate temperature T* of one
 * explicit Euler step of dT/dt + u . grad T = 0 in each phase (2D and 3D):
 *   T*[c] = T_k[c] - dt * (u_0 D_0 + u_1 D_1 + u_2 D_2),
 * with k the cell's colour (cell_colour 1: T_liq and u_l; 0: T_vap and u_v),
 * u_a the mean of the cell's two a-faces in u_k, and D_a the third-order
 * WENO derivative of Jiang & Shu (1996): the difference over h of the
 * values at the cell's two a-faces, each reconstructed from the upwind side
 * given by the sign of u_a (stencils (m, 0) and (0, p), linear weights 1/3
 * and 2/3, smoothness (T_0 - T_m)^2 and (T_p - T_0)^2, weights
 * d_r / (eps + beta_r)^2).  A zero component contributes nothing.  A
 * stencil cell beyond a wall takes the value of the nearest cell inside;
 * periodic axes wrap.  Every stencil reads one phase's field, so T_liq must
 * hold liquid values two cells into the vapour near the interface and T_vap
 * vapour values two cells into the liquid (Eq. extrapolation: ebit_extend
 * with EBIT_EXT_LIQ_TO_VAP / EBIT_EXT_VAP_TO_LIQ).
 * T_liq, T_vap, T_star: cells; u_l[a], u_v[a] (a < dim): axis-a face arrays;
 * cell_colour: uint8 per cell.  All device, caller-owned; T_star must not be
 * T_liq or T_vap (neighbours are read while cells are written).  eps: the
 * WENO regulariser (Jiang & Shu: 1e-6), in [1e-60, 1e60] (the kernel forms
 * products of four squared indicators).  No stability check: the caller
 * keeps |u_a| dt / h small (the explicit step).  The call does not need
 * ebit_build_coeffs and is asynchronous on the context stream.
 * Errors: EBIT_EINVAL for a NULL pointer (among the first dim face arrays),
 * T_star equal to an input, dt negative or not finite, eps outside
 * [1e-60, 1e60] (or NaN). */
ebit_status ebit_advect_energy(ebit_ctx* ctx, const double* T_liq, const double* T_vap, const double* const u_l[3],
                               const double* const u_v[3], const uint8_t* cell_colour, double dt, double eps,
                               double* T_star);

/* ---- inspection entry points (same conventions) --------------------------- */

/* Copy the geometry of the last ebit_build_coeffs: theta[a] (axis-a faces,
 * NaN where the link is not cut), flags (uint8 per cell: bits 0..5 cut link
 * on side -x,+x,-y,+y,-z,+z; bit 6 liquid; bit 7 interface cell) and facet
 * (6 arrays of cells back to back: centroid x,y,z then normal x,y,z; only
 * interface cells are defined).  Any output may be NULL. */
ebit_status ebit_get_geometry(ebit_ctx* ctx, double* const theta[3], uint8_t* flags, double* facet);

/* y = A x for system EBIT_SYS_HEAT (the heat matrix) or EBIT_SYS_PRESSURE
 * (the negated Poisson matrix -L, symmetric positive definite), FP64. */
ebit_status ebit_apply(ebit_ctx* ctx, int system, const double* x, double* y);

/* Right-hand side of the heat system for T_star (cells -> cells). */
ebit_status ebit_heat_rhs(ebit_ctx* ctx, const double* T_star, double* b);

/* First half of ebit_project: writes the ghost values into u_l / u_v and the
 * right-hand side b of the SPD pressure system (-L p = b). */
ebit_status ebit_project_rhs(ebit_ctx* ctx, double* const u_l[3], double* const u_v[3],
                             const double* mdot_cell, double* b);

/* Kernel classes the profiler times (ebit_profile_read). */
typedef enum {
  EBIT_KC_FINE_SMOOTH = 0,    /* fine-level red-black sweeps (the first       */
                              /* post-smoothing sweep adds the prolongation)  */
  EBIT_KC_FINE_RESTRICT = 1,  /* fine-level residual + restriction             */
  EBIT_KC_COARSE = 2,         /* sweeps + restrictions of the explicit coarse  */
                              /* levels above the tail                        */
  EBIT_KC_OUTER_APPLY = 3,    /* outer loop: search direction update + A p     */
  EBIT_KC_OUTER_UPDATE = 4,   /* outer loop: x and r update                    */
  EBIT_KC_TAIL = 5            /* single-work-group solve of the coarsest levels */
} ebit_kernel_class;

/* Profiling of launches with hipEvents recorded on the solve stream around
 * each launch of the classes above -- around each run of consecutive fine
 * sweeps as one bracket (enable != 0 turns it on and clears the totals; the
 * events are created by this call, once).  ebit_profile_read returns, for
 * one class, the number of launches timed and their summed device time in
 * milliseconds, after synchronising.  While profiling is on, the iteration
 * blocks are launched one kernel at a time instead of replayed as graphs.
 * Meant for measurement runs: the events add a little host work. */
ebit_status ebit_profile(ebit_ctx* ctx, int enable);
ebit_status ebit_profile_read(ebit_ctx* ctx, int kernel_class, long long* launches, double* ms);

/* Levels of the multigrid hierarchy and their sizes (host outputs). */
ebit_status ebit_levels(const ebit_ctx* ctx, int* nlevels, int* sizes /* [3*nlevels] */);

/* ---- batches of independent cases --------------------------------------
 * A batch groups existing contexts (any grid sizes, one dim, equal solver
 * options except theta_min) so that every kernel of a solve is ONE launch
 * over all cases: a work list maps each launch's blocks onto (case, block),
 * and a per-case active mask lets converged cases drop out while the others
 * iterate.  The other steps (geometry, right-hand sides, mass flux, face
 * update) are launched case by case on the batch stream.  Results per case
 * equal those of the same calls on each context.  While a batch call runs,
 * its contexts must not be used on their own; the batch never frees them.
 * Arrays of per-case pointers are HOST arrays of DEVICE pointers; marker,
 * u_l and u_v hold 3 entries per case (entry 3 c + a). */
typedef struct ebit_batch ebit_batch;

/* Device workspace of a batch of ncases (plan tables and work lists). */
size_t ebit_batch_workspace_bytes(int ncases, const ebit_opts* opts);
/* ws: >= ebit_batch_workspace_bytes(ncases, &opts of ctx[0]) bytes, 256-byte
 * aligned, caller-owned.  EBIT_EINVAL if the contexts differ in dim or in
 * the solver options above, or a context appears twice. */
ebit_status ebit_batch_create(ebit_batch** out, int ncases, ebit_ctx* const ctx[], void* workspace, size_t bytes,
                              void* hip_stream);
ebit_status ebit_batch_destroy(ebit_batch* batch);
const char* ebit_batch_last_error(const ebit_batch* batch);
/* ebit_build_coeffs of every case (one synchronisation for all geometry
 * checks); dt[] per case. */
ebit_status ebit_batch_build_coeffs(ebit_batch* batch, const double* const marker[], const uint8_t* const vcol[],
                                    const uint8_t* const ccol[], const double dt[]);
/* ebit_heat_solve / ebit_mass_flux / ebit_project of every case; stats[]
 * (may be NULL) gets each case's figures and status, seconds = the whole
 * batch call; the return value is the first failing case's status.  The
 * batched mass flux with stats NULL does not wait for the device. */
ebit_status ebit_batch_heat_solve(ebit_batch* batch, const double* const T_star[], double* const T[], int use_guess,
                                  ebit_stats stats[]);
ebit_status ebit_batch_mass_flux(ebit_batch* batch, const double* const T[], double* const mdot[], ebit_stats stats[]);
ebit_status ebit_batch_project(ebit_batch* batch, double* const u_l[], double* const u_v[], const double* const mdot[],
                               double* const p[], int use_guess, ebit_stats stats[]);

/* ---- autotuning ----------------------------------------------------------
 * Pick the solve schedule -- sweeps nu1 = nu2 in {1, 2, 3}, the top size of
 * the single-work-group tail in {256, 1024, 4096, 16384} cells (capped by
 * the LDS), and the iteration-block length check_every in {1, 2, 4} -- by
 * timing cold-start solves to rtol of the caller's right-hand sides of the
 * current coefficients (after ebit_build_coeffs): b_heat and b_press are
 * device arrays of a heat and a pressure right-hand side (either may be
 * NULL), x a device array the solves write.  Each candidate solves each
 * system three times (the first captures its graphs) and counts the faster
 * of the last two.  The fastest candidate whose solves all converge becomes
 * the context's (batch's) schedule and is returned in *chosen with its
 * summed solve time (ms) in *best_ms.
 * Clobbers the contexts' internal right-hand-side buffers.  A batch's
 * contexts keep their own options. */
ebit_status ebit_autotune(ebit_ctx* ctx, const double* b_heat, const double* b_press, double* x, ebit_opts* chosen,
                          double* best_ms);
ebit_status ebit_batch_autotune(ebit_batch* batch, const double* const b_heat[], const double* const b_press[],
                                double* const x[], ebit_opts* chosen, double* best_ms);

/* ---- the tuned-schedule cache ----------------------------------------------
 * A text file of one schedule per line,
 *   ebit-schedule <key> nu tail_cells check_every ms
 * where the key of a context is "dim n0 n1 n2 precision outer" and that of a
 * batch "batch dim ncases total_cells largest_case_cells precision outer".
 * Lines are appended; the last line with a key wins; other lines are
 * ignored.  Host code only (no device work).
 *
 * ebit_tune_lookup: *found = 1 and the schedule (nu1 = nu2, tail_cells,
 * check_every) written into *chosen (its other fields copied from *base)
 * when the file holds the key of (grid, base), else *found = 0 and *chosen =
 * *base; a missing or unreadable file is not an error.  EBIT_EINVAL for a
 * NULL argument or a bad grid.
 * ebit_tune_store: appends the line of (grid, chosen, ms), creating the
 * file.  EBIT_EINVAL for a NULL argument or a bad grid, EBIT_EIO when the
 * file cannot be written. */
ebit_status ebit_tune_lookup(const char* path, const ebit_grid* grid, const ebit_opts* base, ebit_opts* chosen,
                             int* found);
ebit_status ebit_tune_store(const char* path, const ebit_grid* grid, const ebit_opts* chosen, double ms);

/* ebit_autotune / ebit_batch_autotune through the cache at path: a schedule
 * stored for the key is applied without timing (*from_cache = 1, *best_ms
 * the stored time); otherwise the candidates are timed as by
 * ebit_autotune, the winner is applied and appended to the file
 * (*from_cache = 0).  Errors as ebit_autotune, and EBIT_EIO when the file
 * cannot be written. */
ebit_status ebit_autotune_cached(ebit_ctx* ctx, const char* path, const double* b_heat, const double* b_press,
                                 double* x, ebit_opts* chosen, double* best_ms, int* from_cache);
ebit_status ebit_batch_autotune_cached(ebit_batch* batch, const char* path, const double* const b_heat[],
                                       const double* const b_press[], double* const x[], ebit_opts* chosen,
                                       double* best_ms, int* from_cache);

/* ---- the geometry pass without allocation --------------------------------
 * For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the cut
 * fractions theta and the flags of ebit_build_coeffs (Sec. 2.1 and the
 * theta of Eq. ghost_T, through the same kernels and the same arithmetic)
 * for a grid of at most EBIT_NOALLOC_MAX_CELLS cells, with no context and no
 * workspace.  The interface facets and the status word live in a file-scope
 * device array of the library (12 MiB + 256 B per GPU, held by every GPU the
 * call runs on until the process ends); the call makes no device or host
 * allocation.
 * Arguments: grid as for ebit_create (only dim, n, h and the periodic sides
 * are used); marker[a], vertex_colour, cell_colour as for
 * ebit_build_coeffs; theta[a] (axis-a face arrays) and flags (one byte per
 * cell) are caller-owned device outputs with the layout of
 * ebit_get_geometry.  Work is enqueued on hip_stream (NULL = the null
 * stream) and the call waits for it to read the status word.
 * Errors: EBIT_EINVAL for a bad grid or argument, or more than
 * EBIT_NOALLOC_MAX_CELLS cells (nothing is launched); EBIT_EGEOM as for
 * ebit_build_coeffs; EBIT_EHIP if a HIP call fails (no context holds the
 * text).  Every call on one GPU shares that GPU's array: calls that overlap
 * on one GPU (two streams, two host threads) race and must not. */
#define EBIT_NOALLOC_MAX_CELLS (1 << 18)
ebit_status ebit_cut_fractions_noalloc(const ebit_grid* grid, const double* const marker[3],
                                       const uint8_t* vertex_colour, const uint8_t* cell_colour,
                                       double* const theta[3], uint8_t* flags, void* hip_stream);

#ifdef __cplusplus
}
#endif
#endif /* EBIT_H */
