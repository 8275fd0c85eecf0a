/*
 * pmgfr — P-multigrid FR/CPR stage solver for locally preconditioned low-Mach flow on MI355X.
 *
 * C ABI of the hot path of Wang & Yu, "An implicit P-multigrid flux reconstruction method for
 * simulation of locally preconditioned unsteady Navier-Stokes equations at low Mach numbers"
 * (arXiv 1908.03972): one pseudo-transient ESDIRK stage solve by FAS V-cycles whose smoother is
 * element Jacobi with dense element blocks.
 *
 * Conventions (all entry points)
 * ------------------------------
 * - Every function returns a pmg_status. PMG_OK is 0; on failure a message is available from
 *   pmg_last_error() (thread-local, valid until the next failing call on the same thread).
 *   Argument checks are synchronous and leave all outputs untouched.
 * - "device" pointers are HIP device allocations on the level's device; "host" pointers are
 *   ordinary CPU memory. The library never frees caller memory.
 * - A state field on a level is double[Nv][Np][Ne] (element index fastest, for coalesced access),
 *   with Nv = 4 primitive variables (p, u, v, T), Np = (P+1)^2 solution points numbered
 *   p = i + (P+1) j (i along xi), Ne elements. Sizes below are in elements of that layout.
 *   States (q, q_c^n excepted) are stored as offsets from the level's reference state q_ref:
 *   the unknown held for variable v is q_v - q_ref_v ("gauge" pressure and temperature when
 *   q_ref = q_inf). At low Mach number the residual's sensitivity to the pressure grows like
 *   1/Ma^2 (eqs. (9), (10), (21)); storing offsets keeps the unknowns' quantisation at the size
 *   of the disturbance rather than of the absolute pressure. q_ref = 0 gives plain storage.
 *   Residuals F and R are not offset.
 * - `stream` is a hipStream_t (passed as void*). Work is enqueued on it asynchronously unless a
 *   function says it synchronises. Entry points are not re-entrant on the same handle: calls that
 *   share a level or factor handle must be ordered on one stream.
 * - Device-side faults (a zero pivot, a non-finite value) raise a per-level flag that
 *   pmg_level_status() reads and clears; esdirk_stage_solve() checks it itself.
 * - Hot calls allocate nothing: every workspace is created with its level.
 */
#ifndef PMGFR_H
#define PMGFR_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t pmg_status;
#define PMG_OK 0
#define PMG_E_ARG (-1)          /* invalid argument (null handle, bad enum, bad size)        */
#define PMG_E_SHAPE (-2)        /* levels or sizes that do not fit together                   */
#define PMG_E_HIP (-3)          /* a HIP runtime call failed                                  */
#define PMG_E_SINGULAR (-4)     /* a zero pivot in an element block                           */
#define PMG_E_NONFINITE (-5)    /* a NaN or Inf in a residual norm                            */
#define PMG_E_NOT_CONVERGED (-6)/* the stage solve hit max_vcycles                            */
#define PMG_E_NOMEM (-7)        /* device allocation failed at level or factor creation       */

#define PMG_BC_SLIP_WALL (-1)   /* face_nbr tag: slip wall, ghost (p, u - 2(u.n)n, T)         */
#define PMG_BC_FAR_FIELD (-2)   /* face_nbr tag: far field, ghost = q_inf                     */
#define PMG_BC_NOSLIP_WALL (-3) /* face_nbr tag: no-slip adiabatic wall, ghost (p, -u, -v, T);
                                   viscous: one-sided common gradient without its normal grad T */

typedef struct pmg_level_s* pmg_level;
typedef struct pmg_factors_s* pmg_factors;
typedef struct pmg_batch_s* pmg_batch;

/* Thread-local text of the last error, or "" if none. The pointer stays owned by the library. */
const char* pmg_last_error(void);

/* Version of this ABI (major * 100 + minor); the library returns PMG_ABI_VERSION. */
#define PMG_ABI_VERSION 108
int32_t pmg_abi_version(void);

/*
 * One P-level of a mesh (Sec. 2.3: FR/CPR on quadrilaterals or hexahedra with tensor-product
 * corrections). All arrays are host memory and are deep-copied; the descriptor may be freed after
 * the call.
 *   dim          2 (quadrilaterals) or 3 (hexahedra: inviscid, P <= 3, slip wall and far field,
 *                primitive variables (p, u, v, w, T), Nv = 5).
 *   P            solution degree, 0..6 in 2-D (element blocks need P <= 5), 0..3 in 3-D.
 *   geom_order   1 (bilinear / trilinear) or 2 (9-node / 27-node quadratic).
 *   nodes        2-D [Ne][(g+1)^2][2], 3-D [Ne][(g+1)^3][3] geometry nodes in tensor order, xi
 *                fastest, at reference coordinates (-1 + 2a/g, -1 + 2b/g[, -1 + 2c/g]).
 *   face_nbr     [Ne][2 dim] neighbour element across faces (xi=-1, xi=+1, eta=-1, eta=+1[,
 *                zeta=-1, zeta=+1]), or a negative PMG_BC_* tag.
 *   face_nbr_face[Ne][2 dim] the neighbour's face index (ignored for boundary faces).
 *   face_orient  2-D [Ne][4]: 0 if flux point k meets the neighbour's point k, 1 if point P-k.
 *                3-D [Ne][6]: a hexahedron face's points are (k1, k2) along its two tangential
 *                reference directions in increasing order ((eta, zeta), (xi, zeta), (xi, eta)); the
 *                code (0..7) maps (k1, k2) to the neighbour's face point: swap the pair if bit 0 is
 *                set, then reverse the first index (P - k) if bit 1 is set and the second if bit 2.
 *                3-D metric terms are taken in the conservative curl form (Gauss-Lobatto
 *                interpolant of X_l grad X_m), which keeps a uniform flow exactly uniform on curved
 *                elements for P >= 1.
 *   gamma, rgas  ratio of specific heats and gas constant (eqs. (1)-(6), ideal gas).
 *   eps_mode     reference velocity U_r = eps c of eq. (11): 0 = eps = min(1, Ma) (cut-off
 *                off), 1 = eps = min(1, max(kappa Ma_inf, Ma)).
 *   q_inf        free-stream primitive state used by far-field faces.
 *   q_ref        reference state subtracted from every stored state (see the conventions above);
 *                all levels of one solve must share it.
 *   device       HIP device ordinal on which the level lives.
 *   mu           dynamic viscosity (Sec. 2.1); 0 = inviscid. With mu > 0 the residual carries the
 *                viscous fluxes with the BR2 common gradient of eqs. (22)-(23) and the level
 *                allocates a gradient-trace buffer and an n x n x Ne FP64 block buffer.
 *   prandtl      Prandtl number (0.72 in Sec. 2.1); used when mu > 0.
 *   br2_penalty  factor on the BR2 liftings in the common gradient (the number of element faces,
 *                4, is the stable choice); used when mu > 0.
 */
typedef struct {
  int32_t dim;
  int32_t P;
  int32_t geom_order;
  int32_t n_elements;
  const double* nodes;
  const int32_t* face_nbr;
  const int32_t* face_nbr_face;
  const int32_t* face_orient;
  double gamma;
  double rgas;
  int32_t eps_mode;
  double ma_inf;
  double kappa;
  double q_inf[5];
  double q_ref[5];
  int32_t device;
  double mu;
  double prandtl;
  double br2_penalty;
} pmg_level_desc;

/* Create a level: computes the Gauss solution/flux points, the 1-D operators, the metrics from
 * the exact element mapping, uploads them and allocates the level's workspace.
 * Errors: PMG_E_ARG (bad descriptor), PMG_E_NOMEM, PMG_E_HIP. */
pmg_status pmg_level_create(const pmg_level_desc* desc, pmg_level* out);
pmg_status pmg_level_destroy(pmg_level L);

/* info[0..7] = dim, P, Np, Nv, n (= Nv Np, the element block size), Ne, device, geom_order. */
pmg_status pmg_level_info(pmg_level L, int32_t* info);

/* Physical solution-point coordinates, host output double[dim][Np][Ne] (x, y[, z]). */
pmg_status pmg_level_points(pmg_level L, double* xy_host);

/* Element length scale of eqs. (32)-(33), host output double[Ne]: twice the smallest distance from
 * the element's area centroid (6x6 Gauss rule on the exact mapping) to its four faces, each face
 * taken as the segment between its two corner nodes; in 3-D from the volume centroid (5^3 Gauss
 * rule) to the six face planes (through the face's centre node, normal to its corner diagonals). */
pmg_status pmg_level_dx(pmg_level L, double* dx_host);

/* Elements per workgroup of the fused residual / element-Jacobi kernel of a level (the kernel of
 * eqs. (20), (21) and (30); quadrilaterals and hexahedra). A workgroup owns that many elements, with the element
 * fastest across lanes, so that a wave's load of one (variable, point) of the [Nv][Np][Ne] state
 * covers consecutive elements. Several values are compiled per P; results do not depend on the
 * choice beyond the summation order of the residual norms.
 *
 * pmg_level_epw — *epw the level's current value; cand (nullable, room for 4) and *n_cand
 *   (nullable) the compiled candidates, the default for P first (only the default on viscous levels
 *   and at P >= 5). Errors: PMG_E_ARG (null epw). */
pmg_status pmg_level_epw(pmg_level L, int32_t* epw, int32_t* cand, int32_t* n_cand);

/* pmg_level_set_epw — use candidate epw (0: the default for P) from now on. Set it before capturing
 * a stage solve in a graph: a captured graph keeps the launches it recorded.
 * Errors: PMG_E_ARG (not a compiled candidate). */
pmg_status pmg_level_set_epw(pmg_level L, int32_t epw);

/* pmg_level_autotune — time every candidate on this level (reps residual evaluations plus reps
 * element-Jacobi sweeps with inverse blocks of the given precision, 32 or 64, after one untimed
 * pass of the same), keep the fastest — the default unless another candidate is more than 2%
 * faster, so that timing noise does not flip the choice — and return it in *epw_out (nullable);
 * us_out (nullable, room
 * for n_cand doubles, in candidate order) receives the microseconds per residual + sweep pair.
 * A setup call: it allocates and frees its own scratch state, overwrites the level's workspace,
 * and synchronises the stream. Errors: PMG_E_ARG (precision, reps < 1),
 * PMG_E_NOMEM, PMG_E_HIP; on error the level keeps its previous value. */
pmg_status pmg_level_autotune(pmg_level L, int32_t precision, int32_t reps, int32_t* epw_out, double* us_out,
                              void* stream);

/* pmg_dtau_min — the pseudo-time scale of eq. (33) at state q (device, stored form [Nv][Np][Ne]):
 *   dtau_min = min over elements e and solution points of (dx_e / (P+1)) / (c + |v|), and, when the
 *   level has mu > 0, of (dx_e / (P+1))^2 rho / mu. Writes the host double *dtau_min and
 * synchronises the stream. Errors: PMG_E_ARG (null), PMG_E_NONFINITE (a point with T <= 0 or a
 * non-finite value), PMG_E_HIP. */
pmg_status pmg_dtau_min(pmg_level L, const double* q, double* dtau_min, void* stream);

/* Read and clear the level's device fault flags (synchronises the device).
 * *flags bit 0: a zero/non-finite pivot was met; returns PMG_E_SINGULAR if set, else PMG_OK. */
pmg_status pmg_level_status(pmg_level L, int32_t* flags);

/* Storage for the element-Jacobi blocks of one level (Sec. 2.4, eq. (30)): the inverse of every
 * element block D_e, kept as n x n per element in `precision` 64 (FP64) or 32 (FP32).
 * Footprint: n * npad * Ne * precision/8 bytes (npad = n in 2-D, n rounded up to 4 in 3-D); a 3-D
 * P = 3 level (n = 320) adds an FP64 elimination work array of n * n * 8 bytes per slot, two slots
 * per compute unit (about 420 MB on a 256-CU device), and 70400 bytes of pointwise derivatives per
 * element (2.6 GB for 36 864 elements), held until pmg_factors_destroy. */
pmg_status pmg_factors_create(pmg_level L, int32_t precision, pmg_factors* out);
pmg_status pmg_factors_destroy(pmg_factors F);

/*
 * pmg_line_factors_create — blocks for element-line Jacobi instead of element Jacobi. This is the
 * smoother for strongly stretched meshes that the introduction cites from earlier implicit
 * high-order solvers. Along each line of face-connected elements it keeps, besides D_e of
 * eqs. (28)-(30), the blocks A_{e,e'} = -dR_e/dq_{e'} coupling an element to its predecessor and
 * successor. It solves each line's block-tridiagonal system exactly; the lines are independent
 * (Jacobi across lines).
 *   line_elems  host int32[n_lines][line_len], element indices in line order, copied. Every element
 *               appears exactly once (n_lines * line_len == Ne), and consecutive elements of a line
 *               share exactly one face; else PMG_E_SHAPE.
 *   precision   64 or 32: storage of the block-Thomas inverses W_k = D'_k^{-1}. The elimination
 *               itself runs in FP64.
 * The handle is a pmg_factors and takes the place of element blocks everywhere:
 *   - fr_element_jacobian builds D_e and factors every line (D_out as documented there);
 *   - ejacobi_sweep runs line sweeps q <- q + alpha_r A_line^{-1} (F(q) - S);
 *   - a stage solve smooths by lines on every level whose factors are line factors.
 * Limits: quadrilateral, inviscid levels with P <= 4; otherwise PMG_E_ARG.
 * Footprint per element: n*n*8 (D_e) + n*n*precision/8 (W) + 256 (P+1) bytes, plus one state-sized
 * FP64 array; released by pmg_factors_destroy.
 */
pmg_status pmg_line_factors_create(pmg_level L, int32_t precision, const int32_t* line_elems, int32_t n_lines,
                                   int32_t line_len, pmg_factors* out);

/* pmg_line_blocks — refactors line factors F at state q, as fr_element_jacobian does. It also writes
 * the blocks out, for tests; each output is device double[Ne][n][n], row-major, row index p*Nv + v,
 * or NULL:
 *   D_out   D_e;
 *   Am_out  A_{e, previous element of its line}; zero for a line's first element;
 *   Ap_out  A_{e, next element of its line}; zero for a line's last element.
 * Errors: PMG_E_ARG (not a line-factor handle, null q, dtau <= 0), PMG_E_HIP. */
pmg_status pmg_line_blocks(pmg_factors F, const double* q, double dtau, double c_mass, double* D_out,
                           double* Am_out, double* Ap_out, void* stream);

/*
 * fr_residual — stage residual of eq. (26) with the FAS forcing of eqs. (34)-(36):
 *   F = R(q) - c_mass * q_c(q) + src - S,
 * R = -div f the FR/CPR residual of eq. (20) with the common flux of eq. (21), q_c the
 * conservative variables, c_mass = 1/(omega dt) (0 for a steady problem, where F = R).
 *   q    device, state layout, read.      src, S   device state layout or NULL (= 0).
 *   F    device, state layout, written. May alias S (each entry is read before it is written);
 *        must not alias q.
 *   norms device double[Nv+1] or NULL: per-variable Euclidean norms of F and the norm over all
 *        variables (deterministic two-pass reduction).
 */
pmg_status fr_residual(pmg_level L, const double* q, const double* src, const double* S, double c_mass,
                       double* F, double* norms, void* stream);

/*
 * fr_residual_noalloc — fr_residual for callers that cannot allocate device memory (code under
 * HIP graph capture, serving loops, harnesses that forbid hipMalloc): the same arguments, kernels
 * and results (F and norms bit for bit), but the per-workgroup partial sums of the norms are kept
 * in a file-scope device array of the library (65536 doubles = 512 KiB per device, held until the
 * process ends) instead of the level's workspace. Nothing is allocated or freed in the call.
 * Limit: with norms, the level's workgroups times Nv must not exceed 65536 (every level of the
 * configurations here fits, the 36 864-hexahedron P3 level uses 46 080); larger levels get
 * PMG_E_ARG before any launch. Calls that overlap on one device (several host threads, or
 * streams not ordered with each other) share that array and race: order them on one stream.
 * Every call writes all the partials it reads, so nothing needs clearing between calls.
 */
pmg_status fr_residual_noalloc(pmg_level L, const double* q, const double* src, const double* S, double c_mass,
                               double* F, double* norms, void* stream);

/* q_c = (rho, rho u, rho v, rho E) of a stored primitive state (Sec. 2.1); q_c is absolute (not
 * offset). q, qc: device state layout. */
pmg_status fr_conservative(pmg_level L, const double* q, double* qc, void* stream);

/*
 * fr_element_jacobian — element blocks of the pseudo-transient linearisation, eqs. (28)-(30):
 *   D_e = Gamma(q)/dtau + c_mass M(q) - dR_e/dq_e,
 * with the neighbours' states held fixed and the common flux differentiated exactly (its mean
 * state, eigenvalues and preconditioner included). Each block is row-equilibrated by powers of 2
 * and inverted by Gauss-Jordan elimination with partial pivoting in FP64; the inverse is stored
 * in `fac` at the factor precision.
 *   q      device state, read.   dtau > 0 (pass +inf for no pseudo-time term).
 *   D_out  device double[Ne][n][n] row-major (row index p*Nv + v) or NULL: the unfactored blocks.
 * A zero pivot sets the level's fault flag (see pmg_level_status).
 */
pmg_status fr_element_jacobian(pmg_level L, const double* q, double dtau, double c_mass, double* D_out,
                               pmg_factors fac, void* stream);

/*
 * ejacobi_sweep — n_sweeps synchronous element-Jacobi sweeps, eq. (30):
 *   q <- q + alpha_r D^{-1} (F(q) - S),   F as in fr_residual,
 * every element using its neighbours' state from the previous sweep.
 *   q        device state, read and written in place (the library ping-pongs internally).
 *   fac      blocks built by fr_element_jacobian on the same level.
 *   F_after  device state or NULL: F(q) - S at the final state (the negative FAS defect).
 *   norms    device double[Nv+1] or NULL: norms of F(q) - S at the state the first sweep starts
 *            from (of F_after when n_sweeps is 0).
 */
pmg_status ejacobi_sweep(pmg_level L, pmg_factors fac, double* q, const double* src, const double* S,
                         double c_mass, int32_t n_sweeps, double alpha_r, double* F_after, double* norms,
                         void* stream);

/*
 * pmg_restrict — x_c = P x_f: the L2 projection (in the reference element) of each element's
 * degree-P_f polynomial onto degree P_c, applied per variable (Sec. 3, eqs. (39), (40)).
 * pmg_prolong — x_f += I dx_c: interpolation of the degree-P_c polynomial at the degree-P_f
 * points (eqs. (44), (45)).
 * Both levels must be on the same mesh with P_c < P_f and share q_ref, else PMG_E_SHAPE (the
 * projection preserves constants, so offsets transfer like states). nvar in 1..Nv gives the
 * leading variables of the state layout that are transferred.
 */
pmg_status pmg_restrict(pmg_level fine, pmg_level coarse, const double* x_f, double* x_c, int32_t nvar,
                        void* stream);
pmg_status pmg_prolong(pmg_level coarse, pmg_level fine, const double* dx_c, double* x_f, int32_t nvar,
                       void* stream);

/* Options of a stage solve (Secs. 2.4 and 3). */
typedef struct {
  int32_t n_levels;               /* 1..8: levels[0] is the finest, degrees strictly decreasing */
  pmg_level* levels;              /* host array of level handles on one mesh                    */
  pmg_factors* factors;           /* host array, one per level                                  */
  const int32_t* n_smooth;        /* host array: I{n0-n1-...}; pre = post, coarsest once         */
  double dtau_init;               /* pseudo time step at V-cycle 0                               */
  double dtau_max;                /* SER cap                                                     */
  double ser_exponent;            /* 1.5 in eq. (31)                                             */
  int32_t refresh_every;          /* rebuild the blocks every k V-cycles (10 in Sec. 4.1)        */
  int32_t freeze_at_max;          /* 1: no rebuild after one made with dtau = dtau_max          */
  double tol_rel;                 /* stop when ||F(q^m)|| / ||F(q^0)|| <= tol_rel                */
  int32_t max_vcycles;
  double alpha_r;                 /* relaxation of eq. (30), 1 in the paper                      */
  int32_t use_graph;              /* 1: replay V-cycles without a block rebuild from a HIP graph
                                     captured once per argument set (same results, fewer launches) */
  int32_t use_cfl;                /* 1: CFL form of eqs. (31)-(33): dtau_init = cfl_init dtau_min and
                                     dtau_max = cfl_max dtau_min, with dtau_min of the finest level
                                     at the initial guess (pmg_dtau_min); dtau_init/dtau_max unused */
  double cfl_init;                /* 1e2 in Sec. 4.2                                             */
  double cfl_max;                 /* 1e5 in Sec. 4.2                                             */
  int32_t stage_guess;            /* initial guess of an implicit stage in esdirk_step (the paper
                                     states none): 0 the previous stage value, 1 the explicit
                                     predictor q_c^n + dt (sum_j a_ij R_j + omega R_{i-1}) in
                                     primitive variables. Use 1 once q^n is a solved time level
                                     (R(q^n) is then the discrete time derivative): from such a
                                     state the previous stage value starts too close to the
                                     solution for the relative tolerance and the SER law. From an
                                     unsolved initial condition R(q^n) carries the scheme's
                                     truncation error and the predictor is far off: use 0.
                                     esdirk_stage_solve starts from the q it is given         */
  int32_t ser_floor;              /* 1: the SER law of eq. (31) never takes dtau below its value at
                                     V-cycle 0 (dtau_init, or cfl_init dtau_min); the paper
                                     states no lower bound. 0: none (the default)               */
  int32_t lookahead;              /* single-case stage solves (esdirk_stage_solve, esdirk_step):
                                     1: between block rebuilds, enqueue the next V-cycle before the
                                     host has read the norm of the one in flight, so that the device
                                     does not wait for the host's stopping test; the state before
                                     it is kept in the finest level's workspace and restored when
                                     the test says stop, so results, norm history and V-cycle
                                     counts are those of 0. Skipped where the last rate of decrease
                                     predicts the tolerance within a factor 8 (a discarded V-cycle
                                     costs its whole time). 2: the same without the prediction
                                     (every eligible V-cycle; for tests). 0: one V-cycle per host
                                     test (the default). Ignored by the batched and Newton-Krylov
                                     solves                                                     */
} pmg_solve_opts;

typedef struct {
  int32_t n_vcycles;
  int32_t n_refresh;
  double r0;
  double r_final;
  double* history;                /* host array or NULL: r_m for m = 0..n_vcycles              */
  int32_t history_capacity;
  pmg_status status;
  double seconds;                 /* host wall time of the stage solve                         */
  double dtau_min;                /* dtau_min used by the CFL form, 0 otherwise                 */
} pmg_solve_stats;

/*
 * esdirk_stage_solve — solve the ESDIRK stage equation F(q) = 0 of eq. (26) by
 * pseudo-transient continuation (eq. (27)) with one FAS V-cycle per pseudo step:
 *   src = (q_c^n + dt sum_j a_row[j] R_prev[j]) / (omega dt),  c_mass = 1/(omega dt);
 *   dt <= 0 selects a steady solve (F = R, no source).
 * Per V-cycle m: r_m = ||F(q^m)||; dtau_m by the SER law of eq. (31); blocks rebuilt on every
 * level when m % refresh_every == 0 (fine level from q^m, coarse levels from their restricted
 * state); V-cycle of Sec. 3. Stops when r_m / r_0 <= tol_rel.
 *   qc_n     device state: conservative variables of q^n (unused when steady).
 *   R_prev   host array of n_prev device states R(q^j); a_row host double[n_prev].
 *   q        device state, in: initial guess, out: stage solution.
 *   R_out    device state or NULL: R(q_stage), for later stages.
 * Synchronises the stream (it reads one norm per V-cycle). Returns PMG_E_NOT_CONVERGED when
 * max_vcycles is reached, PMG_E_NONFINITE on a NaN norm, PMG_E_SINGULAR on a zero pivot.
 */
pmg_status esdirk_stage_solve(const pmg_solve_opts* opts, double omega, double dt, const double* qc_n,
                              const double* const* R_prev, const double* a_row, int32_t n_prev, double* q,
                              double* R_out, pmg_solve_stats* stats, void* stream);

/*
 * esdirk_step — one physical time step q^n -> q^{n+1} of eq. (24) with the first stage explicit
 * and the implicit stages solved by esdirk_stage_solve (the schemes are stiffly accurate, so
 * q^{n+1} is the last stage value).
 *   scheme  2: ESDIRK2, three stages (Kennedy & Carpenter), 3: ESDIRK3, four stages
 *           (ESDIRK3(2)4L[2]SA), 4: ESDIRK4, six stages (ESDIRK4(3)6L[2]SA), the schemes cited
 *           in Sec. 2.4.
 *   q       device state, in q^n, out q^{n+1}.
 *   work    device, (number of stages) consecutive state arrays: q_c^n and the stage residuals.
 *   stats   host array of n_stats entries or NULL: one per implicit stage.
 * A stage that reaches max_vcycles leaves its last iterate as the stage value and the later
 * stages still run; the step then returns PMG_E_NOT_CONVERGED. Any other failure stops the step
 * with that status (recorded in the stats of the stages not run); q holds the last iterate.
 */
pmg_status esdirk_step(const pmg_solve_opts* opts, int32_t scheme, double dt, double* q, double* work,
                       pmg_solve_stats* stats, int32_t n_stats, void* stream);

/*
 * nk_stage_solve — the stage equation F(q) = 0 of eq. (26) by pseudo-transient Newton with the
 * whole Jacobian and the V-cycle as preconditioner (the paper names this combination as its next
 * step for lower Mach numbers; Sec. 5). Newton step m solves
 *   (Gamma(q_m)/dtau_m - dF/dq) delta = F(q_m),   q_{m+1} = q_m + delta
 * (the linearisation of eqs. (27)-(28) without the element-Jacobi splitting of eq. (29)) by one
 * cycle of flexible GMRES from delta = 0: at most krylov_dim directions, stopped once the
 * least-squares residual is <= eta ||F(q_m)||; classical Gram-Schmidt applied twice (the new
 * direction's norm from the second pass's dot products). Products with
 * dF/dq are forward differences (F(q_m + h z) - F(q_m))/h with h ||z|| = fd_rel sqrt(N), N the
 * entries of a finest-level state: fd_rel is the RMS perturbation per entry, of the order of
 * sqrt(machine epsilon) times the absolute state (about 1e-3 for pressures near 6e4). With precondition = 1 each direction v is preconditioned by
 * one FAS V-cycle of Sec. 3 (the opts' levels, factors and smoothing counts) started at q_m on
 * F(q) - S_0 = 0 with S_0 = F(q_m) - e v: M^{-1} v = (V(q_m) - q_m)/e with e = pc_rel sqrt(N)
 * (||v|| = 1).
 * dtau_m follows eq. (31) from ||F(q_m)|| as in esdirk_stage_solve (dtau or CFL form), and the
 * blocks are rebuilt with the same rule (the coarse ones inside the first preconditioner V-cycle
 * of a refresh step). Arguments as esdirk_stage_solve, plus:
 *   nk        host options.
 *   work      device, at least nk_work_elems(levels[0], krylov_dim) doubles, caller-owned.
 *   stats     as esdirk_stage_solve, with n_vcycles = Newton steps and history[m] = ||F(q_m)||.
 *   n_krylov  host int32 or NULL: Krylov directions over all Newton steps (= preconditioner
 *             V-cycles and Jacobian products).
 * Synchronises the stream several times per direction (host dot products). Returns
 * PMG_E_NOT_CONVERGED after max_newton steps without r_m / r_0 <= tol_rel.
 */
typedef struct pmg_nk_opts {
  int32_t krylov_dim;    /* 1..32 */
  int32_t max_newton;    /* >= 0 */
  double eta;            /* >= 0 */
  double fd_rel;         /* > 0, e.g. 1e-3 at Ma 0.005 */
  double pc_rel;         /* > 0, e.g. 1e-3 */
  int32_t precondition;  /* 0 or 1 */
} pmg_nk_opts;

int64_t nk_work_elems(pmg_level L0, int32_t krylov_dim);   /* -1 for bad arguments */
pmg_status nk_stage_solve(const pmg_solve_opts* opts, const pmg_nk_opts* nk, double omega, double dt,
                          const double* qc_n, const double* const* R_prev, const double* a_row, int32_t n_prev,
                          double* q, double* work, pmg_solve_stats* stats, int32_t* n_krylov, void* stream);

/* Number of stages of an ESDIRK scheme id (3, 4 or 6), or 0 for an unknown id. */
int32_t esdirk_stages(int32_t scheme);
/* The Butcher matrix of an ESDIRK scheme id, row-major s x s into host A_out (s*s doubles; NULL
 * only queries s); returns s, or 0 for an unknown id. */
int32_t esdirk_butcher(int32_t scheme, double* A_out);

/*
 * Batches of independent cases (several meshes, degrees or flow conditions advanced together).
 *
 * pmg_batch_create copies the case options (the level and factor handles stay owned by the
 * caller and must outlive the batch; no two cases may share a level). The batch owns one HIP
 * stream per case (default priority) and a small pinned host buffer.
 * Errors: PMG_E_ARG (null, n_cases outside 1..64, shared levels), PMG_E_SHAPE (cases on different
 * devices), PMG_E_HIP, PMG_E_NOMEM.
 */
pmg_status pmg_batch_create(const pmg_solve_opts* cases, int32_t n_cases, pmg_batch* out);
pmg_status pmg_batch_destroy(pmg_batch B);
int32_t pmg_batch_size(pmg_batch B);

/*
 * esdirk_stage_solve_batched — esdirk_stage_solve for every case of the batch, with per-case
 * arguments (arrays of length n_cases; dt[c] <= 0 makes case c steady and its qc_n, R_prev, a_row,
 * n_prev entries unused; R_out may be NULL, or hold NULL entries; stats may be NULL or an array of
 * n_cases). The cases are forked from `stream`, solved concurrently on the batch's streams and
 * joined back into `stream`; every case stops at its own tolerance. Returns PMG_OK, or
 * PMG_E_NOT_CONVERGED if some case hit max_vcycles (its stats say which), or the first hard error.
 */
pmg_status esdirk_stage_solve_batched(pmg_batch B, const double* omega, const double* dt,
                                      const double* const* qc_n, const double* const* const* R_prev,
                                      const double* const* a_row, const int32_t* n_prev, double* const* q,
                                      double* const* R_out, pmg_solve_stats* stats, void* stream);

/*
 * esdirk_step_batched — one time step of ESDIRK scheme `scheme` (2 or 3) for every case, per-case
 * dt[c] > 0; q[c] in: q^n, out: q^{n+1}; work[c]: device scratch of esdirk_stages(scheme) states of
 * that case's finest level; stats: NULL or [n_cases][stages - 1] (case-major). Stage solves that
 * stop at max_vcycles continue with their last iterate, as in esdirk_step. Synchronises `stream`.
 */
pmg_status esdirk_step_batched(pmg_batch B, int32_t scheme, const double* dt, double* const* q, double* const* work,
                               pmg_solve_stats* stats, void* stream);

#ifdef __cplusplus
}
#endif

#endif /* PMGFR_H */
