/*
 * sph.h - C ABI of libsph, the MI355X (gfx950) implementation of the SPH
 * solid-body right-hand side of Schaefer et al. (2016), "A smooth particle
 * hydrodynamics code to model collisions between solid, self-gravitating
 * objects" (arXiv:1604.03290).
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 *  - Every array pointer is a DEVICE pointer owned by the caller (for example
 *    the data pointer of a contiguous torch tensor).  The library allocates no
 *    device memory and keeps no state between calls; scratch space is passed in
 *    as a caller-owned workspace whose size sph_workspace_bytes() returns.  Two
 *    exceptions: sph_rhs_noalloc works in a static device array of the library
 *    (for callers that cannot allocate), and the diagnostic timing table
 *    (sph_timing_*, off by default) keeps HIP events between calls.
 *  - Particle data are structure-of-arrays in double precision, one array per
 *    component, as in the paper's implementation section (section 3.5):
 *    positions x, y, z; velocities vx, vy, vz; density rho; mass m; deviatoric
 *    stress S in six arrays (xx, yy, zz, xy, xz, yz; S is symmetric).  The index
 *    of a particle in these arrays is its "user index".
 *  - Work is enqueued on the caller's HIP stream (a hipStream_t passed as
 *    void*, NULL = the null stream) and is asynchronous unless stated.  The
 *    int return value is the status of the host-side validation and of the
 *    launches: SPH_OK or a negative sph_status code.  sph_last_error() gives a
 *    message for the last failure on the calling thread.
 *  - Conditions that only the device can see (non-finite input, a particle that
 *    moved further than the grid's skin allows, non-positive density) raise a
 *    flag inside the workspace; sph_workspace_status() synchronises the stream
 *    and returns it.  Each entry point clears the flag of the workspace it is
 *    given when it starts.
 *  - h is the paper's smoothing length: the support radius of the cubic
 *    B-spline (section 3.1.1).  Particles a != b interact when their squared
 *    distance, formed as ((dx*dx + dy*dy) + dz*dz) with dx = x_b - x_a and every
 *    operation rounded to double, is strictly below h*h (section 3.5.2).
 */
#ifndef SPH_MI355X_H
#define SPH_MI355X_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum sph_status {
    SPH_OK = 0,
    SPH_ERR_INVALID_ARG = -1,   /* null pointer, n <= 0, h <= 0, non-finite parameter, ... */
    SPH_ERR_CAPACITY = -2,      /* an output array is too small; the required size is returned */
    SPH_ERR_WORKSPACE = -3,     /* workspace smaller than sph_workspace_bytes() */
    SPH_ERR_HIP = -4,           /* a HIP runtime call or launch failed */
    SPH_ERR_DOMAIN = -5,        /* device flag: non-finite input or non-positive density */
    SPH_ERR_NOT_IMPLEMENTED = -6,
    SPH_ERR_STALE_GRID = -7     /* device flag: a particle left its cell by more than skin/2 */
};

enum sph_precision {
    SPH_FP64 = 0,       /* every operation in double precision */
    SPH_FP32_COMP = 1   /* pair terms in single precision with Kahan-compensated single-
                           precision sums per particle; partner test, equation of state,
                           limiter and stress rate in double precision */
};

enum sph_op {
    SPH_OP_BUILD = 0,
    SPH_OP_NEIGHBOURS = 1,
    SPH_OP_RHS = 2,
    SPH_OP_ADJOINT = 3,
    SPH_OP_LEAPFROG = 4,
    SPH_OP_LEAPFROG_ADJOINT = 5,
    SPH_OP_PAIRS = 6,
    SPH_OP_GRAVITY = 7   /* ncells: inner-node capacity of the tree (<= 0: 2 n) */
};

/* Frozen candidate-pair list built by sph_build_pairs (the interaction list of
 * section 3.5.2 widened by the grid's skin): for every slot s, the slots whose
 * distance was below h + skin at build time.  Slots are grouped by 64; inside
 * group B the j-th candidate of slot s = 64 B + l is slot[block_start[B] + 64 j
 * + l] for j < count[s]; each group's lists are padded to its longest (the group's
 * steps: the largest count among its slots) with the slot itself (n - 1 for the
 * lanes of the last group past n), so every entry of those steps is a valid slot.
 * The group's room, block_start[B + 1] - block_start[B], is 64 times the largest
 * upper bound of its slots' counts and may exceed 64 times its steps; entries past
 * the steps are not written.  All arrays are device arrays owned by the caller. */
typedef struct {
    int64_t n;             /* slots */
    double radius;         /* h + skin at build time */
    double skin;           /* tolerated movement since the build: skin / 2 */
    int32_t *count;        /* [n] candidates per slot */
    int64_t *block_start;  /* [ceil(n / 64) + 1] first entry of each group; last = total */
    int32_t *slot;         /* [capacity] candidate slots, interleaved by 64 */
    int64_t capacity;
    double *x0;            /* [3 n] slot-ordered positions at build time (x, y, z per slot) */
    int32_t *partners;     /* [n] or NULL: partners of each slot at build time (distance
                              below the grid's h), counted by the fill */
} sph_pairs;

/* Uniform grid of cubic cells ("helping grid", section 3.5.2) produced by
 * sph_build_cells.  Cells are numbered by tiles of 4 x 4 x 4 cells (x fastest
 * inside a tile: ix % 4 + 4 (iy % 4) + 16 (iz % 4)), the 64 tiles of a block of
 * 16 x 16 x 16 cells in Morton order (bits of the tile coordinates interleaved x, y,
 * z from the lowest), blocks x fastest: c = 4096 (bx + Bx (by + By bz)) + 64 tile +
 * local, B = ceil(dims / 16) blocks per axis, so consecutive slots form compact
 * pieces of space;
 * particles outside the box [lo, lo + dims * cell) are binned into the nearest
 * boundary cell, which keeps every partner reachable.  The grid stays valid for
 * later positions as long as no particle has moved by more than skin / 2 since
 * the build (checked by sph_rhs / sph_rhs_adjoint / sph_neighbours). */
typedef struct {
    int64_t n;            /* particles binned */
    int32_t dims[3];      /* cells per axis */
    int64_t ncells;       /* 4096 Bx By Bz (cells of the whole blocks) */
    double lo[3];         /* lower corner of cell (0,0,0) */
    double cell;          /* cell edge length */
    double h;             /* largest support radius the grid serves */
    double skin;          /* displacement allowance: 2 x the tolerated movement */
    int32_t *perm;        /* device [n]: sorted slot -> user index; slots ordered by
                             (cell, user index) */
    int32_t *cell_start;  /* device [ncells + 1]: first slot of each cell; last = n */
    int32_t *cell_of;     /* device [n]: cell of each slot */
    const sph_pairs *pairs; /* host pointer, NULL until sph_build_pairs; when set, the
                             right-hand side, adjoint and leapfrog take candidates from
                             the list instead of sweeping the cells */
} sph_grid;

/* Particle state (inputs), all device arrays of length n, user order.  u, the
 * specific internal energy, is read by the Tillotson equation of state only and may
 * be NULL (zero).  d, the damage of the Grady-Kipp model (section 2.7, in [0, 1]),
 * may be NULL (intact material); with it the stress that enters the momentum
 * equation is sigma_d = -p^ I + (1 - d) f_Y S, p^ = p for p >= 0 and (1 - d) p
 * below.  flaw_ptr (int64, n + 1 entries, flaw_ptr[0] = 0, non-decreasing) and
 * flaw_eps (flaw_ptr[n] entries) list each particle's activation threshold
 * strains, ascending within a particle (section 3.2); they are read only for the
 * damage-rate outputs of sph_deriv and may be NULL otherwise.  The adjoints and the
 * leapfrog hold d fixed (no cotangent for it, no evolution). */
typedef struct {
    int64_t n;
    const double *x, *y, *z;
    const double *vx, *vy, *vz;
    const double *rho;
    const double *sxx, *syy, *szz, *sxy, *sxz, *syz;
    const double *m;
    const double *u;
    const double *d;
    const int64_t *flaw_ptr;
    const double *flaw_eps;
} sph_state;

/* Material and numerical constants (SI units).  h: support radius; rho0, c:
 * linear equation of state p = c^2 (rho - rho0) (section 2.5.1); mu: shear
 * modulus; Y0: von Mises yield stress (section 2.6); alpha, beta, eps_v:
 * artificial viscosity (section 3.1.3); rho_cut: pressure is set to zero where
 * rho / rho0 < rho_cut (tension cut-off of section 2.5.1; 0 disables it);
 * correction: 1 applies the correction tensor of section 3.1.6 (linear
 * consistency) to the velocity gradient that drives the stress rate, 0 uses the
 * standard gradient; eps_s, n_s, dmpd: artificial stress of section 3.1.4 (0
 * disables it): a particle with negative pressure contributes
 * zeta = -eps_s sigma / rho^2 to the momentum bracket, scaled by
 * (W(r) / W(dmpd))^n_s, dmpd in (0, h) being the mean particle distance of the
 * initial distribution; xsph: XSPH
 * factor in [0, 1] (section 3.1.5), used by the dx/dt output; eos: 0 the liquid
 * equation above, 1 Murnaghan (section 2.5.2, exponent n_M, K0 = rho0 c^2), 2
 * Tillotson (section 2.5.3, constants a_T .. E_cv; compressed form for rho >= rho0
 * or u <= E_iv, expanded form for rho < rho0 and u >= E_cv, linear in u between).
 * With eos 1 or 2 each particle's sound speed is the thermodynamic one,
 * c^2 = dp/drho|u + p / rho^2 dp/du|rho (floored at 0), and Pi uses the pair's mean
 * (the adjoint of one right-hand side takes both, with the gradient of u for
 * Tillotson; the leapfrog and its adjoint take Murnaghan and refuse Tillotson). */
typedef struct {
    double h, rho0, c, mu, Y0, alpha, beta, eps_v, rho_cut, correction;
    double eps_s, n_s, dmpd, xsph;
    double eos, n_M, a_T, b_T, A_T, B_T, E0_T, alpha_T, beta_T, E_iv, E_cv;
} sph_params;

/* Time derivatives (outputs) in user order.  rho_sum may be NULL.  du and
 * dx, dy, dz (all four NULL, or none) request the specific internal energy rate
 * (eq. energy_sph; the bracket holds -Pi* I as in the momentum equation, without
 * the artificial stress) and the particle velocity dx/dt with XSPH (section
 * 3.1.5: v_a + xsph sum_b 2 m_b / (rho_a + rho_b) (v_b - v_a) W_ab; = v_a when
 * xsph = 0).  dd3 and n_act (both NULL, or neither; the state's flaw
 * lists are then required) request the damage model's rate d(d^(1/3))/dt and the
 * number of activated flaws (section 3.2): with sigma_max the largest principal
 * value of sigma_d, the strain eps = sigma_max / ((1 - d) E) (infinite at d = 1),
 * E = 9 K mu / (3 K + mu), K = rho0 c^2 (A_T for Tillotson); n_act counts the
 * particle's thresholds below eps; dd3 = n_act c_g / R_s with
 * c_g = 0.4 sqrt((K + 4/3 (1 - d) mu) / rho) and R_s = (3 m / (4 pi rho))^(1/3),
 * and 0 once d n_tot >= n_act (the limiter d <= n_act / n_tot, n_tot the
 * particle's flaw count).  vgrad (NULL, or device [n 9], [n 15] with
 * params->correction = 1; SPH_FP64 only) receives the velocity gradient that the
 * pair sums form (section 3.1.6, before the correction), for sph_rhs_adjoint
 * (sph_deriv_cot.vgrad) to reuse: one record of m = 9 (15) values per slot, in the
 * grid's slot order, component i of slot s at vgrad[m s + i]: L row by row
 * (dv^x/dx, dv^x/dy, ..., dv^z/dz), then with the correction the moment matrix M
 * (xx yy zz xy xz yz).  rec (NULL, or device [n 16] doubles, either precision)
 * receives the operand records of the prepass (per slot, in the grid's slot order:
 * the pair operands of each particle, a layout internal to the library), for
 * sph_rhs_adjoint (sph_deriv_cot.rec) to reuse. */
typedef struct {
    double *ax, *ay, *az;
    double *drho;
    double *dsxx, *dsyy, *dszz, *dsxy, *dsxz, *dsyz;
    double *rho_sum;
    double *du;
    double *dx, *dy, *dz;
    double *dd3;
    int32_t *n_act;
    double *vgrad;
    double *rec;
} sph_deriv;

/* Cotangents of the derivatives (inputs of the adjoint), user order.  A NULL
 * pointer means a zero cotangent.  du and dx, dy, dz are the cotangents of the
 * energy rate and of dx/dt (XSPH) of sph_deriv.  vgrad is not a cotangent: NULL, or
 * the velocity gradient that sph_rhs (SPH_FP64) wrote into sph_deriv.vgrad for the
 * same grid, state and params, which the adjoint then reads instead of forming it
 * again (a reverse-mode caller keeps it from its forward call, as it keeps any
 * intermediate); a vgrad of another state gives wrong gradients, unchecked.  rec
 * likewise: NULL, or the records sph_rhs wrote into sph_deriv.rec for the same grid,
 * state and params; the adjoint then runs no prepass of its own (nor its check that
 * no particle has left its cell, which the forward call made). */
typedef struct {
    const double *ax, *ay, *az;
    const double *drho;
    const double *dsxx, *dsyy, *dszz, *dsxy, *dsxz, *dsyz;
    const double *rho_sum;
    const double *du;
    const double *dx, *dy, *dz;
    const double *vgrad;
    const double *rec;
} sph_deriv_cot;

/* Writable per-particle fields (no mass): used for gradients with respect to
 * the state (outputs of the adjoints; per stored component of S, an
 * off-diagonal entry standing for both of its matrix positions) and for the
 * final state of a trajectory.  Outputs are overwritten. */
typedef struct {
    double *x, *y, *z;
    double *vx, *vy, *vz;
    double *rho;
    double *sxx, *syy, *szz, *sxy, *sxz, *syz;
    double *u; /* gradient of u: written by sph_rhs_adjoint with the Tillotson
                  equation (required there), otherwise unused and may be NULL */
} sph_fields;

typedef sph_fields sph_state_grad;

/* Read-only per-particle fields (cotangents of a final state).  NULL = zero. */
typedef struct {
    const double *x, *y, *z;
    const double *vx, *vy, *vz;
    const double *rho;
    const double *sxx, *syy, *szz, *sxy, *sxz, *syz;
} sph_cfields;

/* Library version string. */
const char *sph_version(void);

/* Message describing the last failing call on this thread ("" if none). */
const char *sph_last_error(void);

/* Scratch bytes needed by an operation (enum sph_op) for n particles and
 * ncells cells (ncells is ignored by SPH_OP_RHS and SPH_OP_ADJOINT). */
size_t sph_workspace_bytes(int op, int64_t n, int64_t ncells);

/* Host-only: grid geometry for the box [lo, hi] at support radius h, skin and
 * cells_per_h (1 or 2): cell = (h + skin) (1 + 2^-40) / cells_per_h,
 * dims = max(1, ceil((hi - lo) / cell)), ncells = 4096 prod(ceil(dims / 16)) (the
 * cells of whole 16^3 blocks, see sph_grid).  Lets the caller size cell_start. */
int sph_grid_geometry(const double lo[3], const double hi[3], double h, double skin,
                      int cells_per_h, int32_t dims_out[3], int64_t *ncells_out,
                      double *cell_out);

/* Cell list of the particles (the paper's helping grid of section 3.5.2):
 * bins every particle into the grid given by sph_grid_geometry(lo, hi, h,
 * skin, cells_per_h), counting-sorts the slots by cell (one digit of radix
 * ncells) and orders each cell by user index, so the result is deterministic.
 *   x, y, z     device [n] positions (user order)
 *   perm        device [n] out; cell_of device [n] out
 *   cell_start  device [ncells_cap + 1] out
 *   grid_out    host struct, filled in (pointers are the caller's arrays)
 * Errors: INVALID_ARG (null pointer, n <= 0, n >= 2^31, h <= 0, skin < 0,
 * lo >= hi, cells_per_h not 1 or 2), CAPACITY (ncells > ncells_cap; grid_out->
 * ncells holds the required count), WORKSPACE.  Device flag DOMAIN for
 * non-finite positions. */
int sph_build_cells(const double *x, const double *y, const double *z, int64_t n,
                    const double lo[3], const double hi[3], double h, double skin,
                    int cells_per_h, int32_t *perm, int32_t *cell_start,
                    int64_t ncells_cap, int32_t *cell_of, sph_grid *grid_out,
                    void *ws, size_t ws_bytes, void *stream);

/* Frozen candidate-pair list for the grid's slots at the current positions
 * (the paper's interaction list of section 3.5.2, widened by the grid's skin so
 * it can be reused while particles move): a bound pass (each slot's bound: the
 * slots of the cells within reach of it, no distance test), per-group room and scan,
 * then one pass that tests the candidates and writes them.  Synchronises the stream
 * once to learn the size.
 *   out         host struct filled in; grid->pairs is set to out (keep it alive)
 *   count       device [n]; block_start device [ceil(n/64) + 1]
 *   partners    device [n] or NULL: receives each slot's partners at build time
 *               (distance below grid->h, the test sph_neighbours applies), so that
 *               sph_neighbours called with grid->h at these very positions (checked
 *               bit for bit) takes its row lengths from here instead of counting, and
 *               writes the rows whose candidates are all partners without testing them
 *   slot        device [capacity] (may be NULL when capacity is 0)
 *   x0          device [3 n] positions at build time (slot order)
 *   needed      host, receives the number of entries of room the list takes
 *               (64 times the largest bound of each group, summed)
 * Later calls flag SPH_ERR_STALE_GRID when a particle has moved by more than
 * skin / 2 since this build.  Errors: INVALID_ARG, CAPACITY (needed >
 * capacity; nothing is filled and grid->pairs is unchanged), WORKSPACE
 * (sph_workspace_bytes(SPH_OP_PAIRS, n, 0)), STALE_GRID (grid older than the
 * positions by more than its skin). */
int sph_build_pairs(sph_grid *grid, const double *x, const double *y, const double *z,
                    sph_pairs *out, int32_t *count, int32_t *partners, int64_t *block_start,
                    int32_t *slot, int64_t capacity, double *x0, int64_t *needed, void *ws,
                    size_t ws_bytes, void *stream);

/* Interaction partner lists (the paper's interactionsList of section 3.5.2)
 * at the current positions: row a of the CSR holds the user indices b of all
 * partners of user particle a, ascending, self excluded.
 *   row_ptr   device [n + 1] int64 out
 *   col       device [col_cap] int32 out
 *   nnz_out   host, receives the number of ordered pairs
 * Synchronises the stream once (to learn nnz).  Errors: INVALID_ARG (h > grid
 * h), CAPACITY (nnz > col_cap: nothing is written to col, *nnz_out holds the
 * requirement), WORKSPACE, STALE_GRID, DOMAIN. */
int sph_neighbours(const sph_grid *grid, const double *x, const double *y, const double *z,
                   double h, int64_t *row_ptr, int32_t *col, int64_t col_cap,
                   int64_t *nnz_out, void *ws, size_t ws_bytes, void *stream);

/* Right-hand side for every particle, with the partner set re-derived from
 * the grid at the current positions:
 *   prepass   p = c^2 (rho - rho0) (section 2.5.1); f_Y = min(Y0^2 / (3 J2), 1),
 *             J2 = S:S / 2 (section 2.6); sigma = -p I + f_Y S (section 2.2), or
 *             sigma_d with damage (section 2.7), and the damage rate outputs
 *   pairs     rho_sum_a = m_a W(0) + sum_b m_b W_ab  (eq. density_by_kernel_sum)
 *             L_a = sum_b (m_b/rho_b) (v_b - v_a) (x) grad_a W_ab  (section 3.1.6)
 *             a_a = sum_b m_b [sigma_a/rho_a^2 + sigma_b/rho_b^2 - Pi*_ab I] grad_a W_ab
 *             with the artificial viscosity Pi*_ab of section 3.1.3 (only for
 *             approaching pairs) and the B-spline of section 3.1.1
 *   postpass  drho_a = -rho_a tr L_a (eq. continuity_equation_sph);
 *             dS_a = 2 mu (edot - tr(edot) I / 3) + R S~ - S~ R with edot, R the
 *             symmetric and antisymmetric parts of L and S~ = f_Y S (section 2.4)
 * precision: enum sph_precision.  Outputs are overwritten (user order).
 * Errors: INVALID_ARG (state->n != grid->n, h > grid->h, non-finite or
 * non-positive h, c, rho0, negative mu or Y0, ...), WORKSPACE.  Device flags
 * STALE_GRID, DOMAIN (non-positive density; non-finite density, velocity or
 * stress; damage outside [0, 1]; flaw offsets out of order). */
int sph_rhs(const sph_grid *grid, const sph_state *state, const sph_params *params,
            int precision, const sph_deriv *out, void *ws, size_t ws_bytes, void *stream);

/* Largest particle count sph_rhs_noalloc serves. */
#define SPH_NOALLOC_MAX_N 262144

/* sph_rhs without a workspace, for callers that cannot allocate device memory
 * (code under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc).  Same outputs as sph_rhs (same kernels, bit for bit); its scratch is a
 * static device array of the library sized for SPH_NOALLOC_MAX_N particles (about
 * 53 MiB), which every device the library runs on holds until the process ends.  The
 * call allocates nothing (no hipMalloc, hipFree or allocating library routine); the
 * first call on a device looks up that device's copy of the array.
 *   status  device int32 or NULL: receives the call's device flag (SPH_OK, or
 *           SPH_ERR_STALE_GRID / SPH_ERR_DOMAIN as sph_workspace_status reports them
 *           for sph_rhs), written on the stream after the right-hand side
 * Every call on one device shares that device's scratch, and each call overwrites
 * it, so calls that overlap on one device (on different streams or threads) race:
 * serialise them.  Errors: as sph_rhs, and CAPACITY when grid->n exceeds
 * SPH_NOALLOC_MAX_N. */
int sph_rhs_noalloc(const sph_grid *grid, const sph_state *state, const sph_params *params,
                    int precision, const sph_deriv *out, int32_t *status, void *stream);

/* Vector-Jacobian product of sph_rhs in double precision: given
 * cotangents of (a, drho, dS, rho_sum) returns the gradients with respect to
 * positions, velocities, densities and stresses (masses are constants) and,
 * in dparams (device double[2], overwritten), with respect to mu and Y0.  The
 * partner set is the one sph_rhs uses at the same positions; every pair term
 * vanishes with its first derivative at distance h, so the product is exact.
 * Gather form: each particle sums its own terms from its partners' data; no
 * atomics, reproducible bit for bit.  With params->correction = 1 the
 * correction tensor C = M^-1 is differentiated too (M depends on positions and,
 * through V = m / rho, on densities); where C fell back to the identity M gets
 * no cotangent.  With the Murnaghan equation the pressure's slope and the sound
 * speeds in Pi are differentiated too; with Tillotson also (grad->u, user order,
 * overwritten) the gradient with respect to u, through the pressure and through the
 * sound speed, whose partials need the second derivatives of p (each region's form
 * differentiated, the region held; the floor of c^2 at 0 passes no gradient).  So is
 * the artificial stress (its tension switch held), and the energy rate and dx/dt when
 * their cotangents are given.  Errors as sph_rhs, and INVALID_ARG for Tillotson with
 * grad->u NULL. */
int sph_rhs_adjoint(const sph_grid *grid, const sph_state *state, const sph_params *params,
                    const sph_deriv_cot *cot, const sph_state_grad *grad, double *dparams,
                    void *ws, size_t ws_bytes, void *stream);

/* Self-gravity by the Barnes-Hut tree with monopoles (section 3.3, eq.
 * gravitational_force; the octree of section 3.5.1):
 *   tree      root cube of edge s0 = max over axes of (max x - min x) at the per-axis
 *             minima; a node of depth d has edge s0 / 2^d; the inner nodes are the
 *             cubes that hold two or more particles, the particles are the leaves.
 *             Octant membership uses q = floor((x - lo) / s0 * 2^21) clamped to
 *             [0, 2^21 - 1] (q = 0 when s0 = 0); depth 21 is the last, its cubes'
 *             particles are all leaves of it.  Children are ordered by octant
 *             4 bx + 2 by + bz (the axis bits of q at that depth).
 *   monopole  each inner node carries its total mass and centre of mass, summed over
 *             its children in that order (an inner child counts as m_c at x_c).
 *   walk      from the root in that order: an inner node with edge s and distance r
 *             from the particle to its centre of mass acts as one pseudo-particle
 *             when s / r < theta, tested as s^2 < theta^2 r^2, else its children are
 *             visited; every other leaf acts directly; each acting body p adds
 *             a += G m_p (x_p - x_a) / (r + eps)^3 (nothing at r = 0).
 *             theta = 0 gives the direct sum.
 * The keys, the monopoles and the opening tests are evaluated in double precision in
 * the order stated, without fused multiply-adds (so the tree and the bodies each
 * particle takes are fixed by the input); the force terms use reciprocal square roots
 * refined to double precision.  Results do not depend on the launch.
 *   x, y, z, m  device, n particles (user order), 1 <= n <= 2^26; m > 0
 *   G           gravitational constant; theta in [0, 1); eps >= 0 (the distance
 *               added to r, the paper's second smoothing scheme)
 *   ax, ay, az  device, n, overwritten
 *   count       device int32 [n] or NULL: bodies each particle took a term from
 *   node_cap    inner nodes the workspace holds (the ncells argument of
 *               sph_workspace_bytes(SPH_OP_GRAVITY, n, node_cap); <= 0: 2 n; at
 *               most 22 n, which no tree exceeds)
 *   nodes_out   host or NULL, receives the number of inner nodes
 * Synchronises the stream once (to learn the tree's size).  Errors: INVALID_ARG,
 * CAPACITY (more inner nodes than node_cap: nothing is written to the outputs,
 * *nodes_out holds the requirement), WORKSPACE, HIP.  Device flag DOMAIN for a
 * non-finite position or a mass that is not positive and finite. */
int sph_gravity(const double *x, const double *y, const double *z, const double *m, int64_t n,
                double G, double theta, double eps, double *ax, double *ay, double *az,
                int32_t *count, int64_t node_cap, int64_t *nodes_out, void *ws, size_t ws_bytes,
                void *stream);

/* Kick-drift-kick leapfrog that drives the gradient workloads (the paper's
 * own integrators are those of section 3.4).  With U = (v, rho, S) and
 * F = sph_rhs in double precision on the given (frozen) grid:
 *   F_0 = F(x_0, U_0); for n = 0 .. steps-1:
 *     U_{n+1/2} = U_n + dt/2 F_n,  then S <- f_Y(S) S
 *     x_{n+1}   = x_n + dt v_{n+1/2}
 *     F_{n+1}   = F(x_{n+1}, U_{n+1/2})
 *     U_{n+1}   = U_{n+1/2} + dt/2 F_{n+1},  then S <- f_Y(S) S
 *   s0           initial state (device arrays, user order)
 *   s_final      final state out (may alias the arrays of s0)
 *   checkpoints  device, sph_checkpoint_bytes(n, steps) bytes, or NULL; holds
 *                (x, v, rho, S, F) at the start of every step and at the end
 *                and the velocity gradient behind each F (with the correction
 *                tensor also its moment matrix), all in the grid's slot order (the trajectory is integrated in slot order), as
 *                needed by sph_leapfrog_adjoint, which must be given the same
 *                grid
 * The grid must have been built with a skin covering the trajectory's largest
 * displacement (device flag STALE_GRID otherwise).  Errors: as sph_rhs. */
int sph_leapfrog(const sph_grid *grid, const sph_state *s0, const sph_params *params,
                 double dt, int steps, const sph_fields *s_final, double *checkpoints,
                 void *ws, size_t ws_bytes, void *stream);

/* Reverse sweep of sph_leapfrog (the adjoint applied through the trajectory):
 * given the checkpoints of a forward run and the cotangent of the final state,
 * writes the gradient with respect to the initial state into grad0 and
 * (overwriting) dparams[0] = d/d mu, dparams[1] = d/d Y0 (device double[2]).
 * Deterministic.  Errors: as sph_rhs_adjoint. */
int sph_leapfrog_adjoint(const sph_grid *grid, const sph_state *s0, const sph_params *params,
                         double dt, int steps, const double *checkpoints,
                         const sph_cfields *cot_final, const sph_fields *grad0,
                         double *dparams, void *ws, size_t ws_bytes, void *stream);

/* Bytes of the checkpoint buffer of sph_leapfrog for n particles and steps steps. */
size_t sph_checkpoint_bytes(int64_t n, int steps);

/* Diagnostics.  When enabled, the library brackets its hot kernels with HIP
 * events recorded on the caller's stream ("pairs_fp64", "pairs_fp32comp",
 * "adjoint_pairs", ...).  sph_timing_read synchronises on the recorded events
 * and returns the summed duration in milliseconds and the number of launches
 * since the last reset.  Off by default.  Errors: INVALID_ARG, HIP. */
int sph_timing_enable(int on);
int sph_timing_read(const char *kernel, double *total_ms, int64_t *launches);
int sph_timing_reset(void);

/* Synchronise the stream and return the device flag of a workspace (SPH_OK or
 * a negative status).  Errors: INVALID_ARG, HIP. */
int sph_workspace_status(const void *ws, void *stream);

#ifdef __cplusplus
}
#endif

#endif /* SPH_MI355X_H */
