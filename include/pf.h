/*
 * pf.h -- C ABI of libpfrac, an explicit-dynamics phase-field fracture step
 * on 2D linear-triangle (P1) meshes for AMD Instinct MI355X (gfx950).
 *
 * The operations follow the matrix-free explicit phase-field method of
 * "A matrix-free, differentiable PyTorch solver for phase-field fracture"
 * (arXiv 2606.23458):
 *   - pf_mesh_create    P1 geometry and lumped mass precomputed once
 *                       (Sec. 2.3, eq. grad_phi and the lumped mass m_i);
 *   - pf_explicit_step  velocity-Verlet predictor, strain, energy split with
 *                       degradation g(d), internal force, corrector and the
 *                       history maximum (Sec. 2.1-2.3, eq. spectral_split,
 *                       eq. amor_split, eq. vv_u, eq. vv_a, eq. vv_v);
 *   - pf_damage_solve   the bound-constrained AT1/AT2 damage update by a
 *                       matrix-free projected preconditioned CG (Sec. 2.2,
 *                       eq. damage_pde_at2, eq. damage_pde_at1; Sec. 2.4);
 *   - pf_step_backward  the reverse (adjoint) of one staggered step, with
 *                       the damage solve differentiated implicitly
 *                       (Sec. 4.2, eq. implicit_adjoint_linear_system,
 *                       eq. implicit_gc_l0_element_term).
 *
 * Conventions shared by every entry point
 *   - Units are whatever the caller uses consistently (SI in the tests).
 *   - A mesh handle holds one or more independent instances ("batched"
 *     mode); n_instances = 1 is the plain case and takes the same path.
 *   - Device arrays are caller-owned, contiguous, of the mesh dtype (float
 *     for PF_F32, double for PF_F64) unless stated otherwise, and aligned
 *     to at least 16 bytes.  Node arrays have n_nodes_total entries in the
 *     mesh's INTERNAL node order; element arrays (the history H) have
 *     n_elems_total entries in the INTERNAL element order.  pf_mesh_node_perm
 *     and pf_mesh_elem_perm give the map from internal to the caller's ids.
 *     Instances occupy contiguous ranges (pf_mesh_instance).
 *   - Every entry point validates its arguments on the host first; on an
 *     argument error nothing is enqueued and PF_ERR_ARG is returned.
 *   - Work is enqueued on the given HIP stream and runs asynchronously.
 *     pf_damage_solve and pf_step_backward may synchronise that stream to
 *     test convergence (see pf_cg_opts_t.check_every).
 *   - None of pf_explicit_step, pf_damage_solve, pf_step_backward allocates
 *     memory: the workspaces are allocated by pf_mesh_create.
 *   - A handle is not safe for concurrent calls from several threads or
 *     streams; one call at a time per handle.
 *   - No C++ exception crosses this interface.  On a non-OK status,
 *     pf_last_error() returns a thread-local message.
 */
#ifndef PF_H
#define PF_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct pf_mesh_s* pf_mesh_t;
typedef void* pf_stream_t;   /* a hipStream_t; NULL is the null stream */

typedef enum {
    PF_OK = 0,
    PF_ERR_ARG = 1,            /* invalid argument (null pointer, size, enum, aliasing) */
    PF_ERR_MESH = 2,           /* invalid mesh (index out of range, zero-area triangle, unused node) */
    PF_ERR_HIP = 3,            /* a HIP runtime call failed; see pf_last_error() */
    PF_ERR_NOMEM = 4,          /* device or host allocation failed */
    PF_ERR_NOT_CONVERGED = 5,  /* CG reached max_iter; the last iterate is written */
    PF_ERR_NONFINITE = 6,      /* a non-finite value appeared in a CG reduction */
    PF_ERR_UNSUPPORTED = 7     /* combination not supported (e.g. mixed splits in one handle) */
} pf_status_t;

typedef enum { PF_F32 = 0, PF_F64 = 1 } pf_dtype_t;

enum { PF_AT1 = 1, PF_AT2 = 2 };
enum { PF_SPLIT_NONE = 0, PF_SPLIT_SPECTRAL = 1, PF_SPLIT_VOLDEV = 2, PF_SPLIT_STARCONVEX = 3 };
enum { PF_PLANE_STRAIN = 0, PF_PLANE_STRESS = 1 };
enum { PF_BOUNDS_PROJECTED = 0, PF_BOUNDS_POSTCLAMP = 1 };

/* stats.flags bits, and active_out bits */
enum { PF_FLAG_NOT_CONVERGED = 1, PF_FLAG_NONFINITE = 2 };
enum { PF_ACTIVE_LOWER = 1, PF_ACTIVE_UPPER = 2 };

/* One instance's mesh, host memory, read only during pf_mesh_create. */
typedef struct {
    int32_t n_nodes;
    int32_t n_elems;
    const double* xy;        /* [n_nodes][2] node coordinates */
    const int32_t* tri;      /* [n_elems][3] 0-based node ids, either orientation */
    const uint8_t* fixed;    /* [n_nodes][2] 1 = velocity-prescribed DOF; NULL = none */
} pf_mesh_desc_t;

/* Tile plan options; NULL selects the defaults. */
typedef struct {
    int32_t tile_nodes;      /* owned nodes per tile, 64..2048; 0 = default (512 in
                                FP32, 256 in FP64) */
    int32_t explicit_block;  /* workgroup size of the explicit-step kernel: 256 or 512;
                                0 = default (256) */
    int32_t explicit_chunks; /* element chunks of the explicit step per workgroup:
                                1, 2, or 0 = automatic (2 when halving the
                                corner-force space in LDS lets more workgroups
                                share a CU).  The result does not depend on it. */
    int32_t damage_chunks;   /* element chunks of the damage CG passes per
                                workgroup: 1, 2, or 0 = automatic (2 when halving
                                the corner-value space in LDS lets all of a
                                pass's workgroups be resident at once and one
                                chunk does not).  The result does not depend
                                on it. */
} pf_tile_opts_t;

/* Material and model of one instance (Sec. 2.1-2.2).  Geometry-independent. */
typedef struct {
    double E, nu, rho;       /* Young's modulus, Poisson ratio, density */
    double Gc, l0;           /* fracture energy, regularisation length */
    double eta;              /* residual stiffness in g(d) = (1-d)^2 + eta */
    double gamma_star;       /* star-convex parameter (split 3 only), >= 0 */
    int32_t model;           /* PF_AT1 | PF_AT2 */
    int32_t split;           /* PF_SPLIT_*; the same for every instance of a handle */
    int32_t plane;           /* PF_PLANE_STRAIN | PF_PLANE_STRESS */
    int32_t bounds;          /* PF_BOUNDS_PROJECTED | PF_BOUNDS_POSTCLAMP (AT2 only) */
} pf_params_t;

/* Device pointers to one state; node arrays [n_nodes_total], H [n_elems_total].
 * t is the time of the state, device double [n_instances] (the loading
 * ramps of pf_set_loading are functions of it); NULL where the caller keeps
 * no time (allowed unless loading is registered; adjoint states ignore it). */
typedef struct {
    void *ux, *uy, *vx, *vy, *ax, *ay, *d, *H;
    double* t;
} pf_state_t;

typedef struct {
    double tol;              /* stop when max_i |r_i|/A_ii <= tol on free nodes and
                                no node held at a bound has a scaled residual
                                r_i/A_ii pointing inward by more than tol/4
                                (held nodes beyond that are released) */
    int32_t max_iter;        /* CG rounds per solve, >= 1 (a round is one pass
                                over the tiles and one reduction; with the
                                Jacobi preconditioner one matrix-vector
                                product) */
    int32_t check_every;     /* > 0: synchronise the stream to stop early: first
                                after as many CG rounds as the handle's previous
                                solve of the same kind needed (8 on the first
                                solve), then every check_every rounds (the
                                default path); 1: after every round;
                                0: enqueue exactly max_iter rounds and never
                                synchronise (suitable for HIP-graph capture) */
    int32_t start;           /* damage solve: 0: start from d_prev;
                                1: start from clamp(2 d_prev - d, d_prev, 1),
                                where the output array d holds, on entry, the
                                damage of the step before d_prev (a linear
                                extrapolation in time).  pf_step_backward:
                                1: warm start from the multipliers of the
                                handle's previous calls; 0: start from zero and
                                forget them (the first call of a reverse sweep,
                                so that a sweep repeats a fresh handle's bits) */
    int32_t monotone;        /* damage solve only.  1: use the monotone
                                projected CG from the start instead of
                                held-set updates between CG runs (slower; the
                                solver falls back to it by itself when the
                                held set does not settle) */
    int32_t rounds;          /* check_every = 0 only: CG rounds to enqueue
                                (0 = max_iter); rounds of an instance that has
                                finished do nothing */
    int32_t resume;          /* damage solve only.  1: continue the solve left
                                unfinished by this handle's previous
                                pf_damage_solve call with the same arguments
                                (no set-up pass; iterate, held set and CG
                                scalars are kept).  Every call ends with the
                                final pass, so d, active_out and stats always
                                hold the current iterate.  With check_every = 0
                                and resume, a step can be captured once as a
                                HIP graph of a fixed number of rounds and
                                continued, rarely, by a second graph. */
    int32_t precond;         /* preconditioner of the CG runs.  0 or 1: Jacobi
                                (M = D^-1 on the free nodes).  2, 3 or 4: the
                                Chebyshev-Jacobi polynomial of that degree,
                                M = p(D^-1 A) D^-1, on the interval
                                [lmax/10, lmax] where lmax is a Gershgorin
                                bound of D^-1 A taken at set-up (so M is SPD);
                                a round then makes `precond` matrix-vector
                                products and one reduction, and max_iter and
                                the iteration counts of pf_cg_stats_t count
                                rounds.  Damage solve and adjoint alike. */
} pf_cg_opts_t;

/* Per-instance solve statistics, written to DEVICE memory by the solve. */
typedef struct {
    int32_t iters;           /* matrix-vector products */
    int32_t restarts;        /* active-set restarts */
    int32_t n_active;        /* nodes held at the lower bound at exit */
    int32_t flags;           /* PF_FLAG_* */
    double resid;            /* final scaled residual measure */
} pf_cg_stats_t;

typedef struct {
    int32_t node_offset, n_nodes;    /* internal node range of the instance */
    int32_t elem_offset, n_elems;    /* internal element range of the instance */
    int32_t tile_offset, n_tiles;
    double h_min;                    /* min incircle diameter 4 A_e / perimeter (Sec. 2.3, CFL) */
    double area;                     /* total area */
} pf_instance_info_t;

typedef struct {
    int32_t n_instances, n_nodes, n_elems, n_tiles;
    int32_t dtype;                   /* pf_dtype_t */
    int32_t max_tile_nodes, max_tile_elems;
    int32_t tile_elems_total;        /* element records incl. halo copies */
    size_t device_bytes;             /* device memory held by the handle */
    int32_t damage_chunks;           /* element chunks of the damage passes (1, 2) */
} pf_mesh_totals_t;

/*
 * Build a handle from n_instances meshes (Sec. 2.3: X, T given; grad phi,
 * A_e and the lumped mass m_i = rho sum A_e/3 are precomputed once in FP64
 * and stored in the handle's dtype).  Triangles are reoriented
 * counter-clockwise; a zero-area triangle, an index out of range or a node
 * used by no triangle gives PF_ERR_MESH.  Nodes are renumbered into tiles
 * of nearby nodes (recursive coordinate bisection) for the element kernels.
 * Allocates every device buffer the handle needs; synchronous on `stream`.
 * On success *out owns the handle (free it with pf_mesh_destroy).
 */
pf_status_t pf_mesh_create(const pf_mesh_desc_t* inst, int32_t n_instances, pf_dtype_t dtype,
                           const pf_tile_opts_t* tile, pf_stream_t stream, pf_mesh_t* out);

/* Release a handle and its device memory (synchronises the device first). NULL is ignored. */
pf_status_t pf_mesh_destroy(pf_mesh_t m);

pf_status_t pf_mesh_totals(pf_mesh_t m, pf_mesh_totals_t* out);
pf_status_t pf_mesh_instance(pf_mesh_t m, int32_t inst, pf_instance_info_t* out);

/* Host output [n_nodes_total]: internal node id -> the caller's node id within its instance. */
pf_status_t pf_mesh_node_perm(pf_mesh_t m, int32_t* out);
/* Host output [n_elems_total]: internal element id -> the caller's element id within its instance. */
pf_status_t pf_mesh_elem_perm(pf_mesh_t m, int32_t* out);

/*
 * One explicit step (Sec. 2.2 staggered scheme, first half; Sec. 2.3):
 *   u_{n+1} = u_n + dt v_n + dt^2/2 a_n                          (eq. vv_u)
 *   eps_e = sym grad u_{n+1};  d_e = (d_0 + d_1 + d_2)/3 of d_n
 *   sigma_e = g(d_e) sigma+(eps_e) + sigma-(eps_e),  g = (1-d)^2 + eta
 *   f_int,i = sum over corners of A_e sigma_e grad phi_k, gathered per node
 *             in a fixed order (no atomics: bitwise reproducible)
 *   a_{n+1} = m^-1 (f_ext - f_int) on free DOFs, 0 on prescribed DOFs (eq. vv_a)
 *   v_{n+1} = v_n + dt/2 (a_n + a_{n+1})                          (eq. vv_v)
 *   H_{n+1} = psi+(eps_e) if psi+ > H_n else H_n  (one value per element)
 * `p` and `dt` are host arrays with one entry per instance.  Reads in->{u,v,a,d,H};
 * writes out->{u,v,a,H}; out->d is not touched.  `in` and `out` must not share
 * any array.  When in->t and out->t are both given, out->t = in->t + dt (in
 * FP64).  f_ext is a device array [2][n_nodes_total] (x block, then y
 * block) or NULL for no external force.  Prescribed DOFs keep their
 * velocity (a must be 0 there in `in`), unless pf_set_loading registered
 * ramped loads: then in->t and out->t are required, f_ext must be NULL, the
 * external force is S(t_{n+1}) F and prescribed DOFs move with the ramped
 * velocity (see pf_set_loading), all evaluated inside the kernel from in->t,
 * so the step stays capturable in a HIP graph.
 */
pf_status_t pf_explicit_step(pf_mesh_t m, const pf_params_t* p, const double* dt,
                             const pf_state_t* in, pf_state_t* out, const void* f_ext,
                             pf_stream_t stream);

/*
 * Damage update (Sec. 2.2, eq. damage_pde_at2 / eq. damage_pde_at1; Sec. 2.4):
 * the minimiser of 1/2 d'Ad - b'd subject to d_prev <= d <= 1, with
 *   AT2: A = Gc l0 K + sum_e (Gc/l0 + 2 H_e) M^e,  b_i = sum 2 H_e A_e/3
 *   AT1: A = 3/4 Gc l0 K + sum_e 2 H_e M^e,        b_i = sum (2 H_e - 3 Gc/(8 l0)) A_e/3
 * K^e = A_e grad phi grad phi', consistent mass M^e_kl = A_e (1 + delta_kl)/12.
 * Solved matrix-free by Jacobi-preconditioned projected CG warm-started from
 * d_prev: CG runs on the free nodes with the held nodes frozen at their
 * bound, and the held set is updated between CG runs (primal-dual active-set
 * steps, with a monotone projected-CG fallback) until the KKT conditions hold
 * to tol.  Nodes with d_prev = 1 stay at 1.  In PF_BOUNDS_POSTCLAMP mode
 * (AT2) the CG is unconstrained and the result is clamped to [d_prev, 1].
 * H: device [n_elems_total]; d_prev: device [n_nodes_total]; d: device output
 * [n_nodes_total] (must not alias d_prev).  active_guess: device uint8
 * [n_nodes_total] whose PF_ACTIVE_* bits seed the held set (normally the
 * previous step's active_out), or NULL for an empty start; it only affects
 * the iteration count and the result within tol.  active_out: device uint8
 * [n_nodes_total] (PF_ACTIVE_* bits) or NULL; it may be the same array as
 * active_guess.  stats: device array of n_instances pf_cg_stats_t, or NULL.
 * Returns PF_ERR_NOT_CONVERGED / PF_ERR_NONFINITE only when check_every > 0
 * (otherwise read stats.flags); the last iterate is written in every case.
 */
pf_status_t pf_damage_solve(pf_mesh_t m, const pf_params_t* p, const void* H, const void* d_prev,
                            void* d, const uint8_t* active_guess, uint8_t* active_out,
                            const pf_cg_opts_t* opts, pf_cg_stats_t* stats, pf_stream_t stream);

/*
 * Reverse of one staggered step n -> n+1 (explicit step then damage solve).
 * Given the forward states s_n, s_np1 and active_np1 (the active_out of the
 * solve that produced s_np1->d), and the adjoints of s_np1 in adj_np1
 * (u, v, a, d, H), writes the adjoints of s_n into adj_n and adds
 * dL/dGc to dGc[inst] (device double, one per instance).  The damage solve
 * is differentiated implicitly: one adjoint CG solve with the same operator
 * restricted to the free nodes (Sec. 4.2), the Gc term
 * -(l0 lambda'K d + lambda'M d / l0) for AT2 (eq. implicit_gc_l0_element_term)
 * and its AT1 counterpart; nodes held at d_prev pass their adjoint to d_prev,
 * nodes held at 1 pass none.  The adjoint CG warm-starts from the linear
 * extrapolation of the previous two calls' multipliers held by the handle
 * (from the previous one on the second call); opts->start = 0 starts it from
 * zero and counts calls afresh (a fresh handle's first call starts from zero
 * too).  Projected bounds only.
 * adj_np1 is read only; adj_n must not alias adj_np1, s_n or s_np1.
 */
pf_status_t pf_step_backward(pf_mesh_t m, const pf_params_t* p, const double* dt,
                             const pf_state_t* s_n, const pf_state_t* s_np1,
                             const uint8_t* active_np1, const pf_state_t* adj_np1,
                             pf_state_t* adj_n, double* dGc, const pf_cg_opts_t* opts,
                             pf_cg_stats_t* stats, pf_stream_t stream);

/*
 * Energy budget of a state, per instance and per unit thickness (the energy
 * histories of Sec. 3, dynamic SENT; energies of Sec. 2.1-2.2):
 *   E_kin  = 1/2 sum_i m_i |v_i|^2 with the lumped mass,
 *   E_el   = sum_e A_e (g(d_e) psi+ + psi-),  d_e the element mean of d,
 *   E_frac = Gc (d'Md/(2 l0) + l0/2 d'Kd) (AT2),
 *            3 Gc/8 (int d / l0 + l0 d'Kd) (AT1).
 * Reads s->{u, v, d}.  out: device double [n_instances][3] = (E_kin, E_el,
 * E_frac); written on `stream` (sums in a fixed order, FP64).
 */
pf_status_t pf_energies(pf_mesh_t m, const pf_params_t* p, const pf_state_t* s, double* out, pf_stream_t stream);

/*
 * pf_energies for callers that cannot allocate device memory (code under
 * HIP-graph capture, tight serving loops, harnesses that forbid hipMalloc).
 * Same arguments, kernels, summation order and results as pf_energies, bit
 * for bit; the per-tile partial sums live in a fixed array of
 * 3 * PF_ENERGY_STATIC_MAX_TILES doubles (768 KiB) in device memory that the
 * library holds on each GPU it runs on until the process ends (its address is
 * resolved by pf_mesh_create, once per device).  The call allocates nothing,
 * on the device or through any library.
 *   - A handle with more than PF_ENERGY_STATIC_MAX_TILES tiles
 *     (pf_mesh_totals_t.n_tiles) is rejected with PF_ERR_ARG before anything
 *     is enqueued; use pf_energies for it.
 *   - Every call on one GPU shares that GPU's array: calls that overlap in
 *     time on one GPU (on different streams, or from several threads) race
 *     and must be ordered by the caller.  Each call writes every partial it
 *     reads, so nothing has to be cleared between calls.
 *   - As in pf_energies, new per-instance parameters are copied to the handle
 *     with a blocking copy (no allocation); repeated calls with the same
 *     parameters copy nothing.
 */
enum { PF_ENERGY_STATIC_MAX_TILES = 32768 };
pf_status_t pf_energies_static(pf_mesh_t m, const pf_params_t* p, const pf_state_t* s, double* out,
                               pf_stream_t stream);

/*
 * Spatially varying fracture toughness, Gc_e = Gc * phi_e per element (the
 * per-element Gc(x) inverse problem that Sec. 4 names as the next step; each
 * element's damage weak form, eq. damage_pde_at2 / damage_pde_at1, takes its
 * own Gc_e, and so does its share of E_frac in pf_energies).  The element
 * term of eq. implicit_gc_l0_element_term is then dL/dGc_e.
 *   phi: device [n_elems_total] in the internal element order (as H), mesh
 *        dtype, every value finite and > 0; copied into the handle, so the
 *        caller may free it on return.  NULL restores a uniform Gc (phi = 1).
 *   dgc_field: device double [n_elems_total] (internal order), caller-owned
 *        and kept alive while the handle uses it, or NULL.  Every later
 *        pf_step_backward adds dL/dGc_e to dgc_field[e] for each element e;
 *        its per-instance dGc output is then sum_e phi_e dL/dGc_e (the
 *        derivative along a common scaling of the field).
 * The explicit step does not depend on Gc.  A set-up call: the first call
 * with a field allocates n_te values of the mesh dtype in the handle; the
 * field is read back to the host and checked (PF_ERR_ARG names the first bad
 * element and leaves the previous field in place), and the call synchronises
 * `stream`.  Work already enqueued on other streams must be ordered before
 * this call by the caller; HIP graphs captured before the call are not
 * updated (capture them again).
 */
pf_status_t pf_set_gc_field(pf_mesh_t m, const void* phi, double* dgc_field, pf_stream_t stream);

/*
 * Ramped boundary loads of the explicit step (the loading protocols of
 * Sec. 3: eq. smooth_traction_ramp, eq. kalthoff_velocity_ramp).  With
 * t_n = in->t[k] and t_{n+1} = t_n + dt of instance k, every later
 * pf_explicit_step uses
 *   f_ext = S_k(t_{n+1}) F,  S(t) = 0 for t <= 0, (1 - cos(pi t / t_r))/2 for
 *           0 < t < t_r, 1 for t >= t_r  (t_r = t_traction[k]; t_r <= 0
 *           gives S = 1 for t > 0);
 *   v     = R_k(t_n + dt/2) v_full on the prescribed DOFs, R(t) = min(max(t, 0), t_v)/t_v
 *           (t_v = t_velocity[k]; t_v <= 0 gives R = 1); evaluated at the step
 *           midpoint, so u += dt v moves a prescribed DOF by the exact integral
 *           of the linear ramp over the step.  The velocity the step writes
 *           to out->v there is that value.
 *   F:       device [2][n_nodes_total] (x block, then y block) full-load
 *            nodal force, mesh dtype, or NULL for no traction.
 *   v_full:  device [2][n_nodes_total] velocity of the prescribed DOFs at
 *            full ramp (other entries are not read), mesh dtype, or NULL to
 *            keep the state's velocity on prescribed DOFs.
 *   t_traction, t_velocity: host double [n_instances], finite; NULL = zeros.
 * F and v_full are copied into the handle (the caller may free them on
 * return); the first call allocates 4 node vectors there.  F = v_full = NULL
 * clears the loading.  pf_step_backward then treats the prescribed
 * velocities as inputs of no adjoint.  A set-up call: it synchronises
 * `stream`; HIP graphs captured before it are not updated.
 */
pf_status_t pf_set_loading(pf_mesh_t m, const void* F, const void* v_full, const double* t_traction,
                           const double* t_velocity, pf_stream_t stream);

/*
 * CFL time step of every instance (Sec. 2.3): dt_k = factor * h_min,k / c_p,k
 * with c_p = sqrt((lambda + 2 mu)/rho) and lambda of the instance's plane.
 * dt_out is a host array of n_instances doubles.
 */
pf_status_t pf_cfl_dt(pf_mesh_t m, const pf_params_t* p, double factor, double* dt_out);

/*
 * Damage subcycling limit (Sec. 2.3, subcycling): the damage front moves at
 * most ~0.6 c_R while the explicit step resolves c_p, so solving the damage
 * sub-problem only every N_sub-th step is admissible for
 *     N_sub <= N_max = floor(c_p / (0.6 c_R)),
 * with c_p the plane's dilatational speed (as in pf_cfl_dt), c_s = sqrt(mu/rho)
 * and c_R the Rayleigh speed of the same 2D medium (root of the Rayleigh
 * equation).  Host outputs, one per instance: n_max_out (required) and the
 * continuous ratio c_p / (0.6 c_R) in ratio_out (NULL allowed).  The
 * subcycled schedule itself is the caller's: explicit steps every step (the
 * history H advances every step), pf_damage_solve on every N_sub-th.
 */
pf_status_t pf_subcycle_limit(pf_mesh_t m, const pf_params_t* p, int32_t* n_max_out, double* ratio_out);

/*
 * Tile-size autotuning (a set-up call, not part of the method; it allocates).
 * For each candidate owned-node count per tile it builds the tile plan of the
 * given meshes, times `reps` explicit steps from a zero state (with 256- and
 * with 512-thread workgroups, each with its elements in one and in two
 * chunks, keeping the fastest) and `reps` damage CG rounds (the launches of
 * one CG iteration, on a linear solve over all nodes), and scores the plan as
 *     explicit_us + cg_rounds_per_step * cg_round_us.
 * The smallest score wins; pass out->best, out->best_explicit_block and
 * out->best_explicit_chunks as pf_tile_opts_t.tile_nodes, .explicit_block
 * and .explicit_chunks.
 * Candidates whose tiles need more LDS than a workgroup may use are skipped
 * (status PF_ERR_UNSUPPORTED).  `inst`, `n_instances`, `dtype` and `p` are as
 * for pf_mesh_create and pf_explicit_step.  Synchronous on `stream`; the
 * result depends on the device, so callers cache it per size class.
 */
enum { PF_TUNE_MAX = 8 };

typedef struct {
    int32_t n_candidates;        /* entries of tile_nodes[] to try, 0..8; 0 = the default set
                                    {128, 192, 256, 384, 448, 512, 768, 1024} */
    int32_t tile_nodes[PF_TUNE_MAX];
    int32_t reps;                /* timed launches per candidate, 0..10000; 0 = 20 */
    double cg_rounds_per_step;   /* weight of one CG round in the score; <= 0 selects 16 */
} pf_tune_opts_t;

typedef struct {
    int32_t best;                       /* the chosen tile_nodes */
    int32_t best_explicit_block;        /* the chosen pf_tile_opts_t.explicit_block */
    int32_t n_tried;                    /* candidates tried (entries filled below) */
    int32_t tile_nodes[PF_TUNE_MAX];
    int32_t status[PF_TUNE_MAX];        /* pf_status_t of each candidate's plan */
    int32_t explicit_block[PF_TUNE_MAX];/* the faster explicit workgroup size (256, 512) */
    double explicit_us[PF_TUNE_MAX];    /* mean explicit-step time with that workgroup size
                                           and chunk count */
    double cg_round_us[PF_TUNE_MAX];    /* mean damage CG round time */
    double score_us[PF_TUNE_MAX];
    int32_t best_explicit_chunks;       /* the chosen pf_tile_opts_t.explicit_chunks */
    int32_t explicit_chunks[PF_TUNE_MAX];/* the faster element chunk count (1, 2) */
} pf_tune_result_t;

pf_status_t pf_tune_tiles(const pf_mesh_desc_t* inst, int32_t n_instances, pf_dtype_t dtype,
                          const pf_params_t* p, const pf_tune_opts_t* opts, pf_tune_result_t* out,
                          pf_stream_t stream);

/* Thread-local description of the last non-OK status on this thread. */
const char* pf_last_error(void);

/* Library version string. */
const char* pf_version(void);

/*
 * Kernel timing: when enabled, every kernel launch of this handle is
 * bracketed by HIP events on its stream.  pf_timer_read synchronises the
 * stream, returns the summed milliseconds and launch count of one kernel
 * family (0 explicit step, 1 damage CG passes, 2 damage set-up and final
 * passes, 3 adjoint kernels, 4 per-instance CG reductions) and resets that
 * family.
 */
pf_status_t pf_timer_enable(pf_mesh_t m, int32_t on);
pf_status_t pf_timer_read(pf_mesh_t m, int32_t family, double* total_ms, int64_t* launches);

/*
 * Throughput of the damage CG pass (a measurement aid, outside the solver):
 * enqueues n_passes >= 1 launches of the pass that the handle's last
 * pf_damage_solve call would run next, back to back on `stream`, with no
 * reduction in between.  H, d_prev and d are the device arrays that call
 * was given (same layout and ownership; the pass reads d_prev, the bounds).
 * The last call must have stopped mid-solve in a conjugate-gradient
 * iteration (check_every = 0 and a round budget the solve did not reach)
 * with the Jacobi preconditioner, and no pf_step_backward call may have run
 * on the handle since (its adjoint solve reuses the control blocks);
 * otherwise PF_ERR_ARG where the control blocks show it (the test reads them
 * back, a synchronisation of `stream`).  Each launch reads the
 * same current vectors and writes the same next ones, so every launch moves
 * the bytes of one iterate pass; the search direction is updated in place
 * each time, so the solve cannot be continued (resume) afterwards, and d
 * keeps the iterate the last call left.
 */
pf_status_t pf_damage_pass_repeat(pf_mesh_t m, const void* H, const void* d_prev, void* d, int32_t n_passes,
                                  pf_stream_t stream);

#ifdef __cplusplus
}
#endif
#endif /* PF_H */
