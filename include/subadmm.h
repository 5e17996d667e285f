/*
 * subadmm.h -- C ABI of the MI355X (gfx950) subsystem-based ADMM step library.
 *
 * The library computes one time step of the subsystem-based ADMM method of
 * Lee, Lee & Lee, "Modular and Parallelizable Multibody Physics Simulation via
 * Subsystem-Based ADMM" (arXiv 2302.14344), Algorithm 1: per-step construction of the
 * subsystem dynamics (Eq. (2), (6)) and constraints (Eq. (3)-(5)), the per-step
 * factorisation of A_i + beta_i J_c,i^T J_c,i (Eq. (15), penalty of Eq. (23)), and the
 * iteration x-update (Eq. (15)) -> residual (Eq. (22)) -> z-update (Eq. (16)-(21)) ->
 * dual update (Eq. (14)), all on the GPU.
 *
 * Conventions used throughout
 * ---------------------------
 * Precision: a problem is created in FP32 or FP64 (SUBADMM_F32 / SUBADMM_F64); every
 *   device array passed to or returned by it has that element type ("real" below).
 * Subsystem i has n_i DOF (1..64).  Subsystems of one scene are contiguous; so are the
 *   interfaces of one scene.  A scene is an independent problem that stops iterating on
 *   its own residual test.
 * Interface j has a kind, a dimension d_j (1..6; 3 for contacts, rows (normal, t1, t2)),
 *   one or two member subsystems (|S_j| = 1 intra-subsystem, 2 coupling) and a friction
 *   coefficient mu_j (contacts).  Constraint value: sum over members of the member's rows
 *   times its v_hat, plus e_j.
 * Slot rows: subsystem i owns one row per (interface j containing i, row k of j),
 *   ordered by ascending j then k; J_c,i of Eq. (9) stacks them.  z, u are per slot row.
 * Dense per-step arrays (all device memory, caller-owned):
 *   A      per subsystem a row-major n_i x n_i block, blocks concatenated (sum n_i^2);
 *   b      per subsystem n_i entries, concatenated (sum n_i; the "DOF" vector layout);
 *   J      per subsystem the row-major nc_i x n_i matrix of its slot rows (sum nc_i n_i);
 *   e      per interface its d_j rows, concatenated (sum d_j; the "row" layout);
 *   lambda same layout as e; constraint force of Eq. (2)/(8) (the impulse over the step
 *          is t * lambda).
 * Penalty: rho > 0 gives every subsystem beta_i = rho; rho <= 0 selects Eq. (23),
 *   beta_i = Tr(A_i)/Tr(J_c,i^T J_c,i) (beta_i = 1 for a subsystem with no slot rows).
 * Stopping test (per scene): r_theta = sqrt(theta)/max(|y^{l+1}|_2, 1e-12) <= tol, with
 *   theta of Eq. (22); or l + 1 = max_iters (returns OK with converged = 0).  On exit
 *   v_hat is that of the last x-update and lambda that of the last z-update.
 * Warm start: z^0, u^0 per slot row; y^0 := beta z^0 + u^0.
 * Streams: every call enqueues on the stream given to subadmm_bind and returns without
 *   synchronising, except subadmm_read_stats / subadmm_check (documented below).
 * Errors: every function returns an int status (enum subadmm_status) and never throws;
 *   subadmm_last_error() gives a message for the last failure on a problem.
 */
#ifndef SUBADMM_H
#define SUBADMM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum subadmm_status {
  SUBADMM_OK = 0,
  SUBADMM_E_ARG = -1,        /* invalid argument or descriptor */
  SUBADMM_E_NOT_SPD = -2,    /* a factorised matrix had a non-positive pivot */
  SUBADMM_E_NONFINITE = -3,  /* NaN/Inf reached the residual */
  SUBADMM_E_DEVICE = -4,     /* HIP runtime error */
  SUBADMM_E_WORKSPACE = -5,  /* not bound, or workspace too small */
  SUBADMM_E_STATE = -6       /* call out of order (e.g. model missing) */
};

enum subadmm_kind {
  SUBADMM_IF_EQUALITY = 0,   /* hard equality (Eq. (4) as an equation): lambda free */
  SUBADMM_IF_CONTACT = 1,    /* Signorini-Coulomb contact, Eq. (5)/(21) */
  SUBADMM_IF_HARD_INEQ = 2,  /* hard inequality, Eq. (17)/(19): 0 <= lambda _|_ value >= 0 */
  SUBADMM_IF_SOFT = 3        /* soft constraint, Eq. (3): lambda = -k (e + alpha J v_hat), with the
                              * z-update of Eq. (20); gain k and alpha from the interface.  In
                              * assembled problems, and in the rigid model as links
                              * (subadmm_rigid_set_links); the FEM model rejects it */
};

enum subadmm_dtype { SUBADMM_F32 = 0, SUBADMM_F64 = 1 };

enum subadmm_warm {
  SUBADMM_WARM_COLD = 0,     /* z^0 = u^0 = 0 */
  SUBADMM_WARM_PREV = 1,     /* final (z, u) of the previous solve/step of this problem */
  SUBADMM_WARM_GIVEN = 2,    /* z0, u0 arguments (device, slot layout) */
  SUBADMM_WARM_LEARNED = 3   /* rigid step only: networks attached with subadmm_set_warm_model
                                predict the change of (z, u) from the previous step's values;
                                scenes that do not reach tol from it are solved again from the
                                previous step's values (plain ADMM fallback) */
};

typedef struct subadmm_problem subadmm_problem;

typedef struct {
  int32_t n_dof;   /* DOF of the subsystem, 1..64 */
  int32_t scene;   /* scene index; non-decreasing over the subsystem list */
} subadmm_subsystem;

#define SUBADMM_MAX_MEMBERS 4

typedef struct {
  int32_t kind;    /* enum subadmm_kind */
  int32_t dim;     /* rows d_j, 1..6 (3 for contacts) */
  int32_t n_sub;   /* members |S_j|, 1..SUBADMM_MAX_MEMBERS (Sec. III-B: one for rows inside a
                    * subsystem, two or more for couplings; the z-update of Eq. 16-21 sums
                    * over all of them) */
  int32_t sub[SUBADMM_MAX_MEMBERS];  /* member subsystems, distinct, one scene (first n_sub used) */
  double mu;       /* friction coefficient (contacts) */
  double k;        /* soft interfaces: gain k_j >= 0 of Eq. (3) (ignored otherwise) */
  double alpha;    /* soft interfaces: alpha_j > 0 of Eq. (3) (ignored otherwise) */
} subadmm_interface;

typedef struct {
  int64_t n_dof, n_slot, n_rows;  /* sum n_i, sum nc_i, sum d_j */
  int64_t n_A, n_J;               /* sum n_i^2, sum nc_i n_i */
  int32_t n_sub, n_if, n_scene;
  int32_t max_dof, max_slot_sub, max_slot_scene;
} subadmm_sizes;

typedef struct {
  int32_t iters;        /* number of x-updates performed in the last solve/step */
  int32_t converged;    /* 1 if r_theta <= tol was reached */
  double theta;         /* Eq. (22) at exit */
  double r_theta;       /* relative residual at exit */
  int64_t iters_total;  /* x-updates summed over all solves/steps since bind or reset */
  int64_t unconverged_total; /* iteration runs that stopped at max_iters, since bind or reset */
  int64_t fallback_total;    /* learned-start runs redone from the previous step's values */
  /* ADMM's standard primal and dual residuals of the returned iterate (Boyd et al. 2011,
   * Sec. 3.3), with option SUBADMM_OPT_BOYD_RESIDUALS (NaN without it, and after FEM
   * steps): the z-update (Eq. 16-21) and dual update (Eq. 14) that would follow the last
   * x-update (Eq. 15), taken aside, give z', u'; r_prim = |x - z'| / max(|x|, |z'|) and
   * r_dual = |beta (z' - z)| / |u'| over the scene's slot rows (floors 1e-12), x the last
   * x-update's (the one v_hat comes from), z, u the returned ones.  Reported only: the
   * stop is decided by r_theta. */
  double r_prim;
  double r_dual;
} subadmm_stats;

/* Kernels timed by subadmm_timing_* (index into the ms array). */
enum subadmm_kernel {
  SUBADMM_K_ASSEMBLE = 0,  /* construction of A, b, J, e */
  SUBADMM_K_FACTOR = 1,    /* beta, factorisation, slot-space operators */
  SUBADMM_K_LOOP = 2,      /* the ADMM iteration */
  SUBADMM_K_ADVANCE = 3,   /* state update */
  SUBADMM_K_STEPS = 4,     /* the multi-step kernel (subadmm_rigid_steps: all of the above) */
  SUBADMM_K_WARM = 5,      /* learned start: features, networks and the (z, u) it gives */
  SUBADMM_NUM_KERNELS = 6
};

/* Creates a problem from host descriptors (copied).  Validates: 1 <= n_dof <= 768 (the
 * per-subsystem factorisation of subadmm_solve takes n_dof <= 512: in LDS while its FP64
 * working arrays, K, J and the nc + 1 right-hand sides, fit there, else in device memory
 * within the workspace; the rigid model takes n_dof <= 64; the FEM model up to 768),
 * scenes non-decreasing and contiguous, interfaces grouped by scene in scene order,
 * members in range and in the interface's scene, 1 <= dim <= 6, contact dim == 3,
 * mu >= 0.  rho: see "Penalty".  dtype: enum subadmm_dtype.  Returns E_ARG on any
 * violation (message in subadmm_last_error(NULL) when *out could not be created). */
int subadmm_setup(const subadmm_subsystem* subs, int32_t n_sub, const subadmm_interface* ifs,
                  int32_t n_if, double rho, int32_t dtype, subadmm_problem** out);

enum subadmm_option {
  /* Arithmetic of the per-step factorisation (Alg. 1 factorisation step and the slot-
   * space operators derived from it): 1 = FP64 (default), 0 = the problem's dtype.  With
   * an FP32 problem the iteration always runs in FP32; FP64 here keeps the rounding of
   * the per-step operator, which the coupled constraint system amplifies, out of the
   * constraint forces. */
  SUBADMM_OPT_FACTOR_FP64 = 1,
  /* Form of the iteration kernel: 0 (default) = one thread per slot row and per
   * interface, two barriers per iteration; 1 = one lane team per interface inside a
   * wave, one barrier per iteration, used when the scene's operators fit in LDS; 2 = one
   * wave per scene, each lane owning up to four slot rows and one interface, no
   * workgroup barrier (E_ARG unless every scene has at most 256 slot rows and 64
   * interfaces and its operators fit in LDS).  All compute the same iteration; which is
   * fastest depends on the scene shape. */
  SUBADMM_OPT_TEAM_KERNEL = 2,
  /* Iteration budget of the learned-start run of SUBADMM_WARM_LEARNED: 0 (default) =
   * max_iters, else min(value, max_iters).  Scenes that do not reach tol within it are
   * solved again from the previous step's values with max_iters. */
  SUBADMM_OPT_LEARNED_BUDGET = 3,
  /* Factorisation size classes: 1 (default) = run concurrently on streams forked from the
   * bound stream and joined back into it; 0 = one after another on the bound stream. */
  SUBADMM_OPT_FACTOR_STREAMS = 4,
  /* FEM-block iteration (FP32 problems): 1 (default) = each workgroup keeps its block's
   * operator in registers and LDS for the whole step, when every block's operator fits
   * and all workgroups can be resident; 0 = the operator is read from device memory in
   * every iteration.  Both compute the same products in the same order. */
  SUBADMM_OPT_FEM_RESIDENT = 5,
  /* Thread-per-slot-row iteration kernel (SUBADMM_OPT_TEAM_KERNEL = 0): 1 = the product
   * H_i w_i of a slot row whose subsystem has many slot rows is split over 2 or 4 lanes
   * (more than 4 or 8 vectors of 16 bytes per row), when every scene's lanes fit one
   * workgroup (which may grow); 2 = the same within the default workgroup: per scene the
   * subsystems with the longest rows first take 2, then 4 lanes per row (more than 2, then
   * 8 vectors) while the scene's lanes fit (the multi-step launch, subadmm_rigid_steps,
   * takes this form too); 0 (default) = one or two lanes per row for the whole scene.  Same
   * iteration; the partial sums of a split row are added in a fixed order. */
  SUBADMM_OPT_SPLIT_ROWS = 6,
  /* Contact z-update (Eq. 21), for every solve and step of the problem: 0 (default) = the
   * exact Signorini-Coulomb projection (normal and tangential parts decouple in the scalar
   * metric of the z-subproblem); 1 = the relaxed convex model the paper names in its
   * convergence discussion, the Euclidean projection onto the friction cone
   * {|lambda_t| <= mu lambda_n}: its fixed point has lambda in that cone and the
   * constraint velocity in the dual cone, so a sliding contact separates slightly. */
  SUBADMM_OPT_CONTACT_MODEL = 7,
  /* Iteration path of subadmm_solve / subadmm_rigid_step: 0 (default) = one workgroup per
   * scene (the kernel forms above) when every scene fits it (at most 512 slot rows and 512
   * interfaces, slot vectors in LDS), else the large-scene path; 1 = always the large-scene
   * path; 2 = always its phase form.  The large-scene path keeps the slot vectors and reads
   * the operators in device memory.  Scenes of at most 2048 slot rows run it with one
   * workgroup per scene in one launch (workgroup barriers between the phases); larger ones
   * (single coupled scenes of thousands of subsystems) run one launch per phase of each
   * iteration over all scenes (x-update per slot row, residual and stopping test per
   * scene, z-update per interface), and eager steps stop launching once every scene has
   * stopped (checked every 32 iterations).  Both forms compute the same iteration bit for
   * bit; scenes stop independently.  The learned start and subadmm_rigid_steps need the
   * per-scene kernel. */
  SUBADMM_OPT_LARGE_PATH = 8,
  /* 1 = after every solve and rigid step (subadmm_solve, subadmm_solve_scratch,
   * subadmm_rigid_step, its graph form, and the last step of subadmm_rigid_steps) one
   * more kernel forms the statistics' r_prim and r_dual from the returned (z, u) and the
   * step's operators (an x-update and a z-update per scene, in the solve's precision,
   * sums in FP64); 0 (default) = not formed (NaN in the statistics).  FEM steps do not
   * form them. */
  SUBADMM_OPT_BOYD_RESIDUALS = 9,
  /* Precision of the FEM blocks' factorisation (FP32 problems; FP64 problems always factor
   * in FP64; the paper does not state its arithmetic): FP64 for the stiffest blocks only.
   * 0 (default) = every block in FP64; k > 0 = an FP32 trial factorisation of every block
   * (FP32 matrix cores) gives kappa_est = (max_r L_rr / min_r L_rr)^2, a lower bound on the
   * condition number of the block's K = A + beta J^T J; blocks with kappa_est > k, or a
   * pivot that is not positive, are factorised again in FP64, the others keep their FP32
   * factors (stored as FP32).  The per-block outcome: subadmm_fem_block_precision.  An
   * FP32 factor of an n-DOF block carries a backward error of order n eps32 whatever its
   * condition (2.2e-5 at n = 375), which the iteration's result inherits. */
  SUBADMM_OPT_FEM_KAPPA_MAX = 10,
  /* lambda output of the steps (subadmm_rigid_step, its graph form, subadmm_rigid_steps,
   * subadmm_fem_step and its graph form): 0 (default) = the constraint force lambda of
   * Eq. (2); 1 = the impulse over the step, t lambda (Eq. (2) at force level, scaled by the
   * step's t).  subadmm_solve, which has no t, always returns lambda. */
  SUBADMM_OPT_IMPULSE_OUTPUT = 11
};

/* Sets an option of enum subadmm_option; E_ARG for an unknown option or bad value. */
int subadmm_set_option(subadmm_problem* p, int32_t option, int64_t value);

/* Sizes of the dense arrays of the layout above. */
int subadmm_get_sizes(const subadmm_problem* p, subadmm_sizes* out);

/* Rigid-box model for subadmm_rigid_step / subadmm_rigid_assemble (Eq. (2), maximal
 * coordinates; host arrays, FP64, copied).  Body k belongs to subsystem body_sub[k] at
 * 6-DOF block body_local[k]; its generalised velocity is (v world frame, omega body
 * frame), M = diag(m I3, diag(inertia)), the weight m g acts along -z.
 * Joints (revolute, 5 rows): bodies joint_body[2q], [2q+1]; anchors joint_anchor[6q..]
 * (body a frame, then body b frame); joint_frame_a[9q..] rows (h, u, v) orthonormal in
 * body a's frame (h the hinge axis); joint_axis_b[3q..] the hinge axis in body b's
 * frame; joint_if[q] its interface (kind equality, dim 5, members = subsystems of a and
 * b, or one member when both lie in one subsystem).  Rows: anchor velocity difference
 * along world x, y, z; relative world angular velocity along R_a u, R_a v.  Errors:
 * Baumgarte gamma * phi / t (phi: anchor separation; (R_a u, R_a v) . (R_b h_b x R_a h)).
 * Contacts (plane z = 0, 3 rows (e_z, e_x, e_y)): body contact_body[q], point
 * contact_point[3q..] (body frame), interface contact_if[q] (kind contact, one member);
 * error (gap/t, 0, 0).  Every interface is a joint, a contact or a link (set before with
 * subadmm_rigid_set_links).  Must precede subadmm_workspace_bytes/subadmm_bind. */
int subadmm_rigid_set_model(subadmm_problem* p, int32_t nb, const int32_t* body_sub,
                            const int32_t* body_local, const double* mass, const double* inertia,
                            int32_t nj, const int32_t* joint_body, const double* joint_anchor,
                            const double* joint_frame_a, const double* joint_axis_b,
                            const int32_t* joint_if, int32_t ncon, const int32_t* contact_body,
                            const double* contact_point, const int32_t* contact_if,
                            double gravity, double baumgarte);

/* Links of the rigid model: constraint rows between two bodies, or on one body, along
 * directions fixed in the first body's frame; to be called before subadmm_rigid_set_model
 * (which checks the bodies and members).  Link q (host arrays, copied): link_type[q] 0 =
 * linear (the velocity of the anchor point of body a minus that of body b along each
 * direction), 1 = angular (the world angular velocity of a minus that of b along each
 * direction); bodies link_body[2q], [2q+1] (-1: rows on body a alone, with no error: a
 * velocity-level, e.g. non-holonomic, constraint); anchors link_anchor[6q..] (a's frame,
 * then b's); link_frame[9q..] rows f_0, f_1, f_2 in a's frame, the first d_j used;
 * interface link_if[q] (1 to 3 rows; members: the bodies' subsystems, one member when
 * both lie in one subsystem or b = -1).  With phi_k = (x_a - x_b) . R_a f_k (linear,
 * x the anchor points) or -f_k . log(R_a^T R_b) (angular) the interface's kind sets e:
 * soft (Eq. 3) e = phi, so lambda = -k (phi + alpha J v_hat) (a spring at the step's
 * midpoint for alpha = t/2); equality or hard inequality (Eq. 4) e = gamma phi / t; contact
 * (Eq. 5, three linear rows normal, tangent, tangent, two bodies) e = (phi_0 / t, 0, 0).
 * link_type[q] = 2: a sphere contact (contact interface, 3 rows): radius r_a in
 * link_anchor[6q]; two bodies: radius r_b in link_anchor[6q+3], normal n = (x_a - x_b) /
 * |x_a - x_b| from the centres, gap |x_a - x_b| - r_a - r_b, tangents t1 = the world axis least
 * aligned with n made orthogonal to n and normalised, t2 = n x t1; one body (-1): a plane whose
 * world normal and tangents are link_frame[9q..] rows 0, 1, 2 and whose offset is
 * link_anchor[6q+3], gap n . x_a - offset - r_a.  The contact points sit on the spheres along
 * n (-r_a n from a's centre, +r_b n from b's); each row is the relative velocity of the two
 * contact points along n, t1, t2 (the contact frame follows the bodies each step).
 * link_if[q] = -1: a soft link between two bodies of one subsystem folded into that
 * subsystem's own dynamics (the option of the remark after Eq. 6) instead of an interface:
 * link_dim[q] rows (1 to 3), gain link_k[q] >= 0 and link_alpha[q] > 0 of Eq. 3, and
 * construction adds k alpha J^T J to A_i and -k J^T phi to b_i.  link_dim, link_k and
 * link_alpha are read only for such links (NULL when there are none). */
int subadmm_rigid_set_links(subadmm_problem* p, int32_t nl, const int32_t* link_type, const int32_t* link_body,
                            const double* link_anchor, const double* link_frame, const int32_t* link_if,
                            const int32_t* link_dim, const double* link_k, const double* link_alpha);

/* Device workspace the library needs (bytes, 256-byte aligned start required). */
size_t subadmm_workspace_bytes(const subadmm_problem* p);

/* Binds caller-allocated device memory (ownership stays with the caller; it must
 * outlive the problem's use) and a HIP stream (hipStream_t; NULL = default stream),
 * uploads the topology/model tables and synchronises the stream once.  Rebinding is
 * allowed.  E_WORKSPACE if bytes < subadmm_workspace_bytes(p). */
int subadmm_bind(subadmm_problem* p, void* dev_workspace, size_t bytes, void* hip_stream);

/* Per-step solve of an assembled problem (Algorithm 1 without the construction
 * steps): factorises A_i + beta_i J_c,i^T J_c,i (Eq. (15), (23)) and iterates
 * Eq. (15) -> Eq. (22) -> Eq. (16)-(21) -> Eq. (14) per scene until the stopping test.
 * Inputs A, b, J, e: device, layout above.  warm: enum subadmm_warm (z0/u0 device
 * arrays used only for SUBADMM_WARM_GIVEN).  Outputs (device, may be NULL): v_hat (DOF
 * layout), lambda (row layout), z_out/u_out (slot layout, final z^l, u^l).  The final
 * (z, u) are also kept for SUBADMM_WARM_PREV. */
int subadmm_solve(subadmm_problem* p, const void* A, const void* b, const void* J, const void* e,
                  int32_t max_iters, double tol, int32_t warm, const void* z0, const void* u0,
                  void* v_hat, void* lambda, void* z_out, void* u_out);

/* subadmm_solve for callers that cannot allocate device memory (code under stream capture,
 * tight serving loops, harnesses that forbid hipMalloc): the same factorisation and
 * iteration kernels, with the problem's tables and per-step arrays placed in a static
 * device array of the library (SUBADMM_SCRATCH_BYTES = 32 MiB per GPU, held by every GPU
 * the library runs on until the process ends) instead of a bound workspace.  Needs only
 * subadmm_setup (a bound workspace, if any, is left untouched and stays in use for the
 * other calls).  Each call uploads the tables from host memory, clears the rest of the
 * array, and runs on hip_stream (hipStream_t; NULL = default stream); the factorisation
 * size classes run one after another on it.  Calls no allocating routine.  Inputs and
 * outputs as subadmm_solve; warm COLD or GIVEN only.  stats_out (host, n_scene entries,
 * may be NULL) receives the per-scene statistics and then the call synchronises the
 * stream.  E_WORKSPACE if subadmm_workspace_bytes(p) exceeds SUBADMM_SCRATCH_BYTES.
 * Every call on one GPU shares that GPU's array and overwrites it: calls that overlap on
 * one GPU (other streams, other threads) race and must be serialised by the caller. */
#define SUBADMM_SCRATCH_BYTES ((size_t)32 << 20)
int subadmm_solve_scratch(subadmm_problem* p, void* hip_stream, const void* A, const void* b, const void* J,
                          const void* e, int32_t max_iters, double tol, int32_t warm, const void* z0,
                          const void* u0, void* v_hat, void* lambda, void* z_out, void* u_out,
                          subadmm_stats* stats_out);

/* Construction steps of Algorithm 1 for the rigid model (Eq. (2)-(5)) at state
 * (pos[3k], rot[9k] row-major world-from-body, vel[3k], omega[3k]; device, real):
 * writes A, b, J, e (device, layout above).  For checking the assembly on its own. */
int subadmm_rigid_assemble(subadmm_problem* p, const void* pos, const void* rot, const void* vel,
                           const void* omega, double dt, void* A, void* b, void* J, void* e);

/* One whole time step of Algorithm 1 for the rigid model: construction, factorisation,
 * iteration, and the state update of Eq. (2): v+ = 2 v_hat - v, p+ = p + t v_hat_lin,
 * R+ = R exp(t [omega_hat]x).  pos/rot/vel/omega (device, real) are updated in place.
 * Optional outputs v_hat (DOF layout) and lambda (row layout). */
int subadmm_rigid_step(subadmm_problem* p, void* pos, void* rot, void* vel, void* omega, double dt,
                       int32_t max_iters, double tol, int32_t warm, void* v_hat, void* lambda);
/* subadmm_rigid_step replayed from a HIP graph: the first call with a given set of
 * arguments captures the step's launches on the bound stream (stream capture, so the
 * factorisation streams forked from it are captured too), later calls with the same
 * arguments replay the graph; other arguments capture again, and so does the first call
 * after subadmm_set_option, subadmm_set_warm_model or subadmm_set_recording on this
 * problem, or after subadmm_mlp_bind / subadmm_mlp_set_input_affine on an attached
 * network.  Same results as subadmm_rigid_step; per-kernel timing is not recorded in
 * graph replays.  The graph holds the pointers it was captured with: their memory must
 * stay valid. */
int subadmm_rigid_step_graph(subadmm_problem* p, void* pos, void* rot, void* vel, void* omega, double dt,
                             int32_t max_iters, double tol, int32_t warm, void* v_hat, void* lambda);

/* n_steps whole time steps of Algorithm 1 for the rigid model in one launch, with the
 * results of n_steps calls of subadmm_rigid_step with the same warm mode (COLD: every step
 * starts cold; PREV: every step starts from the previous step's final values, the first
 * from those kept by the problem's last solve or step).  Each scene is carried through its
 * steps by one workgroup without waiting for the other scenes between steps, so the launch
 * takes as long as the scene whose iterations summed over the steps are the most, not the
 * sum over the steps of each step's slowest scene.  The factorisation and iteration are the
 * per-step kernels' (thread-per-slot-row form, rows not split; the options of the iteration
 * kernel form do not apply).  Statistics: iters, converged, theta and r_theta of the last
 * step; the totals count every step.  v_hat and lambda (optional) receive the last step's
 * values.  E_ARG for another warm mode or n_steps < 1. */
int subadmm_rigid_steps(subadmm_problem* p, void* pos, void* rot, void* vel, void* omega, double dt,
                        int32_t n_steps, int32_t max_iters, double tol, int32_t warm, void* v_hat, void* lambda);

/* Order in which subadmm_rigid_steps hands the scenes to its workgroups (order[k] = the
 * scene of workgroup k; host array, a permutation of 0..n_scene-1, copied; NULL restores
 * the identity).  Workgroups are dispatched over the XCDs and CUs in this order, so it
 * decides which scenes share a CU: the scenes that take the most iterations first spread
 * them over the CUs.  Results do not depend on it.  Synchronises the bound stream. */
int subadmm_set_scene_order(subadmm_problem* p, const int32_t* order);

/* Accuracy measure of a step (the constraint error of the paper's evaluation, Sec. IV,
 * which names the measure and the Fischer-Burmeister function for contacts): for the
 * step's v_hat and lambda (device, the problem's layout), per interface j with
 * c_j = sum_i J_i,j v_hat_i + e_j and w_j = sum_i 1/beta_i (the z-update's metric, beta of
 * the last solve/step) the residual of its law: equality |c_j|; hard inequality
 * FB(c_j, w_j lambda_j) per row, FB(a, b) = a + b - sqrt(a^2 + b^2); soft
 * w_j |lambda_j + k_j (e_j + alpha_j (c_j - e_j))|; contact sqrt(FB(c_n, w lambda_n)^2 +
 * |w lambda_t - P(w lambda_t - c_t)|^2) with P the projection onto the disc of radius
 * mu w lambda_n.  host_out[s] (n_scene doubles) = sqrt(sum over the scene's interfaces whose
 * kind k has bit (1 << k) set in `kinds` of the squares), computed in FP64; SUBADMM_ERR_LAWS
 * takes the interfaces with a feasibility law (equality, contact, hard inequality),
 * SUBADMM_ERR_SOFT the soft couplings.  J, e: the step's arrays (subadmm_solve layout), or
 * both NULL for those of the last rigid or FEM step of the problem's model.  Synchronises the
 * bound stream. */
#define SUBADMM_ERR_LAWS 7
#define SUBADMM_ERR_SOFT 8
int subadmm_constraint_error(subadmm_problem* p, const void* J, const void* e, const void* v_hat,
                             const void* lambda, int kinds, double* host_out);

/* Copies the per-scene statistics of the last solve/step to host memory (n_scene
 * entries); synchronises the bound stream. */
int subadmm_read_stats(subadmm_problem* p, subadmm_stats* host_out);

/* Zeroes the iters_total and unconverged_total counters (enqueued on the bound stream). */
int subadmm_reset_totals(subadmm_problem* p);

/* Measurement support: between timing_begin and timing_end every kernel launch of this
 * problem is bracketed by HIP events recorded on the bound stream (no synchronisation).
 * timing_end synchronises the stream and writes, per enum subadmm_kernel, the summed
 * kernel time in milliseconds (ms_out[SUBADMM_NUM_KERNELS]) and launch count
 * (count_out[SUBADMM_NUM_KERNELS]).  max_launches bounds the number of timed launches
 * (E_ARG if exceeded at timing_end; later launches are not timed). */
int subadmm_timing_begin(subadmm_problem* p, int32_t max_launches);
int subadmm_timing_end(subadmm_problem* p, double* ms_out, int32_t* count_out);

/* Per-subsystem beta_i of the last solve/step (device, real, n_sub entries). */
int subadmm_copy_beta(subadmm_problem* p, void* dev_out);

/* Device-side error flags raised by kernels since the last check (non-positive pivot,
 * non-finite residual).  Synchronises the bound stream; returns OK, E_NOT_SPD or
 * E_NONFINITE and clears the flags. */
int subadmm_check(subadmm_problem* p);

/* ------------------------------------------------------------------------------------
 * Warm-start network (learned initial z, u).  Not part of the paper: the network maps
 * per-interface features to the change of (z, u) relative to the previous step's final
 * values; plain ADMM remains the method and the fallback.
 *
 * A network has n_layers linear layers with widths[0..n_layers] (each 1..1024), ReLU
 * after every layer but the last.  Parameters (FP32, "parameter layout"): per layer k,
 * W_k (widths[k+1] x widths[k], row-major) then b_k (widths[k+1]).  Products run on the
 * matrix cores with BF16 operands (weights and activations rounded to nearest even) and
 * FP32 accumulation; the FP32 master parameters are what Adam updates.  All arrays are
 * device memory (FP32 unless stated); rows are samples.
 * ------------------------------------------------------------------------------------ */
typedef struct subadmm_mlp subadmm_mlp;

/* max_batch: largest batch passed to forward/backward.  E_ARG on bad widths. */
int subadmm_mlp_create(int32_t n_layers, const int32_t* widths, int32_t max_batch, subadmm_mlp** out);
int64_t subadmm_mlp_param_count(const subadmm_mlp* m);
size_t subadmm_mlp_workspace_bytes(const subadmm_mlp* m);
/* Binds caller-allocated device memory and a stream (as subadmm_bind). */
int subadmm_mlp_bind(subadmm_mlp* m, void* dev_workspace, size_t bytes, void* hip_stream);
/* Copies FP32 parameters (parameter layout) in, refreshes the BF16 copies and clears the
 * Adam moments; get copies the master parameters out. */
int subadmm_mlp_set_params(subadmm_mlp* m, const float* params);
int subadmm_mlp_get_params(subadmm_mlp* m, float* params_out);
/* Input normalisation applied in FP32 before the BF16 rounding of the input:
 * x_c <- x_c * scale[c] + shift[c] (device FP32 arrays of widths[0] entries, copied; both
 * NULL switches it off).  Not a trained parameter; cleared by subadmm_mlp_bind. */
int subadmm_mlp_set_input_affine(subadmm_mlp* m, const float* scale, const float* shift);
/* y (batch x widths[n_layers]) = network(x (batch x widths[0])); keeps the activations
 * of this batch for subadmm_mlp_backward. */
int subadmm_mlp_forward(subadmm_mlp* m, int32_t batch, const float* x, float* y);
/* Gradient of 0.5 * sum wt (y - target)^2 for the last forward batch (wt may be NULL for
 * ones) into the network's gradient buffer; optional copies to grad_out (parameter
 * layout) and loss_out (one float). */
int subadmm_mlp_backward(subadmm_mlp* m, int32_t batch, const float* target, const float* wt,
                         float* grad_out, float* loss_out);
/* One Adam step (step >= 1 for bias correction) on the master parameters with the
 * current gradient; refreshes the BF16 copies. */
int subadmm_mlp_adam(subadmm_mlp* m, float lr, float beta1, float beta2, float eps, int32_t step);
/* Inference only (the learned start's forward pass): y = the network's output for x, as
 * subadmm_mlp_forward computes it (the same values bit for bit), in one launch when every
 * width is at most 256 and there are at most 8 layers (else the per-layer forward).  Keeps no
 * activations, so a subadmm_mlp_backward must follow a subadmm_mlp_forward (E_STATE else). */
int subadmm_mlp_infer(subadmm_mlp* m, int32_t batch, const float* x, float* y);
/* Training minibatch gather on the network's stream: dst row r (device, count x width FP32)
 * = src row idx[r] (src: device, n_rows x width FP32, row-major; idx: device, count int32).
 * A row whose index lies outside [0, n_rows) is filled with NaN.  E_ARG on bad sizes. */
int subadmm_mlp_gather_rows(subadmm_mlp* m, const float* src, int64_t n_rows, int32_t width, const int32_t* idx,
                            int32_t count, float* dst);
void subadmm_mlp_destroy(subadmm_mlp* m);
const char* subadmm_mlp_last_error(const subadmm_mlp* m);

/* Learned warm start on a rigid problem.  Interfaces of two classes take part: class 0,
 * contacts (dim 3); class 1, dim-5 equalities (revolute joints); others start from the
 * previous step's values.  Per class the features (rows in interface order) are
 *   class 0, 12 floats: e_n, c (3), lambda_prev / w_hat (3), z_prev (3), log w_hat, mu
 *   class 1, 27 floats: e (5), c (5), lambda_prev / w_hat (5), z_prev of member 0 (5) and
 *                       of member 1 (5, zeros for one member), log w_hat, |S_j| - 1
 * with e_j the constraint error, c = sum_i J_i,j v_i at the start-of-step velocity,
 * (z_prev, u_prev = -lambda_prev) the previous step's final values and
 * w_hat = 1 / sum_i beta_i^-1 (the weight of Eq. (18)); the network outputs
 *   class 0, 6 floats: delta lambda / w_hat (3), delta z (3)
 *   class 1, 15 floats: delta lambda / w_hat (5), delta z of member 0 (5), member 1 (5)
 * and z^0 = z_prev + delta z, u^0 = -(lambda_prev + w_hat delta lambda / w_hat) for every
 * member slot.  A network (NULL to detach) must have widths (12, ..., 6) or
 * (27, ..., 15), max_batch >= the class size and the problem's stream; it stays owned
 * by the caller. */
int subadmm_set_warm_model(subadmm_problem* p, int32_t cls, subadmm_mlp* net);
int subadmm_warm_class_counts(const subadmm_problem* p, int32_t* n_contact, int32_t* n_joint);
/* Training-data recording.  While a pointer is non-NULL every rigid step writes to it
 * (device FP32, rows in class order): xc (n_contact x 12) and xj (n_joint x 27), the
 * features computed before the iteration; tc (n_contact x 6) and tj (n_joint x 15), the
 * targets: the network's outputs that would have started the iteration at the values it
 * converged to; wc, wj (same shapes), the loss weights of the ADMM metric
 * sum_i beta_i |z_i - z*_i|^2 + beta_i^-1 |u_i - u*_i|^2 (w_hat for the lambda entries,
 * beta_i for member i's z entries), zero for absent members and for scenes that stopped
 * at max_iters.  The buffers stay owned by the caller; NULL pointers switch recording off. */
int subadmm_set_recording(subadmm_problem* p, float* xc, float* xj, float* tc, float* tj, float* wc, float* wj);
/* Copy the kept final (z, u) (slot layout, device, real) out of / into the problem (the
 * previous-step warm start; also a checkpoint of the solver state). */
int subadmm_get_warm(subadmm_problem* p, void* z_out, void* u_out);
int subadmm_set_warm(subadmm_problem* p, const void* z, const void* u);

/* Deformable bodies: co-rotated linear-tetrahedron blocks, one subsystem per block (the
 * elastic potential folded into A_i, b_i, as the paper's remark on soft constraints
 * allows; its FEM example of Sec. IV).  Subsystem i holds nodes node_off[i] ..
 * node_off[i+1]-1 with node_off the prefix of n_dof/3 (DOFs (x, y, z) per node), so
 * n_nodes = sum n_dof / 3.  rest: n_nodes x 3 rest positions; tets: n_tets x 4 node
 * indices, all four in one subsystem, positive rest volume; young, poisson: per
 * subsystem (E > 0, 0 <= nu < 0.5); density (kg/m^3) gives lumped node masses.
 * Interfaces must be nodal equalities (kind equality, dim 3, two members; rows +I on
 * member 0's node and -I on member 1's; error gamma (x_p - x_q) / t with gamma =
 * baumgarte) or ground contacts (kind contact, one member; plane z = 0, rows
 * (e_z, e_x, e_y) on the node; error (z / t, 0, 0)); if_node[2j + m] is the node of
 * member m.  Per step: A = (2/t) M + (t/2) K(x), b = (2/t) M v - d psi(x) + M g with the
 * co-rotated stiffness K and elastic force -d psi at the start-of-step positions, and
 * x+ = x + t v_hat, v+ = 2 v_hat - v (Eq. (2)).  Exclusive with the rigid model; must
 * precede subadmm_workspace_bytes/subadmm_bind.  E_ARG on an invalid model. */
int subadmm_fem_set_model(subadmm_problem* p, int32_t n_nodes, const double* rest, int32_t n_tets,
                          const int32_t* tets, const double* young, const double* poisson, double density,
                          const int32_t* if_node, double gravity, double baumgarte);
/* Construction of the FEM step at pos, vel (device, n_nodes x 3 real): A, b, J (dense,
 * the layout of subadmm_solve) and e.  For checking the assembly on its own. */
int subadmm_fem_assemble(subadmm_problem* p, const void* pos, const void* vel, double dt, void* A, void* b,
                         void* J, void* e);
/* One whole time step of Algorithm 1 on the FEM blocks: construction, factorisation
 * (FP64, or per block as option SUBADMM_OPT_FEM_KAPPA_MAX selects), iteration (one launch with every block resident; every scene stops on its own test), v_hat
 * and the state update.  pos, vel (device, real) are updated in place; warm COLD or
 * PREV; optional outputs v_hat (DOF layout) and lambda (row layout).  Every block is
 * resident at once: E_DEVICE if the device cannot hold n_sub workgroups together. */
int subadmm_fem_step(subadmm_problem* p, void* pos, void* vel, double dt, int32_t max_iters, double tol,
                     int32_t warm, void* v_hat, void* lambda);
/* subadmm_fem_step replayed from a HIP graph (the step's launches captured on the first
 * call with a given set of arguments, replayed by later calls with the same arguments;
 * other arguments, or subadmm_set_option in between, capture again).  Same results as
 * subadmm_fem_step; warm COLD or PREV; per-kernel timing is not recorded in replays.  The
 * graph holds the pointers it was captured with: their memory must stay valid. */
int subadmm_fem_step_graph(subadmm_problem* p, void* pos, void* vel, double dt, int32_t max_iters, double tol,
                           int32_t warm, void* v_hat, void* lambda);
/* Form of the last FEM iteration launch on p: *tiles = 0 when the operators were read
 * from device memory in every iteration, else the number of 16 x 16 operator tiles each
 * wave kept in registers (resident form, option SUBADMM_OPT_FEM_RESIDENT); -1 before the
 * first step.  Host-side query, no device work. */
int subadmm_fem_loop_form(const subadmm_problem* p, int32_t* tiles);
/* Per-block record of the last FEM factorisation (option SUBADMM_OPT_FEM_KAPPA_MAX):
 * kappa_est (device, n_sub doubles; +inf where the FP32 trial met a pivot that is not
 * positive) and fp64 (device, n_sub int32: 1 = the block was factorised in FP64, 0 = its
 * factors are FP32), either may be NULL.  Copied on the bound stream (asynchronous).  In
 * the FP32 trial form kappa_est comes from the trial's factor, else from the FP64 one.
 * E_STATE before the first FEM step. */
int subadmm_fem_block_precision(subadmm_problem* p, void* kappa_est, void* fp64);

/* Frees the host-side problem (not the caller's device memory). */
void subadmm_destroy(subadmm_problem* p);

/* Message of the last failure on p (or of the last failed setup when p is NULL). */
const char* subadmm_last_error(const subadmm_problem* p);

#ifdef __cplusplus
}
#endif
#endif /* SUBADMM_H */
