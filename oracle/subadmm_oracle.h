/*
 * FP64 CPU oracle for the per-step subsystem-based ADMM solve
 * (Lee, Lee & Lee, "Modular and Parallelizable Multibody Physics Simulation via
 * Subsystem-Based ADMM", arXiv 2302.14344).
 *
 * TEST INFRASTRUCTURE ONLY.  This library is the independent reference that the HIP
 * path is checked against.  Only the test suite, the smoke check and the CPU-baseline
 * leg of the benchmark may load it; the product path never calls it.  It shares no
 * code, header, table or constant with the HIP library.
 *
 * Storage conventions (all arrays are caller-owned host memory, FP64 unless noted):
 *   - subsystem i has n_i DOF; its DOF start is the prefix sum of n.
 *   - A: per subsystem a dense row-major n_i x n_i block, blocks concatenated.
 *   - b: concatenated per-subsystem vectors (length sum n_i).
 *   - slot rows: subsystem i owns one row per (interface j containing i, row k of j),
 *     ordered by ascending j then k.  J holds, per subsystem, the dense row-major
 *     nc_i x n_i matrix J_c,i of its slot rows; blocks concatenated.
 *   - e, lambda: per interface j its d_j rows, concatenated in interface order.
 *   - z, u: per slot row (length sum nc_i).
 *   - Interface j has kind (0 equality, 1 Signorini-Coulomb contact with rows
 *     (normal, t1, t2), 2 one-sided hard inequality), dimension d_j, 1 or 2 member
 *     subsystems if_sub[2j], if_sub[2j+1] and friction coefficient if_mu[j].
 * Return codes: 0 ok, -1 bad argument, -2 matrix not positive definite.
 */
#ifndef SUBADMM_ORACLE_H
#define SUBADMM_ORACLE_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Algorithm 1, Eq. (12)-(23): per-step solve of an assembled problem.  if_sub holds four
 * entries per interface, its members (1 <= if_nsub <= 4, distinct, one scene; unused
 * entries ignored). */
int oracle_solve(int32_t n_sub, const int32_t* sub_ndof, const int32_t* sub_scene,
                 int32_t n_if, const int32_t* if_kind, const int32_t* if_dim,
                 const int32_t* if_nsub, const int32_t* if_sub, const double* if_mu,
                 const double* A, const double* b, const double* J, const double* e,
                 double rho, int32_t max_iters, double tol,
                 const double* z0, const double* u0,
                 double* v_hat, double* lambda, double* z, double* u, double* beta,
                 int32_t* iters, int32_t* converged, double* theta, double* r_theta,
                 int32_t n_threads);

/* The same with the contact z-update of Eq. (21) chosen: contact_model 0 = exact
 * Signorini-Coulomb projection, 1 = relaxed convex model (Euclidean projection onto the
 * friction cone); if_k, if_alpha: gain and alpha of soft interfaces (kind 3, Eq. 3),
 * NULL when there are none; scene_max_iters: per-scene iteration bound of Alg. 1 (one
 * entry per scene, each >= 1), NULL for max_iters everywhere.  r_prim, r_dual (one per
 * scene, both or neither NULL): the primal and dual residuals of ADMM's standard stopping
 * test (Boyd et al. 2011, Sec. 3.3) for the returned iterate: the z- and u-updates that
 * would follow the last x-update, taken aside; r_prim = |x - z'| / max(|x|, |z'|),
 * r_dual = |beta (z' - z)| / |u'|, floors 1e-12. */
int oracle_solve_model(int32_t n_sub, const int32_t* sub_ndof, const int32_t* sub_scene,
                       int32_t n_if, const int32_t* if_kind, const int32_t* if_dim,
                       const int32_t* if_nsub, const int32_t* if_sub, const double* if_mu,
                       const double* A, const double* b, const double* J, const double* e,
                       double rho, int32_t max_iters, double tol,
                       const double* z0, const double* u0,
                       double* v_hat, double* lambda, double* z, double* u, double* beta,
                       int32_t* iters, int32_t* converged, double* theta, double* r_theta,
                       double* r_prim, double* r_dual,
                       int32_t contact_model, const double* if_k, const double* if_alpha,
                       const int32_t* scene_max_iters, int32_t n_threads);

/* Link rows (linear or angular, between two bodies or on one body) for interfaces of kind
 * soft, equality, hard inequality or contact, added to the arrays of oracle_rigid_assemble. */
int oracle_rigid_links(int32_t n_sub, const int32_t* sub_ndof, int32_t n_if, const int32_t* if_kind,
                       const int32_t* if_dim, const int32_t* if_nsub, const int32_t* if_sub,
                       const int32_t* body_sub, const int32_t* body_local, const double* pos,
                       const double* rot, int32_t nl, const int32_t* link_type, const int32_t* link_body,
                       const double* link_anchor, const double* link_frame, const int32_t* link_if,
                       double dt, double baumgarte, double* J, double* e);

/* Soft links between two bodies of one subsystem (link_if < 0) folded into that subsystem's
 * dynamics (Sec. III-B, the remark after Eq. 6): A_i += k alpha J^T J, b_i -= k J^T phi. */
int oracle_rigid_fold_soft(int32_t n_sub, const int32_t* sub_ndof, const int32_t* body_sub,
                           const int32_t* body_local, const double* pos, const double* rot, int32_t nl,
                           const int32_t* link_type, const int32_t* link_body, const double* link_anchor,
                           const double* link_frame, const int32_t* link_if, const int32_t* link_dim,
                           const double* link_k, const double* link_alpha, double* A, double* b);

/* Eq. (2)-(5) assembled for boxes in maximal coordinates (Alg. 1, construction steps). */
int oracle_rigid_assemble(int32_t n_sub, const int32_t* sub_ndof, int32_t n_if,
                          const int32_t* if_dim, const int32_t* if_nsub, const int32_t* if_sub,
                          int32_t nb, const int32_t* body_sub, const int32_t* body_local,
                          const double* mass, const double* inertia,
                          const double* pos, const double* rot, const double* vel,
                          const double* omega,
                          int32_t nj, const int32_t* joint_body, const double* joint_anchor,
                          const double* joint_frame_a, const double* joint_axis_b,
                          const int32_t* joint_if,
                          int32_t ncon, const int32_t* contact_body, const double* contact_point,
                          const int32_t* contact_if,
                          double dt, double gravity, double baumgarte,
                          double* A, double* b, double* J, double* e);

/* State update of Eq. (2) (Alg. 1, last step): v+ = 2 v_hat - v, p+ = p + t v_hat_lin,
 * R+ = R exp(t [w_hat]x). */
int oracle_rigid_advance(int32_t nb, const int32_t* body_sub, const int32_t* body_local,
                         int32_t n_sub, const int32_t* sub_ndof, const double* v_hat, double dt,
                         const double* pos, const double* rot, const double* vel,
                         const double* omega, double* pos_out, double* rot_out,
                         double* vel_out, double* omega_out);

/* Perceptron with ReLU hidden layers and a linear output layer, FP64 (the learned warm
 * start's network).  widths[0..n_layers]; params holds, per layer k, W_k (widths[k+1] x
 * widths[k], row-major) then b_k (widths[k+1]).  in: batch x widths[0]; out: batch x
 * widths[n_layers]. */
int oracle_mlp_forward(int32_t n_layers, const int32_t* widths, const double* params,
                       int32_t batch, const double* in, double* out);
/* Gradient of L = 0.5 * sum_{b,o} wt[b,o] (out[b,o] - target[b,o])^2 with respect to
 * params (same layout); also returns L. */
int oracle_mlp_backward(int32_t n_layers, const int32_t* widths, const double* params,
                        int32_t batch, const double* in, const double* target,
                        const double* wt, double* grad, double* loss);

/* Co-rotated linear-tetrahedron elastic blocks (one subsystem per block), Eq. (2) with
 * the elastic potential folded into A_i, b_i; see oracle_fem.c for the formulas.
 * Nodes of subsystem i are listed contiguously (sub_nodes[i] of them); tets hold node
 * indices; if_node holds the node of each interface member.  Outputs in the layout of
 * oracle_solve. */
int oracle_fem_assemble(int32_t n_sub, const int32_t* sub_nodes, int32_t n_tets, const int32_t* tets,
                        const int32_t* tet_sub, const double* rest, const double* pos, const double* vel,
                        const double* young, const double* poisson, double density, int32_t n_if,
                        const int32_t* if_kind, const int32_t* if_dim, const int32_t* if_nsub,
                        const int32_t* if_sub, const int32_t* if_node, double dt, double gravity, double baumgarte,
                        double* A, double* b, double* J, double* e);
/* One tetrahedron: 12x12 co-rotated stiffness K and the 12 elastic forces f from rest and
 * current vertex positions (4x3 each). */
int oracle_fem_element(const double* X, const double* x, double young, double poisson, double* K, double* f);
/* Orthogonal polar factor of a 3x3 matrix (row-major). */
int oracle_polar(const double* F, double* R);
/* Eq. (2) state update: x+ = x + t v_hat, v+ = 2 v_hat - v. */
int oracle_fem_advance(int64_t n_nodes, const double* v_hat, double dt, const double* pos, const double* vel,
                       double* pos_out, double* vel_out);

#ifdef __cplusplus
}
#endif
#endif
