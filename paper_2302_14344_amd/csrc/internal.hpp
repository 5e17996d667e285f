// Internal declarations shared by the HIP kernels and the host runtime of libsubadmm.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace subadmm {

// Device-side error flags (bit set by kernels, read by subadmm_check).
enum : int32_t { FLAG_NOT_SPD = 1, FLAG_NONFINITE = 2, FLAG_BARRIER = 4 };

enum : int32_t { KIND_EQUALITY = 0, KIND_CONTACT = 1, KIND_HARD_INEQ = 2, KIND_SOFT = 3 };

constexpr int kMaxDof = 64;      // largest subsystem of the rigid model's kernels
constexpr int kMaxFactorDof = 512;  // largest subsystem of the factorisation (a thread per column)
constexpr int kMaxFemDof = 768;  // largest subsystem (FEM block path)
// copies of the FEM residual partials (each workgroup reads the copy of its index mod
// kPartCopies, so the lines every workgroup polls are spread over more addresses)
constexpr int kPartCopies = 8;
constexpr int kMaxIfDim = 6;     // largest interface dimension
constexpr int kMaxMembers = 4;   // largest member count |S_j| of an interface
constexpr int kLoopThreads = 256;
// the thread-per-row iteration kernel gives each slot row two lanes while the block stays
// within this many threads
constexpr int kTwoLaneMax = 256;
// interface-map entries of single rows: interface index in the low bits, row + 1 above
constexpr int kZRowShift = 26;
constexpr int kZIfMask = (1 << kZRowShift) - 1;
constexpr int kFactorThreads = 128;

// Topology tables in device memory (int32 unless noted).
struct Topo {
  int32_t n_sub, n_if, n_scene;
  int32_t max_row_scene;    // interface rows (e, lambda) of the largest scene
  const int32_t* sub_n;     // DOF per subsystem
  const int32_t* sub_nc;    // slot rows per subsystem
  const int32_t* sub_dof;   // DOF offset
  const int32_t* sub_slot;  // slot offset
  const int64_t* sub_A;     // offset of A_i (n^2 entries)
  const int64_t* sub_J;     // offset of J_i and G_i (nc n entries)
  const int64_t* sub_H;     // offset of H_i (nc^2 entries)
  const int32_t* slot_sub;  // per slot row: subsystem
  const int32_t* slot_loc;  // per slot row: local row inside the subsystem
  const int32_t* slot_if;   // per slot row: interface
  const int32_t* slot_mk;   // per slot row: member * 8 + row inside the interface
  const int32_t* if_kind;
  const int32_t* if_dim;
  const int32_t* if_nsub;
  const int32_t* if_sub0;
  const int32_t* if_sub1;
  const int32_t* if_slot0;  // first slot row of member 0
  const int32_t* if_slot1;  // first slot row of member 1 (-1 if none)
  const int32_t* if_row;    // offset in the row layout
  const int32_t* if_subx;   // members 2 and 3 (2 per interface, -1 if none)
  const int32_t* if_slotx;  // their first slot rows
  const int32_t* sc_sub;    // per scene prefix (n_scene + 1)
  const int32_t* sc_slot;
  const int32_t* sc_if;
  const int32_t* sc_dof;
  // LDS layout of the iteration kernel (16-byte vectors of V = 16/sizeof(real) entries):
  const int32_t* sub_hq;    // per subsystem: vector offset of its blocked H inside the scene
  const int32_t* sub_wq;    // per subsystem: offset of its padded w block inside the scene
  const int32_t* sc_hq;     // per scene: vectors of blocked H (n_scene entries)
  const int32_t* sc_wq;     // per scene: entries of padded w (n_scene entries)
  // lane roles of the team iteration kernel: per scene team_block entries, each
  // (interface << 4 | position in the interface's team) or -1 for an idle lane
  const int32_t* lane_code;
  int32_t team_block;
  // thread-per-interface iteration kernel: per scene zmap_block entries, the interface
  // whose z-update thread t does, or one row r of it (j | (r + 1) << kZRowShift: the rows
  // of equality, hard and soft interfaces of one or two members are independent), -1 for
  // none; arranged so that each wave holds one interface class (kind, rows per thread);
  // nullptr: thread t takes the scene's t-th interface
  const int32_t* zmap;
  int32_t zmap_block;
  // thread-per-slot-row iteration kernel with split rows: per scene rmap_block entries,
  // (slot row in the scene << 5 | lanes of the row << 2 | lane's part) or -1 for an idle
  // lane; the 1, 2 or 4 lanes of a row are consecutive and aligned to their count;
  // nullptr: one or two lanes per row for the whole scene
  const int32_t* rmap;
  int32_t rmap_block;
};

template <typename T>
struct FactorArgs {
  Topo t;
  const T* A;
  const T* b;
  const T* J;
  double rho;
  T* beta;   // per subsystem
  T* H;      // per subsystem nc x nc: H_i = J K^-1 J^T, column-major (symmetric)
  T* d;      // per slot row: J K^-1 b
  T* G;      // per subsystem n x nc: column c = K^-1 J^T e_c
  T* cvec;   // per DOF: K^-1 b
  int32_t* flags;
  const int32_t* order;  // subsystems of this launch: order[first + blockIdx.x]
  int32_t first;
};

template <typename T>
struct LoopArgs {
  Topo t;
  const T* beta;
  const T* H;
  const T* d;
  const T* G;
  const T* cvec;
  const T* e;
  const T* mu;       // per interface
  const T* ksoft;    // per interface: gain k of a soft interface (Eq. 3), else 0
  const T* asoft;    // per interface: alpha of a soft interface (Eq. 3), else 0
  const T* z_in;     // per slot row (nullptr = cold)
  const T* u_in;
  T* z_out;          // per slot row
  T* u_out;
  T* v_hat;          // per DOF
  T* lambda;         // per interface row
  int32_t* st_iters; // per scene
  long long* st_total;  // per scene, cumulative x-updates
  long long* st_unconv; // per scene, cumulative count of runs stopped at max_iters
  int32_t* st_conv;
  double* st_theta;
  double* st_rtheta;
  int32_t* flags;
  int32_t max_iters;
  double tol;
  int32_t contact_model;  // 0: exact Signorini-Coulomb projection, 1: relaxed convex model
  const int32_t* skip_converged;  // if set: scenes with skip_converged[s] != 0 are left as they are
  long long* st_fallback;         // if set: incremented for every scene this launch iterates
};

// Rigid model (maximal coordinates) in device memory.
template <typename T>
struct RigidModel {
  int32_t nb, nj, ncon;
  const int32_t* body_sub;
  const int32_t* body_local;
  const T* mass;
  const T* inertia;         // 3 per body
  const int32_t* sub_body;  // bodies sorted by subsystem
  const int32_t* sub_body_off;  // n_sub + 1
  const int32_t* if_src;    // per interface: joint q -> q, link q -> nj + q, contact q -> -1 - q
  const int32_t* joint_body;    // 2 per joint
  const T* joint_anchor;    // 6 per joint
  const T* joint_frame;     // 9 per joint (rows h, u, v in body a frame)
  const T* joint_axis_b;    // 3 per joint
  const int32_t* contact_body;
  const T* contact_point;   // 3 per contact
  // links (if_src nj + q): rows along directions fixed in body a's frame
  int32_t nl;
  const int32_t* link_type;  // 0 linear (anchor-point velocities), 1 angular
  const int32_t* link_body;  // 2 per link (b = -1: rows on one body)
  const T* link_anchor;      // 6 per link (body frames)
  const T* link_frame;       // 9 per link: row directions in a's frame
  const int32_t* link_dim;   // rows per link
  const T* link_k;           // folded soft links (no interface): k and alpha of Eq. 3
  const T* link_alpha;
  const int32_t* sub_ilink_off;  // n_sub + 1: folded links of each subsystem
  const int32_t* sub_ilink;
  T gravity, baumgarte;
};

template <typename T>
struct RigidState {
  T* pos;    // 3 per body
  T* rot;    // 9 per body
  T* vel;    // 3 per body
  T* omega;  // 3 per body
};

// Several whole time steps of a rigid problem in one launch, one workgroup per scene
// (construction, factorisation, iteration and state update of each step in turn, so that a
// scene's steps follow one another without waiting for the other scenes).
template <typename T>
struct StepsArgs {
  FactorArgs<T> f;   // inputs A, b, J are the construction's outputs
  LoopArgs<T> l;     // e is the construction's output; v_hat the per-step v_hat buffer
  RigidModel<T> m;
  RigidState<T> st;
  T* A;              // construction outputs (dense layout of subadmm_solve)
  T* b;
  T* J;
  T* e;
  T dt;
  int32_t n_steps;
  int32_t lds_factor;      // bytes of LDS a factorisation may use (larger ones use fscr)
  double* fscr;            // global scratch of the factorisations above lds_factor
  const int64_t* sc_fscr;  // per scene: offset into fscr (in doubles), -1 if none is needed
  const int32_t* sc_order; // scene of each workgroup (a permutation of the scenes)
};

// The iteration of scenes too large for one workgroup, one launch per phase per iteration.
template <typename T>
struct LargeArgs {
  LoopArgs<T> l;             // z_in/u_in, outputs and statistics as for the per-scene kernel
  const int32_t* sub_scene;  // per subsystem
  T* y;                      // per slot row: y of the last x-update
  T* u;                      // per slot row: u = -lambda of the last z-update
  T* w;                      // per slot row: w = beta z - u
  double* dy2;               // per slot row: (y^{l+1} - y^l)^2 of the last x-update
  double* yy2;               // per slot row: (y^{l+1})^2
  int32_t* done;             // per scene: stopped
  int32_t* all_done;         // one flag: every scene stopped (written by the poll kernel)
  int64_t n_slot, n_dof;
};

// Constraint error of a step (the accuracy measure), per scene.
template <typename T>
struct ErrorArgs {
  Topo t;
  const T* J;                // dense slot rows (rigid model, assembled problems); nullptr: FEM selections
  const int32_t* slot_dof;   // FEM: local DOF each slot row selects
  const float* slot_sgn;     // FEM: its sign
  const T* e;
  const T* v_hat;
  const T* lambda;
  const T* beta;
  const T* mu;
  const T* ksoft;
  const T* asoft;
  double* out;               // per scene
  int32_t kinds;             // bit k: interfaces of kind k count
};

// LDS budget of the multi-step kernel: four workgroups per CU (160 KB) while the scene's
// iteration fits in it.
constexpr size_t kStepsLds = 39 * 1024;
// LDS of one wave's factorisation of a small subsystem (four waves per workgroup)
constexpr size_t kWaveFactorSlice = 12 * 1024;

// Bytes of the factorisation working arrays of one subsystem (n DOF, nc slot rows) with
// elements of cs bytes: K (n x ld), J (nc x ld), the nc + 1 solves (ld each), two n-vectors.
__host__ __device__ inline size_t factor_bytes(int n, int nc, size_t cs) {
  const size_t ld = (size_t)(n | 1);
  return cs * (ld * (size_t)n + ld * ((size_t)nc + 1) + 2 * (size_t)n);
}

// Learned warm start: interface classes and feature/output widths.
constexpr int kContactIn = 12, kContactOut = 6, kJointIn = 27, kJointOut = 15;

template <typename T>
struct WarmArgs {
  Topo t;
  const int32_t* if_class;  // -1: not learned, 0: contact (dim 3), 1: revolute joint (dim 5)
  const int32_t* if_krow;   // row of the interface in its class's feature matrix
  const T* beta;
  const T* e;
  const T* J;
  const T* v_dof;
  const T* mu;
  const T* z_prev;
  const T* u_prev;
  float* xc;                // features, contacts x kContactIn
  float* xj;                // features, joints x kJointIn
  const float* yc;          // network outputs (nullptr: previous-step values for the class)
  const float* yj;
  T* z0;                    // initial values per slot row
  T* u0;
  // training targets (recorded after the solve): final values, per-scene convergence
  const int32_t* if_scene;
  const int32_t* conv;
  const T* z_fin;
  const T* u_fin;
  float* tc;                // contacts x kContactOut targets, wc their loss weights
  float* tj;                // joints x kJointOut targets, wj their loss weights
  float* wc;
  float* wj;
};

// Co-rotated FEM blocks (one subsystem per block) in device memory.  DOFs of a block are
// its nodes' (x, y, z); the factorisation works in a permuted order with the block's
// constrained DOFs (those selected by a slot row) last.
struct FemModel {
  int32_t n_tets;
  const int32_t* node_off;   // per subsystem: first node (n_sub + 1)
  const int32_t* tet_off;    // per subsystem: first tetrahedron (n_sub + 1), tets sorted by subsystem
  const int32_t* tet_node;   // 4 node indices (global) per tetrahedron
  const double* tet_g;       // 12 per tetrahedron: rest shape-function gradients g_0..g_3
  const double* tet_vol;     // rest volume
  const double* rest;        // 3 per node
  const double* mass;        // lumped mass per node
  const double* lame_l;      // per subsystem
  const double* lame_m;
  const int32_t* pair_off;   // per subsystem: first node pair (n_sub + 1)
  const int32_t* pair_ab;    // per pair: local a | local b << 16
  const int32_t* pent_off;   // per pair: first entry (n_pairs + 1)
  const int32_t* pent;       // entries: local tet << 4 | la << 2 | lb
  const int32_t* node_diag;  // per node (global): index of its pair (a, a), whose entries list its tetrahedra
  const int32_t* m;          // per subsystem: constrained DOF count
  const int32_t* dkey_off;   // per subsystem: prefix of m (n_sub + 1)
  const int64_t* sq_off;     // per subsystem: offset of its m x m operator (lower 16 x 16 tiles, 256 entries each)
  const int32_t* perm;       // per DOF (global index): local DOF at this permuted position
  const int32_t* jtj;        // per DOF (global, original order): slot rows selecting it
  const int32_t* slot_dk;    // per slot: constrained-DOF index (permuted position - (n - m))
  const int32_t* slot_dof;   // per slot: local DOF (original order)
  const float* slot_sgn;     // per slot: +1 / -1
  const int32_t* dk_off;     // per constrained DOF (global over subsystems): first slot in dk_slot
  const int32_t* dk_slot;    // slots (global index) selecting that DOF
  const int32_t* if_node0;   // per interface: node of each member (global)
  const int32_t* if_node1;
  double gravity, baumgarte;
};

template <typename T>
struct FemLoopArgs {
  Topo t;
  FemModel f;
  const T* S;       // per subsystem m x m (row-major, symmetric): K^-1 on the constrained DOFs
  const T* cd;      // per constrained DOF: (K^-1 b) there
  const T* beta;
  const T* e;
  const T* mu;
  const T* z_in;
  const T* u_in;
  T* z_out;
  T* u_out;
  T* w_out;         // per slot: the w of the last x-update (for v_hat)
  T* ybuf;          // 3 x n_slot: y of iterations l mod 3 (entries all-ones until written)
  T* lambda;
  double* part;     // 3 x kPartCopies x 2 per subsystem: theta and |y|^2 partials, as ybuf
  int32_t* st_iters;
  long long* st_total;
  long long* st_unconv;
  int32_t* st_conv;
  double* st_theta;
  double* st_rtheta;
  int32_t* flags;
  int32_t max_iters;
  double tol;
  int32_t contact_model;  // 0: exact Signorini-Coulomb projection, 1: relaxed convex model
  int32_t max_m, max_mt16, max_nc;
  int32_t max_ng;    // most interfaces touching one block
  int32_t n_slot;
  int32_t resident;  // keep each block's S on chip when it fits (FP32 only)
};

// Kernel launchers (defined in the .hip files).
template <typename T>
hipError_t launch_dof_velocity(const Topo& t, const RigidModel<T>& m, const T* vel, const T* omega, T* v_dof,
                               hipStream_t s);
template <typename T>
hipError_t launch_features(const WarmArgs<T>& a, hipStream_t s);
template <typename T>
hipError_t launch_warm_apply(const WarmArgs<T>& a, hipStream_t s);
template <typename T>
hipError_t launch_targets(const WarmArgs<T>& a, hipStream_t s);
template <typename T>
hipError_t launch_factor(const FactorArgs<T>& a, int count, int max_n, int max_nc, bool fp64, hipStream_t s);
// The same factorisation for subsystems whose working arrays exceed the LDS, with the arrays
// in device memory at scr + off[i] bytes (factor_bytes(n, nc, element size) each).
template <typename T>
hipError_t launch_factor_global(const FactorArgs<T>& a, int count, int max_n, bool fp64, char* scr, const int64_t* off,
                                hipStream_t s);
template <typename T>
hipError_t launch_steps(const StepsArgs<T>& a, const StepsArgs<T>* dev_args, int max_slot_scene, int max_if_scene,
                        int max_hq_scene, int max_wq_scene, bool fp64, size_t lds, hipStream_t s);
// poll_every > 0: every poll_every iterations the host reads whether every scene has
// stopped (host_flag, a host int) and launches no further iterations if so (the remaining
// launches would change nothing); 0: all max_iters iterations are launched (graph capture).
template <typename T>
hipError_t launch_large_loop(const LargeArgs<T>& a, hipStream_t s, int poll_every, int32_t* host_flag);
// the same iteration with one workgroup of `threads` (256..1024) carrying each scene (one
// launch)
template <typename T>
hipError_t launch_large_scene(const LargeArgs<T>& a, int threads, hipStream_t s);
// ADMM's primal and dual residuals of the returned (z_in, u_in), per scene (large-scene
// slot arrays as scratch)
template <typename T>
hipError_t launch_boyd_residuals(const LargeArgs<T>& a, double* r_prim, double* r_dual, hipStream_t s);
template <typename T>
hipError_t launch_constraint_error(const ErrorArgs<T>& a, hipStream_t s);
template <typename T>
hipError_t launch_loop(const LoopArgs<T>& a, int max_slot_scene, int max_if_scene, long long max_h_scene,
                       int max_hq_scene, int max_wq_scene, int max_nc, hipStream_t s);
template <typename T>
hipError_t launch_team_loop(const LoopArgs<T>& a, int max_hq_scene, int max_wq_scene, hipStream_t s);
// one wave per scene: scenes of at most 256 slot rows and 64 interfaces whose operators fit in LDS
template <typename T>
hipError_t launch_wave_loop(const LoopArgs<T>& a, int max_slot_scene, int max_if_scene, int max_hq_scene,
                            int max_wq_scene, hipStream_t s);
// FEM pipeline.  A and b in FP64 (dense n x n per block, original DOF order).
template <typename T>
hipError_t launch_fem_assemble(const Topo& t, const FemModel& f, const T* pos, const T* vel, double dt, double* A,
                               double* b, double* tet_scratch, int32_t* flags, hipStream_t s);
template <typename T>
hipError_t launch_fem_rows(const Topo& t, const FemModel& f, const T* pos, double dt, T* e, hipStream_t s);
// beta (Eq. 23 or rho), K = P (A + beta J^T J) P^T, Cholesky L (in place of K), S = K^-1 on
// the constrained DOFs (T) and cd = (K^-1 b) there (T).  kmax > 0 with T = float: an FP32
// trial factor of every block, FP64 again for blocks with kappa_est > kmax; else FP64
// throughout.  prec[i] (1 = FP64 factors) and kest[i] record each block's outcome.
template <typename T>
hipError_t launch_fem_factor(const Topo& t, const FemModel& f, const double* A, double* b, double rho,
                             T* beta, double* L, double* tinv, T* S, T* cd, int32_t* flags, int32_t* prec,
                             double* kest, double kmax, int max_n, int max_m, hipStream_t s);
template <typename T>
hipError_t launch_fem_loop(const FemLoopArgs<T>& a, int* form, hipStream_t s);
// v_hat = K^-1 (b + J^T w) with each block's factors in the precision prec records.
template <typename T>
hipError_t launch_fem_vhat(const Topo& t, const FemModel& f, const double* L, const double* Tw, const double* y,
                           const int32_t* prec, const T* w, T* v_hat, int max_n, hipStream_t s);
template <typename T>
hipError_t launch_fem_advance(int64_t n_dof, const T* v_hat, T dt, T* pos, T* vel, hipStream_t s);
// Dense J (slot rows x n per subsystem) and A, b cast to T, for the generic assembled layout.
template <typename T>
hipError_t launch_fem_export(const Topo& t, const FemModel& f, const double* A, const double* b, T* Ao, T* bo, T* Jo,
                             hipStream_t s);

// per_scene: one workgroup per scene (scenes of a few subsystems), else one per subsystem
template <typename T>
hipError_t launch_rigid_assemble(const Topo& t, const RigidModel<T>& m, const T* pos, const T* rot,
                                 const T* vel, const T* omega, T dt, T* A, T* b, T* J, T* e, bool per_scene,
                                 hipStream_t s);
template <typename T>
hipError_t launch_rigid_advance(const Topo& t, const RigidModel<T>& m, RigidState<T> st,
                                const T* v_hat, T dt, hipStream_t s);

// Relaxed convex contact model for the z-update of Eq. (21) (the convexification named in
// the paper's convergence discussion): the Euclidean projection of p = (p_n, p_t) onto the
// friction cone K = {|l_t| <= mu l_n}.  p itself inside K, 0 inside the polar cone
// {mu |q_t| <= -q_n}, else the point of K's boundary ray along p_t nearest to p.
__device__ inline float cone_sqrt(float x) { return __builtin_sqrtf(x); }
__device__ inline double cone_sqrt(double x) { return __builtin_sqrt(x); }
template <typename T>
__device__ inline void cone_project(const T* p, T mu, T* lam) {
  const T tn = cone_sqrt(p[1] * p[1] + p[2] * p[2]);
  if (tn <= mu * p[0]) {
    lam[0] = p[0];
    lam[1] = p[1];
    lam[2] = p[2];
  } else if (mu * tn <= -p[0]) {
    lam[0] = (T)0;
    lam[1] = (T)0;
    lam[2] = (T)0;
  } else {
    const T ln = (p[0] + mu * tn) / ((T)1 + mu * mu);
    const T f = mu * ln / tn;
    lam[0] = ln;
    lam[1] = f * p[1];
    lam[2] = f * p[2];
  }
}

}  // namespace subadmm
