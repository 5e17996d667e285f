// Host runtime of libsubadmm: the C ABI declared in include/subadmm.h.
//
// setup validates the host descriptors and builds the slot layout (Eq. (9): the slot
// rows of subsystem i are the rows of every interface containing i, by ascending
// interface then row), per-scene ranges and the workspace plan.  bind places every
// table and per-step array in the caller's device workspace.  solve / rigid_step
// enqueue the kernels on the bound stream; nothing synchronises except the explicit
// stats/check calls.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/subadmm.h"
#include "internal.hpp"
#include "mlp_internal.hpp"

#define SUBADMM_API extern "C" __attribute__((visibility("default")))

using namespace subadmm;

namespace {

thread_local std::string g_setup_error;

// iterations between the large-scene path's checks that every scene has stopped
constexpr int kLargePoll = 32;
// largest scene (slot rows) whose large-path iteration one workgroup carries: ~8 rows per
// thread; beyond that one phase of one scene is better spread over the GPU (a 320-segment
// cable of ~3.4k rows took 47 us per iteration in one workgroup, 13 us in the phase form)
constexpr int kLargeSceneMax = 2048;

struct Plan {
  size_t off = 0;
  template <typename X>
  size_t take(size_t count) {
    off = (off + 255) & ~size_t(255);
    const size_t o = off;
    off += sizeof(X) * (count > 0 ? count : 1);
    return o;
  }
};

}  // namespace

struct subadmm_problem {
  int32_t dtype = SUBADMM_F32;
  double rho = 0.0;
  int32_t factor_fp64 = 1;  // per-step factorisation arithmetic (option SUBADMM_OPT_FACTOR_FP64)
  int32_t use_team = 0;     // iteration kernel form (option SUBADMM_OPT_TEAM_KERNEL)
  int32_t learned_budget = 0;  // iterations of the learned-start run (0: max_iters)
  int32_t factor_streams = 1;  // option SUBADMM_OPT_FACTOR_STREAMS
  int32_t fem_resident = 1;    // option SUBADMM_OPT_FEM_RESIDENT
  int32_t split_rows = 0;      // option SUBADMM_OPT_SPLIT_ROWS
  int32_t contact_model = 0;   // option SUBADMM_OPT_CONTACT_MODEL
  int32_t fem_form = -1;       // form of the last FEM iteration launch (tiles per wave on chip)
  int64_t fem_kappa_max = 0;   // option SUBADMM_OPT_FEM_KAPPA_MAX
  int32_t impulse = 0;         // option SUBADMM_OPT_IMPULSE_OUTPUT
  bool fem_factored = false;   // a FEM factorisation has run (its per-block record is valid)
  int32_t n_sub = 0, n_if = 0, n_scene = 0;
  std::vector<int32_t> sub_n, sub_nc, sub_dof, sub_slot, sub_scene;
  std::vector<int64_t> sub_A, sub_J, sub_H;
  std::vector<int32_t> slot_sub, slot_loc, slot_if, slot_mk;
  std::vector<int32_t> if_kind, if_dim, if_nsub, if_sub0, if_sub1, if_slot0, if_slot1, if_row;
  // members 2 and 3 of interfaces with more than two (2 entries per interface, -1 unused)
  std::vector<int32_t> if_subx, if_slotx;
  int32_t max_members = 1;
  std::vector<double> if_mu, if_k, if_alpha;
  std::vector<int32_t> sc_sub, sc_slot, sc_if, sc_dof;
  std::vector<int32_t> sub_hq, sub_wq, sc_hq, sc_wq;  // LDS layout of the iteration kernel
  int32_t max_hq_scene = 0, max_wq_scene = 0;
  // multi-step kernel: its LDS size and, per scene, the offset (doubles) of a global scratch
  // for the factorisations that do not fit in it (-1: none)
  size_t steps_lds = 0;
  std::vector<int32_t> sc_order;  // workgroup -> scene of the multi-step kernel
  std::vector<int64_t> sc_fscr;
  int64_t n_fscr = 0;
  std::vector<int32_t> lane_code;  // team kernel lane roles (n_scene x team_block)
  std::vector<int32_t> zmap;       // thread-per-interface kernel: interface of each thread (n_scene x zmap_block)
  int32_t zmap_block = 0;
  std::vector<int32_t> rmap;       // split-row lane roles (n_scene x rmap_block), then the
  int32_t rmap_block = 0;          // interface map for that block at zmap_split
  std::vector<int32_t> rmap_in;    // split rows within the default block (n_scene x zmap_block)
  size_t zmap_split = 0;
  // learned warm start
  std::vector<int32_t> if_class, if_krow;
  int32_t n_class[2] = {0, 0};
  subadmm_mlp* net[2] = {nullptr, nullptr};
  std::vector<int32_t> if_scene;
  float* rec_xc = nullptr;
  float* rec_xj = nullptr;
  float* rec_tc = nullptr;
  float* rec_tj = nullptr;
  float* rec_wc = nullptr;
  float* rec_wj = nullptr;
  bool recording() const { return rec_xc || rec_xj || rec_tc || rec_tj || rec_wc || rec_wj; }
  int32_t team_block = 0;          // 0: team kernel not usable for this problem
  int64_t n_dof = 0, n_slot = 0, n_rows = 0, n_A = 0, n_J = 0, n_H = 0;
  int32_t max_n = 0, max_nc = 0, max_slot_scene = 0, max_if_scene = 0, max_row_scene = 0, max_sub_scene = 0;
  int64_t max_h_scene = 0;
  // factorisation launches: subsystems grouped by DOF count
  std::vector<int32_t> fac_order;
  // global: the class of subsystems factorised with their working arrays in device memory
  struct Bucket { int32_t first, count, n, max_nc, global; };
  // per subsystem: byte offset of its device-memory factorisation arrays, -1 for the
  // subsystems factorised in LDS; their total bytes and count
  std::vector<int64_t> big_off;
  size_t big_bytes = 0;
  int32_t n_big = 0;
  std::vector<Bucket> buckets;

  // rigid model (host copy)
  bool has_rigid = false;
  int32_t nb = 0, nj = 0, ncon = 0;
  std::vector<int32_t> body_sub, body_local, sub_body, sub_body_off, if_src, joint_body, contact_body;
  std::vector<double> mass, inertia, joint_anchor, joint_frame, joint_axis_b, contact_point;
  // links (subadmm_rigid_set_links, before the model): rows in body a's frame
  int32_t nl = 0;
  std::vector<int32_t> link_type, link_body, link_if, link_dim;
  std::vector<double> link_anchor, link_frame, link_k, link_alpha;
  // soft links folded into a subsystem's dynamics (link_if < 0), grouped by subsystem
  std::vector<int32_t> sub_ilink_off, sub_ilink;
  double gravity = 9.81, baumgarte = 0.2;

  // limits of the per-scene (small-block) solver; when exceeded only the FEM path runs
  bool small_ok = true;
  std::string small_why;
  // every subsystem fits the per-subsystem factorisation; scenes beyond the per-scene
  // kernel (small_ok false) then iterate on the large-scene path
  bool sub_ok = true;
  std::string sub_why;
  int32_t force_large = 0;  // option SUBADMM_OPT_LARGE_PATH
  int32_t boyd = 0;         // option SUBADMM_OPT_BOYD_RESIDUALS
  bool boyd_valid = false;  // the last solve or step wrote r_prim and r_dual

  // FEM model (host copy and derived tables)
  bool has_fem = false;
  int32_t f_n_nodes = 0, f_n_tets = 0, f_max_m = 0, f_max_ng = 0;
  int64_t f_n_sq = 0, f_n_pairs = 0, f_n_pent = 0, f_n_dkey = 0;
  std::vector<int32_t> f_node_off, f_tet_off, f_tet_node, f_pair_off, f_pair_ab, f_pent_off, f_pent, f_node_diag,
      f_m, f_dkey_off, f_perm, f_jtj, f_slot_dk, f_slot_dof, f_dk_off, f_dk_slot, f_if_node0, f_if_node1;
  std::vector<float> f_slot_sgn;
  std::vector<double> f_tet_g, f_tet_vol, f_rest, f_mass, f_lame_l, f_lame_m;
  std::vector<int64_t> f_sq_off;

  // workspace
  char* ws = nullptr;
  size_t ws_bytes = 0;
  hipStream_t stream = nullptr;
  bool bound = false;
  // offsets
  struct {
    size_t sub_n, sub_nc, sub_dof, sub_slot, sub_A, sub_J, sub_H, slot_sub, slot_loc, slot_if, slot_mk;
    size_t if_subx, if_slotx;
    size_t if_kind, if_dim, if_nsub, if_sub0, if_sub1, if_slot0, if_slot1, if_row, sc_sub, sc_slot, sc_if,
        sc_dof, sub_hq, sub_wq, sc_hq, sc_wq, lane_code, if_class, if_krow, if_scene, zmap, rmap, rmap_in;
    size_t fac_order, big_off, fbig, sc_fscr, sfscr, sc_order, steps_args, sub_scene, ly, lu, lw, ldy, lyy, ldone, lall, err;
    size_t zp, up, zl, ul, vdof, xc, xj, yc, yj, st_fb;
    size_t beta, H, d, G, cvec, zw, uw, mu, ksoft, asoft, st_it, st_tot, st_unc, st_cv, st_th, st_rt, flags;
    size_t st_rp, st_rd;
    size_t r_body_sub, r_body_local, r_mass, r_inertia, r_sub_body, r_sub_body_off, r_if_src, r_joint_body,
        r_joint_anchor, r_joint_frame, r_joint_axis_b, r_contact_body, r_contact_point, r_link_type, r_link_body,
        r_link_anchor, r_link_frame, r_link_dim, r_link_k, r_link_alpha, r_sub_ilink_off, r_sub_ilink;
    size_t sA, sb, sJ, se, svh;
    size_t f_node_off, f_tet_off, f_tet_node, f_pair_off, f_pair_ab, f_pent_off, f_pent, f_node_diag, f_m,
        f_dkey_off, f_perm, f_jtj, f_slot_dk, f_slot_dof, f_dk_off, f_dk_slot, f_if_node0, f_if_node1, f_slot_sgn,
        f_tet_g, f_tet_vol, f_rest, f_mass, f_lame_l, f_lame_m, f_sq_off;
    size_t fA, fb, fL, fS, fcd, fscr, fe, fvh, fw, fy, fpart, fprec, fkest;
    size_t static_end;
    size_t total;
  } o{};
  std::vector<char> upload_keep;  // host staging kept alive until bind's synchronisation
  std::string err;
  // kernel timing (measurement support)
  bool timing = false;
  int32_t timing_max = 0, timing_used = 0, timing_dropped = 0;
  std::vector<hipEvent_t> ev0, ev1;
  // factorisation size classes run concurrently on side streams forked from the bound
  // stream and joined back into it (default priority)
  std::vector<hipStream_t> side;
  std::vector<hipEvent_t> side_ev;
  hipEvent_t fork_ev = nullptr;
  // captured rigid step (subadmm_rigid_step_graph) and the arguments it was captured with
  hipGraph_t graph = nullptr;
  hipGraphExec_t graph_exec = nullptr;
  // A captured step holds its launch arguments by value: options, the warm-start networks
  // and their workspaces, the recording pointers.  Every setter that changes one of them
  // advances cfg_gen (a network advances its own generation on bind and input-affine
  // changes), and the key compares those too, so a changed configuration captures again.
  uint64_t cfg_gen = 0;
  struct GraphKey {
    void *pos, *rot, *vel, *omega, *v_hat, *lambda;
    double dt, tol;
    int32_t max_iters, warm;
    uint64_t cfg_gen;
    const void *net0, *net1;
    uint64_t net_gen0, net_gen1;
    bool operator==(const GraphKey& o) const {
      return pos == o.pos && rot == o.rot && vel == o.vel && omega == o.omega && v_hat == o.v_hat &&
             lambda == o.lambda && dt == o.dt && tol == o.tol && max_iters == o.max_iters && warm == o.warm &&
             cfg_gen == o.cfg_gen && net0 == o.net0 && net1 == o.net1 && net_gen0 == o.net_gen0 &&
             net_gen1 == o.net_gen1;
    }
  } graph_key{};
  bool capturing = false;
  bool in_scratch = false;   // subadmm_solve_scratch is running (no host polling there)
  int32_t host_flag = 0;     // read back by the large-scene path's early exit
  hipStream_t cap_stream = nullptr;  // capture happens on this private stream (the bound
                                     // stream may be the device's null stream)
  std::vector<int32_t> ev_kernel;

  size_t rsize() const { return dtype == SUBADMM_F64 ? sizeof(double) : sizeof(float); }
};

namespace {

int fail(subadmm_problem* p, int code, const std::string& msg) {
  if (p) p->err = msg;
  else g_setup_error = msg;
  return code;
}

// LDS of the multi-step kernel and the scratch of the factorisations above it.
void plan_steps(subadmm_problem* p) {
  if ((int32_t)p->sc_order.size() != p->n_scene) {
    p->sc_order.resize(p->n_scene);
    for (int32_t s = 0; s < p->n_scene; ++s) p->sc_order[s] = s;
  }
  p->sc_fscr.assign(p->n_scene, -1);
  p->n_fscr = 0;
  p->steps_lds = 0;
  if (!p->small_ok) return;
  const size_t ns = (size_t)std::max<int32_t>(p->max_slot_scene, 1);
  const size_t with_h =
      16 * (size_t)p->max_hq_scene + p->rsize() * ((size_t)p->max_wq_scene + 2 * ns + (size_t)p->max_row_scene) + 64;
  p->steps_lds = std::max(with_h, kStepsLds);
  for (int32_t sc = 0; sc < p->n_scene; ++sc) {
    size_t big = 0;
    for (int32_t i = p->sc_sub[sc]; i < p->sc_sub[sc + 1]; ++i) {
      const size_t b = factor_bytes(p->sub_n[i], p->sub_nc[i], sizeof(double));
      if (b > p->steps_lds) big = std::max(big, b);
    }
    if (big) {
      p->sc_fscr[sc] = p->n_fscr;
      p->n_fscr += (int64_t)((big / sizeof(double) + 31) / 32 * 32);
    }
  }
}

void plan_workspace(subadmm_problem* p) {
  p->upload_keep.clear();  // staged tables describe the previous layout
  plan_steps(p);
  Plan pl;
  auto& o = p->o;
  const size_t R = p->rsize();
  auto real = [&](size_t count) {
    pl.off = (pl.off + 255) & ~size_t(255);
    const size_t off = pl.off;
    pl.off += R * (count > 0 ? count : 1);
    return off;
  };
  o.sub_n = pl.take<int32_t>(p->n_sub);
  o.sub_nc = pl.take<int32_t>(p->n_sub);
  o.sub_dof = pl.take<int32_t>(p->n_sub + 1);
  o.sub_slot = pl.take<int32_t>(p->n_sub + 1);
  o.sub_A = pl.take<int64_t>(p->n_sub + 1);
  o.sub_J = pl.take<int64_t>(p->n_sub + 1);
  o.sub_H = pl.take<int64_t>(p->n_sub + 1);
  o.slot_sub = pl.take<int32_t>(p->n_slot);
  o.slot_loc = pl.take<int32_t>(p->n_slot);
  o.slot_if = pl.take<int32_t>(p->n_slot);
  o.slot_mk = pl.take<int32_t>(p->n_slot);
  o.if_kind = pl.take<int32_t>(p->n_if);
  o.if_dim = pl.take<int32_t>(p->n_if);
  o.if_nsub = pl.take<int32_t>(p->n_if);
  o.if_sub0 = pl.take<int32_t>(p->n_if);
  o.if_sub1 = pl.take<int32_t>(p->n_if);
  o.if_slot0 = pl.take<int32_t>(p->n_if);
  o.if_subx = pl.take<int32_t>(2 * (size_t)p->n_if);
  o.if_slotx = pl.take<int32_t>(2 * (size_t)p->n_if);
  o.if_slot1 = pl.take<int32_t>(p->n_if);
  o.if_row = pl.take<int32_t>(p->n_if + 1);
  o.sc_sub = pl.take<int32_t>(p->n_scene + 1);
  o.sc_slot = pl.take<int32_t>(p->n_scene + 1);
  o.sc_if = pl.take<int32_t>(p->n_scene + 1);
  o.sc_dof = pl.take<int32_t>(p->n_scene + 1);
  o.sub_hq = pl.take<int32_t>(p->n_sub);
  o.sub_wq = pl.take<int32_t>(p->n_sub);
  o.sc_hq = pl.take<int32_t>(p->n_scene);
  o.sc_wq = pl.take<int32_t>(p->n_scene);
  o.lane_code = pl.take<int32_t>(p->lane_code.size());
  o.zmap = pl.take<int32_t>(p->zmap.size());
  o.rmap = pl.take<int32_t>(p->rmap.size());
  o.rmap_in = pl.take<int32_t>(p->rmap_in.size());
  o.if_class = pl.take<int32_t>(p->n_if);
  o.if_krow = pl.take<int32_t>(p->n_if);
  o.if_scene = pl.take<int32_t>(p->n_if);
  o.fac_order = pl.take<int32_t>(p->n_sub);
  o.big_off = pl.take<int64_t>(p->n_sub);
  o.sc_fscr = pl.take<int64_t>(p->n_scene);
  o.sc_order = pl.take<int32_t>(p->n_scene);
  o.sub_scene = pl.take<int32_t>(p->n_sub);
  if (p->has_fem) {
    o.f_node_off = pl.take<int32_t>(p->f_node_off.size());
    o.f_tet_off = pl.take<int32_t>(p->f_tet_off.size());
    o.f_tet_node = pl.take<int32_t>(p->f_tet_node.size());
    o.f_pair_off = pl.take<int32_t>(p->f_pair_off.size());
    o.f_pair_ab = pl.take<int32_t>(p->f_pair_ab.size());
    o.f_pent_off = pl.take<int32_t>(p->f_pent_off.size());
    o.f_pent = pl.take<int32_t>(p->f_pent.size());
    o.f_node_diag = pl.take<int32_t>(p->f_node_diag.size());
    o.f_m = pl.take<int32_t>(p->f_m.size());
    o.f_dkey_off = pl.take<int32_t>(p->f_dkey_off.size());
    o.f_perm = pl.take<int32_t>(p->f_perm.size());
    o.f_jtj = pl.take<int32_t>(p->f_jtj.size());
    o.f_slot_dk = pl.take<int32_t>(p->f_slot_dk.size());
    o.f_slot_dof = pl.take<int32_t>(p->f_slot_dof.size());
    o.f_dk_off = pl.take<int32_t>(p->f_dk_off.size());
    o.f_dk_slot = pl.take<int32_t>(p->f_dk_slot.size());
    o.f_if_node0 = pl.take<int32_t>(p->f_if_node0.size());
    o.f_if_node1 = pl.take<int32_t>(p->f_if_node1.size());
    o.f_slot_sgn = pl.take<float>(p->f_slot_sgn.size());
    o.f_tet_g = pl.take<double>(p->f_tet_g.size());
    o.f_tet_vol = pl.take<double>(p->f_tet_vol.size());
    o.f_rest = pl.take<double>(p->f_rest.size());
    o.f_mass = pl.take<double>(p->f_mass.size());
    o.f_lame_l = pl.take<double>(p->f_lame_l.size());
    o.f_lame_m = pl.take<double>(p->f_lame_m.size());
    o.f_sq_off = pl.take<int64_t>(p->f_sq_off.size());
  }
  o.mu = real(p->n_if);
  o.ksoft = real(p->n_if);
  o.asoft = real(p->n_if);
  if (p->has_rigid) {
    o.r_body_sub = pl.take<int32_t>(p->nb);
    o.r_body_local = pl.take<int32_t>(p->nb);
    o.r_mass = real(p->nb);
    o.r_inertia = real(3 * (size_t)p->nb);
    o.r_sub_body = pl.take<int32_t>(p->nb);
    o.r_sub_body_off = pl.take<int32_t>(p->n_sub + 1);
    o.r_if_src = pl.take<int32_t>(p->n_if);
    o.r_joint_body = pl.take<int32_t>(2 * (size_t)p->nj);
    o.r_joint_anchor = real(6 * (size_t)p->nj);
    o.r_joint_frame = real(9 * (size_t)p->nj);
    o.r_joint_axis_b = real(3 * (size_t)p->nj);
    o.r_contact_body = pl.take<int32_t>(p->ncon);
    o.r_contact_point = real(3 * (size_t)p->ncon);
    o.r_link_type = pl.take<int32_t>(p->nl);
    o.r_link_body = pl.take<int32_t>(2 * (size_t)p->nl);
    o.r_link_anchor = real(6 * (size_t)p->nl);
    o.r_link_frame = real(9 * (size_t)p->nl);
    o.r_link_dim = pl.take<int32_t>(p->nl);
    o.r_link_k = real(p->nl);
    o.r_link_alpha = real(p->nl);
    o.r_sub_ilink_off = pl.take<int32_t>(p->n_sub + 1);
    o.r_sub_ilink = pl.take<int32_t>(p->sub_ilink.size());
  }
  // everything above is uploaded at bind; everything below starts as zeros
  o.static_end = (pl.off + 255) & ~size_t(255);
  o.beta = real(p->n_sub);
  o.H = real(p->sub_ok ? p->n_H : 0);
  o.d = real(p->sub_ok ? p->n_slot : 0);
  o.G = real(p->sub_ok ? p->n_J : 0);
  o.cvec = real(p->sub_ok ? p->n_dof : 0);
  o.fbig = pl.take<char>(p->sub_ok ? p->big_bytes : 0);
  // large-scene iteration state (per slot row) and per-scene stop flags
  o.ly = real(p->sub_ok ? p->n_slot : 0);
  o.lu = real(p->sub_ok ? p->n_slot : 0);
  o.lw = real(p->sub_ok ? p->n_slot : 0);
  o.ldy = pl.take<double>(p->sub_ok ? p->n_slot : 0);
  o.lyy = pl.take<double>(p->sub_ok ? p->n_slot : 0);
  o.ldone = pl.take<int32_t>(p->n_scene);
  o.lall = pl.take<int32_t>(1);
  o.err = pl.take<double>(p->n_scene);
  o.zw = real(p->n_slot);
  o.uw = real(p->n_slot);
  o.st_it = pl.take<int32_t>(p->n_scene);
  o.st_tot = pl.take<long long>(p->n_scene);
  o.st_unc = pl.take<long long>(p->n_scene);
  o.st_cv = pl.take<int32_t>(p->n_scene);
  o.st_th = pl.take<double>(p->n_scene);
  o.st_rt = pl.take<double>(p->n_scene);
  o.st_rp = pl.take<double>(p->n_scene);
  o.st_rd = pl.take<double>(p->n_scene);
  o.flags = pl.take<int32_t>(1);
  o.st_fb = pl.take<long long>(p->n_scene);
  if (p->has_rigid) {
    o.sA = real(p->n_A);
    o.sb = real(p->n_dof);
    o.sJ = real(p->n_J);
    o.se = real(p->n_rows);
    o.svh = real(p->n_dof);
    o.zp = real(p->n_slot);
    o.up = real(p->n_slot);
    o.zl = real(p->n_slot);
    o.ul = real(p->n_slot);
    o.vdof = real(p->n_dof);
    o.sfscr = pl.take<double>((size_t)p->n_fscr);
    o.steps_args = pl.take<char>(sizeof(StepsArgs<double>));
    o.xc = pl.take<float>((size_t)kContactIn * p->n_class[0]);
    o.xj = pl.take<float>((size_t)kJointIn * p->n_class[1]);
    o.yc = pl.take<float>((size_t)kContactOut * p->n_class[0]);
    o.yj = pl.take<float>((size_t)kJointOut * p->n_class[1]);
  }
  if (p->has_fem) {
    o.fA = pl.take<double>(p->n_A);
    o.fb = pl.take<double>(p->n_dof);
    o.fL = pl.take<double>(p->n_A);
    o.fS = real(p->f_n_sq);
    o.fcd = real(p->f_n_dkey);
    o.fscr = pl.take<double>(18 * (size_t)p->f_n_tets);
    o.fe = real(p->n_rows);
    o.fvh = real(p->n_dof);
    o.fw = real(p->n_slot);
    o.fy = real(3 * (size_t)p->n_slot);
    o.fpart = pl.take<double>(6 * (size_t)kPartCopies * p->n_sub);
    o.fprec = pl.take<int32_t>(p->n_sub);
    o.fkest = pl.take<double>(p->n_sub);
  }
  o.total = (pl.off + 255) & ~size_t(255);
}

template <typename X>
X* at(subadmm_problem* p, size_t off) {
  return reinterpret_cast<X*>(p->ws + off);
}

Topo make_topo(subadmm_problem* p) {
  Topo t;
  t.n_sub = p->n_sub;
  t.n_if = p->n_if;
  t.n_scene = p->n_scene;
  t.max_row_scene = p->max_row_scene;
  auto& o = p->o;
  t.sub_n = at<int32_t>(p, o.sub_n);
  t.sub_nc = at<int32_t>(p, o.sub_nc);
  t.sub_dof = at<int32_t>(p, o.sub_dof);
  t.sub_slot = at<int32_t>(p, o.sub_slot);
  t.sub_A = at<int64_t>(p, o.sub_A);
  t.sub_J = at<int64_t>(p, o.sub_J);
  t.sub_H = at<int64_t>(p, o.sub_H);
  t.slot_sub = at<int32_t>(p, o.slot_sub);
  t.slot_loc = at<int32_t>(p, o.slot_loc);
  t.slot_if = at<int32_t>(p, o.slot_if);
  t.slot_mk = at<int32_t>(p, o.slot_mk);
  t.if_kind = at<int32_t>(p, o.if_kind);
  t.if_dim = at<int32_t>(p, o.if_dim);
  t.if_nsub = at<int32_t>(p, o.if_nsub);
  t.if_sub0 = at<int32_t>(p, o.if_sub0);
  t.if_sub1 = at<int32_t>(p, o.if_sub1);
  t.if_slot0 = at<int32_t>(p, o.if_slot0);
  t.if_subx = at<int32_t>(p, o.if_subx);
  t.if_slotx = at<int32_t>(p, o.if_slotx);
  t.if_slot1 = at<int32_t>(p, o.if_slot1);
  t.if_row = at<int32_t>(p, o.if_row);
  t.sc_sub = at<int32_t>(p, o.sc_sub);
  t.sc_slot = at<int32_t>(p, o.sc_slot);
  t.sc_if = at<int32_t>(p, o.sc_if);
  t.sc_dof = at<int32_t>(p, o.sc_dof);
  t.sub_hq = at<int32_t>(p, o.sub_hq);
  t.sub_wq = at<int32_t>(p, o.sub_wq);
  t.sc_hq = at<int32_t>(p, o.sc_hq);
  t.sc_wq = at<int32_t>(p, o.sc_wq);
  t.lane_code = at<int32_t>(p, o.lane_code);
  t.team_block = p->team_block;
  t.zmap = p->zmap.empty() ? nullptr : at<int32_t>(p, o.zmap);
  t.zmap_block = p->zmap_block;
  t.rmap = nullptr;
  t.rmap_block = 0;
  if (p->split_rows == 2 && !p->rmap_in.empty()) {
    t.rmap = at<int32_t>(p, o.rmap_in);
    t.rmap_block = p->zmap_block;
  } else if (p->split_rows == 1 && p->rmap_block > 0) {
    t.rmap = at<int32_t>(p, o.rmap);
    t.rmap_block = p->rmap_block;
    t.zmap = at<int32_t>(p, o.zmap) + p->zmap_split;
    t.zmap_block = p->rmap_block;
  }
  return t;
}

template <typename T>
RigidModel<T> make_rigid(subadmm_problem* p) {
  RigidModel<T> m;
  auto& o = p->o;
  m.nb = p->nb;
  m.nj = p->nj;
  m.ncon = p->ncon;
  m.body_sub = at<int32_t>(p, o.r_body_sub);
  m.body_local = at<int32_t>(p, o.r_body_local);
  m.mass = at<T>(p, o.r_mass);
  m.inertia = at<T>(p, o.r_inertia);
  m.sub_body = at<int32_t>(p, o.r_sub_body);
  m.sub_body_off = at<int32_t>(p, o.r_sub_body_off);
  m.if_src = at<int32_t>(p, o.r_if_src);
  m.joint_body = at<int32_t>(p, o.r_joint_body);
  m.joint_anchor = at<T>(p, o.r_joint_anchor);
  m.joint_frame = at<T>(p, o.r_joint_frame);
  m.joint_axis_b = at<T>(p, o.r_joint_axis_b);
  m.contact_body = at<int32_t>(p, o.r_contact_body);
  m.contact_point = at<T>(p, o.r_contact_point);
  m.nl = p->nl;
  m.link_type = at<int32_t>(p, o.r_link_type);
  m.link_body = at<int32_t>(p, o.r_link_body);
  m.link_anchor = at<T>(p, o.r_link_anchor);
  m.link_frame = at<T>(p, o.r_link_frame);
  m.link_dim = at<int32_t>(p, o.r_link_dim);
  m.link_k = at<T>(p, o.r_link_k);
  m.link_alpha = at<T>(p, o.r_link_alpha);
  m.sub_ilink_off = at<int32_t>(p, o.r_sub_ilink_off);
  m.sub_ilink = at<int32_t>(p, o.r_sub_ilink);
  m.gravity = (T)p->gravity;
  m.baumgarte = (T)p->baumgarte;
  return m;
}

int dev_err(subadmm_problem* p, hipError_t e, const char* where) {
  if (e == hipSuccess) return SUBADMM_OK;
  return fail(p, SUBADMM_E_DEVICE, std::string(where) + ": " + hipGetErrorString(e));
}

// Factorisation launches.  Subsystems are grouped into LDS size classes (so that the
// many small subsystems are not held to the occupancy of the largest one) and ordered
// largest first inside a class; classes are launched largest first.
void plan_factor(subadmm_problem* p) {
  const size_t cs = p->factor_fp64 ? sizeof(double) : p->rsize();
  auto need = [&](int32_t i) { return factor_bytes(p->sub_n[i], p->sub_nc[i], cs); };
  static const size_t kClass[] = {8 * 1024, 24 * 1024, 48 * 1024, 96 * 1024, 160 * 1024};
  auto cls = [&](int32_t i) {
    const size_t b = need(i);
    int k = 0;
    while (k < 4 && b > kClass[k]) ++k;
    return k;
  };
  // the device-memory class first (largest first), then the LDS classes
  auto big = [&](int32_t i) { return p->big_off.size() == (size_t)p->n_sub && p->big_off[i] >= 0; };
  p->fac_order.resize(p->n_sub);
  for (int32_t i = 0; i < p->n_sub; ++i) p->fac_order[i] = i;
  std::stable_sort(p->fac_order.begin(), p->fac_order.end(), [&](int32_t a, int32_t b) {
    if (big(a) != big(b)) return big(a);
    const int ca = cls(a), cb = cls(b);
    if (ca != cb) return ca > cb;
    return need(a) > need(b);
  });
  p->buckets.clear();
  int32_t k0 = 0;
  if (p->n_big > 0) {
    subadmm_problem::Bucket g{0, p->n_big, 0, 0, 1};
    for (int32_t k = 0; k < p->n_big; ++k) {
      g.n = std::max(g.n, p->sub_n[p->fac_order[k]]);
      g.max_nc = std::max(g.max_nc, p->sub_nc[p->fac_order[k]]);
    }
    p->buckets.push_back(g);
    k0 = p->n_big;
  }
  int last = -1;
  for (int32_t k = k0; k < p->n_sub; ++k) {
    const int32_t i = p->fac_order[k];
    const int c = cls(i);
    if (c != last) {
      p->buckets.push_back({k, 0, 0, 0, 0});
      last = c;
    }
    auto& bk = p->buckets.back();
    bk.count++;
    bk.n = std::max(bk.n, p->sub_n[i]);
    bk.max_nc = std::max(bk.max_nc, p->sub_nc[i]);
  }
  // a class's joint maximum (largest n with largest nc) must still fit
  std::vector<subadmm_problem::Bucket> split;
  for (const auto& bk : p->buckets) {
    if (bk.global || factor_bytes(bk.n, bk.max_nc, cs) <= 150 * 1024) {
      split.push_back(bk);
      continue;
    }
    for (int32_t k = bk.first; k < bk.first + bk.count; ++k) {
      const int32_t i = p->fac_order[k];
      split.push_back({k, 1, p->sub_n[i], p->sub_nc[i], 0});
    }
  }
  p->buckets.swap(split);
}

// Runs one kernel launcher, bracketed by events on the bound stream while timing is on.
template <typename F>
hipError_t timed(subadmm_problem* p, int32_t kernel, F&& launch) {
  if (!p->timing || p->capturing) return launch();
  if (p->timing_used >= p->timing_max) {
    ++p->timing_dropped;
    return launch();
  }
  const int32_t k = p->timing_used++;
  hipError_t e = hipEventRecord(p->ev0[k], p->stream);
  if (e != hipSuccess) return e;
  e = launch();
  if (e != hipSuccess) return e;
  p->ev_kernel[k] = kernel;
  return hipEventRecord(p->ev1[k], p->stream);
}

// Event pair around a stretch of launches that is not one hipError_t call (the learned
// start: features, networks, apply); -1 when not timing.
int timing_begin_span(subadmm_problem* p) {
  if (!p->timing || p->capturing) return -1;
  if (p->timing_used >= p->timing_max) {
    ++p->timing_dropped;
    return -1;
  }
  const int32_t k = p->timing_used++;
  return hipEventRecord(p->ev0[k], p->stream) == hipSuccess ? k : -1;
}

void timing_end_span(subadmm_problem* p, int k, int32_t kernel) {
  if (k < 0) return;
  p->ev_kernel[k] = kernel;
  (void)hipEventRecord(p->ev1[k], p->stream);
}

template <typename T>
int run_factor(subadmm_problem* p, const T* A, const T* b, const T* J) {
  auto& o = p->o;
  FactorArgs<T> fa;
  fa.t = make_topo(p);
  fa.A = A;
  fa.b = b;
  fa.J = J;
  fa.rho = p->rho;
  fa.beta = at<T>(p, o.beta);
  fa.H = at<T>(p, o.H);
  fa.d = at<T>(p, o.d);
  fa.G = at<T>(p, o.G);
  fa.cvec = at<T>(p, o.cvec);
  fa.flags = at<int32_t>(p, o.flags);
  fa.order = at<int32_t>(p, o.fac_order);
  const bool fork = p->factor_streams && !p->side.empty() && p->buckets.size() > 1;
  auto launch_bucket = [&](const FactorArgs<T>& f, const subadmm_problem::Bucket& bk, hipStream_t s) {
    return bk.global ? launch_factor_global<T>(f, bk.count, bk.n, p->factor_fp64 != 0, at<char>(p, o.fbig),
                                               at<int64_t>(p, o.big_off), s)
                     : launch_factor<T>(f, bk.count, bk.n, bk.max_nc, p->factor_fp64 != 0, s);
  };
  return dev_err(p, timed(p, SUBADMM_K_FACTOR, [&] {
                   hipError_t e = hipSuccess;
                   if (fork) e = hipEventRecord(p->fork_ev, p->stream);
                   for (size_t k = 1; k < p->buckets.size() && e == hipSuccess; ++k) {
                     const auto& bk = p->buckets[k];
                     FactorArgs<T> fk = fa;
                     fk.first = bk.first;
                     hipStream_t s = fork ? p->side[(k - 1) % p->side.size()] : p->stream;
                     if (fork) e = hipStreamWaitEvent(s, p->fork_ev, 0);
                     if (e == hipSuccess) e = launch_bucket(fk, bk, s);
                     if (e == hipSuccess && fork) e = hipEventRecord(p->side_ev[k - 1], s);
                   }
                   if (e == hipSuccess && !p->buckets.empty()) {
                     const auto& bk = p->buckets[0];
                     FactorArgs<T> f0 = fa;
                     f0.first = bk.first;
                     e = launch_bucket(f0, bk, p->stream);
                   }
                   for (size_t k = 1; fork && k < p->buckets.size() && e == hipSuccess; ++k)
                     e = hipStreamWaitEvent(p->stream, p->side_ev[k - 1], 0);
                   return e;
                 }),
                 "factor kernel");
}

// Workgroup size of the per-scene large-scene form: a thread per slot row of the largest
// scene, 256 to 1024 (on the mixed workload's scenes of ~1.5k slot rows 1024 threads take
// 0.6 of the time per step of 256).
int large_threads(const subadmm_problem* p) {
  const int32_t need = (std::max(p->max_slot_scene, p->max_if_scene) + 63) / 64 * 64;
  return std::min<int32_t>(1024, std::max<int32_t>(256, need));
}

// One launch of the iteration from (z_in, u_in) (nullptr: cold); final (z, u) go to the
// kept warm buffers.  skip: scenes flagged there are left untouched (fallback runs).
template <typename T>
int run_loop(subadmm_problem* p, const T* e, int32_t max_iters, double tol, const T* z_in, const T* u_in, T* v_hat,
             T* lambda, const int32_t* skip, long long* fallback_count) {
  auto& o = p->o;
  LoopArgs<T> la;
  la.t = make_topo(p);
  la.beta = at<T>(p, o.beta);
  la.H = at<T>(p, o.H);
  la.d = at<T>(p, o.d);
  la.G = at<T>(p, o.G);
  la.cvec = at<T>(p, o.cvec);
  la.e = e;
  la.mu = at<T>(p, o.mu);
  la.ksoft = at<T>(p, o.ksoft);
  la.asoft = at<T>(p, o.asoft);
  la.z_in = z_in;
  la.u_in = u_in;
  la.z_out = at<T>(p, o.zw);
  la.u_out = at<T>(p, o.uw);
  la.v_hat = v_hat;
  la.lambda = lambda;
  la.st_iters = at<int32_t>(p, o.st_it);
  la.st_total = at<long long>(p, o.st_tot);
  la.st_unconv = at<long long>(p, o.st_unc);
  la.st_conv = at<int32_t>(p, o.st_cv);
  la.st_theta = at<double>(p, o.st_th);
  la.st_rtheta = at<double>(p, o.st_rt);
  la.flags = at<int32_t>(p, o.flags);
  la.max_iters = max_iters;
  la.tol = tol;
  la.contact_model = p->contact_model;
  la.skip_converged = skip;
  la.st_fallback = fallback_count;
  if (!p->small_ok || p->force_large) {
    if (skip) return fail(p, SUBADMM_E_ARG, "the learned start needs scenes that fit the per-scene kernel");
    LargeArgs<T> lg;
    lg.l = la;
    lg.sub_scene = at<int32_t>(p, o.sub_scene);
    lg.y = at<T>(p, o.ly);
    lg.u = at<T>(p, o.lu);
    lg.w = at<T>(p, o.lw);
    lg.dy2 = at<double>(p, o.ldy);
    lg.yy2 = at<double>(p, o.lyy);
    lg.done = at<int32_t>(p, o.ldone);
    lg.all_done = at<int32_t>(p, o.lall);
    lg.n_slot = p->n_slot;
    lg.n_dof = p->n_dof;
    // eager steps stop launching once every scene has stopped (checked every 32 iterations);
    // a captured graph and the scratch entry launch every permitted iteration
    const int poll = (p->capturing || p->in_scratch) ? 0 : kLargePoll;
    // scenes of a few thousand slot rows: one workgroup carries each scene's iteration in one
    // launch; larger ones (a single long cable) need the whole GPU per phase
    const bool per_scene = p->force_large != 2 && p->max_slot_scene <= kLargeSceneMax;
    return dev_err(p, timed(p, SUBADMM_K_LOOP, [&] {
                     return per_scene ? launch_large_scene<T>(lg, large_threads(p), p->stream)
                                      : launch_large_loop<T>(lg, p->stream, poll, &p->host_flag);
                   }),
                   "large-scene iteration");
  }
  return dev_err(p, timed(p, SUBADMM_K_LOOP, [&] {
                   if (p->use_team == 2)
                     return launch_wave_loop<T>(la, p->max_slot_scene, p->max_if_scene, p->max_hq_scene,
                                                p->max_wq_scene, p->stream);
                   if (p->team_block > 0 && p->use_team)
                     return launch_team_loop<T>(la, p->max_hq_scene, p->max_wq_scene, p->stream);
                   return launch_loop<T>(la, p->max_slot_scene, p->max_if_scene, p->max_h_scene, p->max_hq_scene,
                                         p->max_wq_scene, p->max_nc, p->stream);
                 }),
                 "loop kernel");
}

// ADMM's primal and dual residuals of the returned (z, u) (option BOYD_RESIDUALS), from the
// operators of the solve just run and its e; timed with the iteration.
template <typename T>
int run_boyd(subadmm_problem* p, const T* e) {
  p->boyd_valid = false;
  if (!p->boyd || !p->sub_ok) return SUBADMM_OK;
  auto& o = p->o;
  LargeArgs<T> lg{};
  lg.l.t = make_topo(p);
  lg.l.beta = at<T>(p, o.beta);
  lg.l.H = at<T>(p, o.H);
  lg.l.d = at<T>(p, o.d);
  lg.l.e = e;
  lg.l.mu = at<T>(p, o.mu);
  lg.l.ksoft = at<T>(p, o.ksoft);
  lg.l.asoft = at<T>(p, o.asoft);
  lg.l.contact_model = p->contact_model;
  lg.l.z_in = at<T>(p, o.zw);
  lg.l.u_in = at<T>(p, o.uw);
  lg.sub_scene = at<int32_t>(p, o.sub_scene);
  lg.y = at<T>(p, o.ly);
  lg.u = at<T>(p, o.lu);
  lg.w = at<T>(p, o.lw);
  lg.dy2 = at<double>(p, o.ldy);
  lg.yy2 = at<double>(p, o.lyy);
  lg.n_slot = p->n_slot;
  lg.n_dof = p->n_dof;
  const int rc = dev_err(p, timed(p, SUBADMM_K_LOOP, [&] {
                           return launch_boyd_residuals<T>(lg, at<double>(p, o.st_rp), at<double>(p, o.st_rd),
                                                           p->stream);
                         }),
                         "residual pair kernel");
  p->boyd_valid = rc == SUBADMM_OK;
  return rc;
}

template <typename T>
int run_solve(subadmm_problem* p, const T* A, const T* b, const T* J, const T* e, int32_t max_iters, double tol,
              int32_t warm, const T* z0, const T* u0, T* v_hat, T* lambda) {
  p->boyd_valid = false;
  int rc = run_factor<T>(p, A, b, J);
  if (rc) return rc;
  const T* zi = nullptr;
  const T* ui = nullptr;
  if (warm == SUBADMM_WARM_PREV) {
    zi = at<T>(p, p->o.zw);
    ui = at<T>(p, p->o.uw);
  } else if (warm == SUBADMM_WARM_GIVEN) {
    zi = z0;
    ui = u0;
  }
  rc = run_loop<T>(p, e, max_iters, tol, zi, ui, v_hat, lambda, nullptr, nullptr);
  return rc ? rc : run_boyd<T>(p, e);
}

int check_solve_args(subadmm_problem* p, int32_t max_iters, double tol, int32_t warm, const void* z0,
                     const void* u0) {
  if (!p) return fail(nullptr, SUBADMM_E_ARG, "null problem");
  if (!p->bound) return fail(p, SUBADMM_E_WORKSPACE, "problem has no bound workspace");
  if (max_iters < 1) return fail(p, SUBADMM_E_ARG, "max_iters must be >= 1");
  if (!(tol >= 0.0) || !std::isfinite(tol)) return fail(p, SUBADMM_E_ARG, "tol must be finite and >= 0");
  if (warm < SUBADMM_WARM_COLD || warm > SUBADMM_WARM_GIVEN) return fail(p, SUBADMM_E_ARG, "unknown warm mode");
  if (warm == SUBADMM_WARM_GIVEN && (!z0 || !u0)) return fail(p, SUBADMM_E_ARG, "warm GIVEN needs z0 and u0");
  return SUBADMM_OK;
}

}  // namespace

SUBADMM_API int subadmm_setup(const subadmm_subsystem* subs, int32_t n_sub, const subadmm_interface* ifs,
                              int32_t n_if, double rho, int32_t dtype, subadmm_problem** out) {
  if (!out) return fail(nullptr, SUBADMM_E_ARG, "out is null");
  *out = nullptr;
  if (n_sub < 1 || !subs) return fail(nullptr, SUBADMM_E_ARG, "need at least one subsystem");
  if (n_if < 0 || (n_if > 0 && !ifs)) return fail(nullptr, SUBADMM_E_ARG, "bad interface list");
  if (dtype != SUBADMM_F32 && dtype != SUBADMM_F64) return fail(nullptr, SUBADMM_E_ARG, "dtype must be F32 or F64");
  if (!std::isfinite(rho)) return fail(nullptr, SUBADMM_E_ARG, "rho must be finite");
  auto* p = new subadmm_problem();
  p->dtype = dtype;
  p->rho = rho;
  p->n_sub = n_sub;
  p->n_if = n_if;
  auto bad = [&](const std::string& m) {
    delete p;
    return fail(nullptr, SUBADMM_E_ARG, m);
  };
  // subsystems and scenes
  for (int32_t i = 0; i < n_sub; ++i) {
    const int32_t n = subs[i].n_dof, s = subs[i].scene;
    if (n < 1 || n > kMaxFemDof) return bad("subsystem " + std::to_string(i) + ": n_dof must be in 1..768");
    if (i == 0 ? s != 0 : (s != subs[i - 1].scene && s != subs[i - 1].scene + 1))
      return bad("subsystem " + std::to_string(i) + ": scenes must start at 0 and be contiguous");
    p->sub_n.push_back(n);
    p->sub_scene.push_back(s);
  }
  p->n_scene = subs[n_sub - 1].scene + 1;
  // interfaces
  std::vector<int32_t> nc(n_sub, 0);
  int32_t prev_scene = 0;
  p->if_row.assign(n_if + 1, 0);
  for (int32_t j = 0; j < n_if; ++j) {
    const auto& f = ifs[j];
    const std::string tag = "interface " + std::to_string(j) + ": ";
    if (f.kind < SUBADMM_IF_EQUALITY || f.kind > SUBADMM_IF_SOFT) return bad(tag + "unknown kind");
    if (f.kind == SUBADMM_IF_SOFT && (!(f.k >= 0.0) || !std::isfinite(f.k) || !(f.alpha > 0.0) || !std::isfinite(f.alpha)))
      return bad(tag + "a soft interface needs a finite gain k >= 0 and alpha > 0");
    if (f.dim < 1 || f.dim > kMaxIfDim) return bad(tag + "dim must be in 1..6");
    if (f.kind == SUBADMM_IF_CONTACT && f.dim != 3) return bad(tag + "contact interfaces have dim 3");
    if (f.n_sub < 1 || f.n_sub > SUBADMM_MAX_MEMBERS) return bad(tag + "n_sub must be in 1..4");
    for (int m = 0; m < f.n_sub; ++m) {
      if (f.sub[m] < 0 || f.sub[m] >= n_sub) return bad(tag + "member out of range");
      for (int q = 0; q < m; ++q)
        if (f.sub[q] == f.sub[m]) return bad(tag + "members must differ");
    }
    const int32_t sc = p->sub_scene[f.sub[0]];
    for (int m = 1; m < f.n_sub; ++m)
      if (p->sub_scene[f.sub[m]] != sc) return bad(tag + "members in different scenes");
    if (sc < prev_scene) return bad(tag + "interfaces must be grouped by scene in scene order");
    prev_scene = sc;
    if (!(f.mu >= 0.0) || !std::isfinite(f.mu)) return bad(tag + "mu must be finite and >= 0");
    p->if_kind.push_back(f.kind);
    p->if_dim.push_back(f.dim);
    p->if_nsub.push_back(f.n_sub);
    p->if_sub0.push_back(f.sub[0]);
    p->if_sub1.push_back(f.n_sub >= 2 ? f.sub[1] : -1);
    p->if_subx.push_back(f.n_sub >= 3 ? f.sub[2] : -1);
    p->if_subx.push_back(f.n_sub >= 4 ? f.sub[3] : -1);
    p->max_members = std::max<int32_t>(p->max_members, f.n_sub);
    p->if_mu.push_back(f.mu);
    p->if_k.push_back(f.kind == SUBADMM_IF_SOFT ? f.k : 0.0);
    p->if_alpha.push_back(f.kind == SUBADMM_IF_SOFT ? f.alpha : 0.0);
    p->if_row[j + 1] = p->if_row[j] + f.dim;
    for (int m = 0; m < f.n_sub; ++m) nc[f.sub[m]] += f.dim;
  }
  // subsystem offsets
  p->sub_dof.assign(n_sub + 1, 0);
  p->sub_slot.assign(n_sub + 1, 0);
  p->sub_A.assign(n_sub + 1, 0);
  p->sub_J.assign(n_sub + 1, 0);
  p->sub_H.assign(n_sub + 1, 0);
  p->sub_nc = nc;
  for (int32_t i = 0; i < n_sub; ++i) {
    const int64_t n = p->sub_n[i];
    p->sub_dof[i + 1] = p->sub_dof[i] + (int32_t)n;
    p->sub_slot[i + 1] = p->sub_slot[i] + nc[i];
    p->sub_A[i + 1] = p->sub_A[i] + n * n;
    p->sub_J[i + 1] = p->sub_J[i] + (int64_t)nc[i] * n;
    p->sub_H[i + 1] = p->sub_H[i] + (int64_t)nc[i] * nc[i];
    p->max_n = std::max<int32_t>(p->max_n, (int32_t)n);
    p->max_nc = std::max<int32_t>(p->max_nc, nc[i]);
  }
  p->n_dof = p->sub_dof[n_sub];
  p->n_slot = p->sub_slot[n_sub];
  p->n_rows = p->if_row[n_if];
  p->n_A = p->sub_A[n_sub];
  p->n_J = p->sub_J[n_sub];
  p->n_H = p->sub_H[n_sub];
  if (p->n_slot >= INT32_MAX / 2 || p->n_dof >= INT32_MAX / 2) return bad("problem too large");
  // slot rows
  p->slot_sub.assign(p->n_slot, 0);
  p->slot_loc.assign(p->n_slot, 0);
  p->slot_if.assign(p->n_slot, 0);
  p->slot_mk.assign(p->n_slot, 0);
  p->if_slot0.assign(n_if, -1);
  p->if_slot1.assign(n_if, -1);
  p->if_slotx.assign(2 * (size_t)n_if, -1);
  std::vector<int32_t> cur(p->sub_slot.begin(), p->sub_slot.end() - 1);
  for (int32_t j = 0; j < n_if; ++j) {
    for (int m = 0; m < p->if_nsub[j]; ++m) {
      const int32_t i = m == 0 ? p->if_sub0[j] : m == 1 ? p->if_sub1[j] : p->if_subx[2 * j + m - 2];
      if (m < 2)
        (m == 0 ? p->if_slot0 : p->if_slot1)[j] = cur[i];
      else
        p->if_slotx[2 * j + m - 2] = cur[i];
      for (int k = 0; k < p->if_dim[j]; ++k) {
        const int32_t g = cur[i] + k;
        p->slot_sub[g] = i;
        p->slot_loc[g] = g - p->sub_slot[i];
        p->slot_if[g] = j;
        p->slot_mk[g] = m * 8 + k;
      }
      cur[i] += p->if_dim[j];
    }
  }
  // scenes
  p->sc_sub.assign(p->n_scene + 1, 0);
  p->sc_if.assign(p->n_scene + 1, 0);
  for (int32_t i = 0; i < n_sub; ++i) p->sc_sub[p->sub_scene[i] + 1] = i + 1;
  for (int32_t s = 0; s < p->n_scene; ++s) p->sc_sub[s + 1] = std::max(p->sc_sub[s + 1], p->sc_sub[s]);
  for (int32_t j = 0; j < n_if; ++j) p->sc_if[p->sub_scene[p->if_sub0[j]] + 1] = j + 1;
  for (int32_t s = 0; s < p->n_scene; ++s) p->sc_if[s + 1] = std::max(p->sc_if[s + 1], p->sc_if[s]);
  p->sc_slot.assign(p->n_scene + 1, 0);
  p->sc_dof.assign(p->n_scene + 1, 0);
  for (int32_t s = 0; s <= p->n_scene; ++s) {
    p->sc_slot[s] = p->sub_slot[p->sc_sub[s]];
    p->sc_dof[s] = p->sub_dof[p->sc_sub[s]];
  }
  // blocked H and padded w inside each scene's LDS area (vectors of 16 bytes)
  {
    const int32_t V = (int32_t)(16 / p->rsize());
    p->sub_hq.assign(n_sub, 0);
    p->sub_wq.assign(n_sub, 0);
    p->sc_hq.assign(p->n_scene, 0);
    p->sc_wq.assign(p->n_scene, 0);
    for (int32_t s = 0; s < p->n_scene; ++s) {
      int64_t hq = 0, wq = 0;
      for (int32_t i = p->sc_sub[s]; i < p->sc_sub[s + 1]; ++i) {
        const int64_t nq = (nc[i] + V - 1) / V;
        p->sub_hq[i] = (int32_t)hq;
        p->sub_wq[i] = (int32_t)wq;
        hq += nq * nc[i];
        wq += nq * V;
      }
      if (hq > INT32_MAX / 4 || wq > INT32_MAX / 4) return bad("scene too large");
      p->sc_hq[s] = (int32_t)hq;
      p->sc_wq[s] = (int32_t)wq;
      p->max_hq_scene = std::max<int32_t>(p->max_hq_scene, (int32_t)hq);
      p->max_wq_scene = std::max<int32_t>(p->max_wq_scene, (int32_t)wq);
    }
  }
  // team kernel: each interface's member slot rows on consecutive lanes of one wave
  {
    std::vector<std::vector<int32_t>> lanes(p->n_scene);
    size_t most = 0;
    for (int32_t s = 0; s < p->n_scene; ++s) {
      auto& L = lanes[s];
      for (int32_t j = p->sc_if[s]; j < p->sc_if[s + 1]; ++j) {
        const int32_t size = p->if_nsub[j] * p->if_dim[j];
        if ((L.size() % 64) + size > 64) L.resize((L.size() + 63) / 64 * 64, -1);
        for (int32_t q = 0; q < size; ++q) L.push_back((j << 4) | q);
      }
      most = std::max(most, L.size());
    }
    const size_t block = std::max<size_t>(64, (most + 63) / 64 * 64);
    const size_t lds = 16 * (size_t)p->max_hq_scene + p->rsize() * 2 * (size_t)p->max_wq_scene + 64;
    if (p->max_members <= 2 && block <= 512 && lds <= 150 * 1024 && n_if < (1 << 26)) {
      p->team_block = (int32_t)block;
      p->lane_code.assign((size_t)p->n_scene * block, -1);
      for (int32_t s = 0; s < p->n_scene; ++s)
        std::copy(lanes[s].begin(), lanes[s].end(), p->lane_code.begin() + (size_t)s * block);
    }
  }
  for (int32_t s = 0; s < p->n_scene; ++s) {
    p->max_slot_scene = std::max(p->max_slot_scene, p->sc_slot[s + 1] - p->sc_slot[s]);
    p->max_row_scene = std::max(p->max_row_scene, p->if_row[p->sc_if[s + 1]] - p->if_row[p->sc_if[s]]);
    p->max_sub_scene = std::max(p->max_sub_scene, p->sc_sub[s + 1] - p->sc_sub[s]);
    p->max_if_scene = std::max(p->max_if_scene, p->sc_if[s + 1] - p->sc_if[s]);
    p->max_h_scene = std::max<int64_t>(p->max_h_scene, p->sub_H[p->sc_sub[s + 1]] - p->sub_H[p->sc_sub[s]]);
  }
  // LDS limits of the small-block path (subadmm_solve, rigid model); a problem beyond
  // them can still run the FEM path
  const size_t R = p->rsize();
  auto small_no = [&](const std::string& why) {
    if (p->small_ok) p->small_why = why;
    p->small_ok = false;
  };
  // subsystems whose factorisation arrays (FP64 size) exceed the LDS are factorised with
  // them in device memory
  if (p->max_n > kMaxFactorDof) small_no("a subsystem has more than 512 DOF");
  p->big_off.assign(n_sub, -1);
  p->big_bytes = 0;
  p->n_big = 0;
  for (int32_t i = 0; i < n_sub && p->small_ok; ++i) {
    const size_t fb = factor_bytes(p->sub_n[i], nc[i], sizeof(double));
    if (fb > 150 * 1024) {
      p->big_off[i] = (int64_t)p->big_bytes;
      p->big_bytes += (fb + 255) & ~size_t(255);
      ++p->n_big;
    }
  }
  p->sub_ok = p->small_ok;
  p->sub_why = p->small_why;
  if (p->max_slot_scene > 512 || p->max_if_scene > 512) small_no("a scene has more than 512 slot rows or interfaces");
  if (R * (3 * (size_t)p->max_slot_scene + (size_t)p->max_row_scene) > 150 * 1024)
    small_no("a scene's slot vectors do not fit in LDS");
  if (p->sub_ok) plan_factor(p);
  if (p->small_ok) {
    // interface map of the thread-per-interface kernel: the block size its launcher
    // chooses, and per scene one interface class (kind, dim) per wave when they fit
    const int32_t ns_max = std::max<int32_t>(p->max_slot_scene, 1);
    const bool two = 2 * ns_max <= kTwoLaneMax && p->max_if_scene <= kTwoLaneMax;
    const int32_t need = two ? std::max(2 * ns_max, p->max_if_scene) : std::max(ns_max, p->max_if_scene);
    const int32_t block = (need + 63) / 64 * 64;
    // per scene one interface class (kind, dim) per wave when they fit in `block` lanes
    auto append_zmap = [&](int32_t block) {
      const size_t z0 = p->zmap.size();
      p->zmap.resize(z0 + (size_t)p->n_scene * block, -1);
      int32_t* zm = p->zmap.data() + z0;
      const int32_t waves = block / 64;
      for (int32_t s = 0; s < p->n_scene; ++s) {
        // first with one thread per row of the interfaces whose rows are independent (their
        // z-update is a few loads and stores per row), then one thread per interface
        bool fits = false;
        for (int per_row = n_if < (1 << kZRowShift) ? 1 : 0; per_row >= 0 && !fits; --per_row) {
          std::vector<std::pair<int64_t, int32_t>> cls;
          for (int32_t j = p->sc_if[s]; j < p->sc_if[s + 1]; ++j) {
            const int32_t kd = p->if_kind[j];
            const bool rows = per_row && p->if_dim[j] > 1 && p->if_nsub[j] <= 2 &&
                              (kd == SUBADMM_IF_EQUALITY || kd == SUBADMM_IF_HARD_INEQ || kd == SUBADMM_IF_SOFT);
            if (rows) {
              for (int32_t r = 0; r < p->if_dim[j]; ++r) cls.push_back({(int64_t)kd * 16 + 1, j | ((r + 1) << kZRowShift)});
            } else {
              cls.push_back({(int64_t)kd * 16 + p->if_dim[j], j});
            }
          }
          std::stable_sort(cls.begin(), cls.end(),
                           [](const std::pair<int64_t, int32_t>& x, const std::pair<int64_t, int32_t>& y) {
                             return x.first < y.first;
                           });
          std::fill(zm + (size_t)s * block, zm + (size_t)(s + 1) * block, -1);
          int32_t wave = 0, lane = 0;
          fits = true;
          for (size_t q = 0; q < cls.size() && fits; ++q) {
            if (q > 0 && cls[q].first != cls[q - 1].first && lane > 0) {
              ++wave;
              lane = 0;
            }
            if (lane == 64) {
              ++wave;
              lane = 0;
            }
            if (wave >= waves) fits = false;
            else zm[(size_t)s * block + wave * 64 + lane++] = cls[q].second;
          }
        }
        if (!fits) {  // contiguous: thread t takes the scene's t-th interface
          for (int32_t t = 0; t < block; ++t) {
            const int32_t j = p->sc_if[s] + t;
            zm[(size_t)s * block + t] = j < p->sc_if[s + 1] ? j : -1;
          }
        }
      }
      return z0;
    };
    p->zmap.clear();
    p->rmap.clear();
    p->rmap_block = 0;
    p->rmap_in.clear();
    if (block <= 512) {
      p->zmap_block = block;
      append_zmap(block);
      // split rows within this block: per scene, the subsystems with the longest rows first
      // take 2, then 4 lanes per row (more than 2, then 8 vectors of H per row) while the
      // scene's lanes, each split row aligned to its lane count, still fit the block
      {
        const int32_t V = 16 / (int32_t)R;
        p->rmap_in.assign((size_t)p->n_scene * block, -1);
        bool any = false;
        for (int32_t s = 0; s < p->n_scene; ++s) {
          const int32_t sb = p->sc_sub[s], se = p->sc_sub[s + 1];
          std::vector<int32_t> kp(se - sb, 1), order(se - sb);
          for (int32_t q = 0; q < se - sb; ++q) order[q] = q;
          auto nq = [&](int32_t q) { return (nc[sb + q] + V - 1) / V; };
          std::stable_sort(order.begin(), order.end(), [&](int32_t x, int32_t y) { return nq(x) > nq(y); });
          auto lanes = [&]() {
            size_t L = 0;
            for (int32_t q = 0; q < se - sb; ++q) {
              L = (L + kp[q] - 1) / kp[q] * kp[q];
              L += (size_t)nc[sb + q] * kp[q];
            }
            return L;
          };
          for (int32_t target : {2, 4}) {
            for (int32_t q : order) {
              if (nq(q) <= (target == 2 ? 2 : 8) || kp[q] >= target) continue;
              const int32_t old = kp[q];
              kp[q] = target;
              if (lanes() > (size_t)block) kp[q] = old;
            }
          }
          std::vector<int32_t> L;
          for (int32_t q = 0; q < se - sb; ++q) {
            const int32_t i = sb + q;
            any |= kp[q] > 1;
            while (L.size() % kp[q]) L.push_back(-1);
            for (int32_t r = 0; r < nc[i]; ++r) {
              const int32_t row = p->sub_slot[i] + r - p->sc_slot[s];
              for (int32_t part = 0; part < kp[q]; ++part) L.push_back((row << 5) | (kp[q] << 2) | part);
            }
          }
          std::copy(L.begin(), L.end(), p->rmap_in.begin() + (size_t)s * block);
        }
        if (!any) p->rmap_in.clear();
      }
      // split rows: the slot rows of a subsystem with more than t1 (t2) vectors of H per
      // row take 2 (4) consecutive lanes each, aligned to that count; thresholds doubled
      // once if a scene's lanes do not fit 512
      const int32_t V = 16 / (int32_t)R;
      for (int32_t t1 = 4; t1 <= 8 && p->rmap_block == 0; t1 *= 2) {
        const int32_t t2 = 2 * t1;
        std::vector<std::vector<int32_t>> rl(p->n_scene);
        size_t most = 0;
        bool any_split = false;
        for (int32_t s = 0; s < p->n_scene; ++s) {
          auto& L = rl[s];
          for (int32_t i = p->sc_sub[s]; i < p->sc_sub[s + 1]; ++i) {
            const int32_t nq = (nc[i] + V - 1) / V;
            const int32_t kp = nq <= t1 ? 1 : nq <= t2 ? 2 : 4;
            any_split |= kp > 1;
            while (L.size() % kp) L.push_back(-1);
            for (int32_t q = 0; q < nc[i]; ++q) {
              const int32_t r = p->sub_slot[i] + q - p->sc_slot[s];
              for (int32_t part = 0; part < kp; ++part) L.push_back((r << 5) | (kp << 2) | part);
            }
          }
          most = std::max(most, L.size());
        }
        most = std::max(most, (size_t)p->max_if_scene);
        const size_t rblock = std::max<size_t>(64, (most + 63) / 64 * 64);
        if (!any_split || rblock > 512) continue;
        p->rmap_block = (int32_t)rblock;
        p->rmap.assign((size_t)p->n_scene * rblock, -1);
        for (int32_t s = 0; s < p->n_scene; ++s)
          std::copy(rl[s].begin(), rl[s].end(), p->rmap.begin() + (size_t)s * rblock);
        p->zmap_split = append_zmap((int32_t)rblock);
      }
    }
  } else {
    p->team_block = 0;
    p->lane_code.clear();
  }
  // learned warm start classes: contacts (dim 3, one member) and dim-5 equalities
  p->if_class.assign(n_if, -1);
  p->if_krow.assign(n_if, -1);
  p->if_scene.assign(n_if, 0);
  for (int32_t j = 0; j < n_if; ++j) {
    p->if_scene[j] = p->sub_scene[p->if_sub0[j]];
    int c = -1;
    if (p->if_kind[j] == SUBADMM_IF_CONTACT && p->if_nsub[j] == 1) c = 0;
    else if (p->if_kind[j] == SUBADMM_IF_EQUALITY && p->if_dim[j] == 5 && p->if_nsub[j] <= 2) c = 1;
    if (c >= 0) {
      p->if_class[j] = c;
      p->if_krow[j] = p->n_class[c]++;
    }
  }
  plan_workspace(p);
  *out = p;
  return SUBADMM_OK;
}

namespace {
int set_option(subadmm_problem* p, int32_t option, int64_t value) {
  switch (option) {
    case SUBADMM_OPT_FACTOR_FP64:
      if (value != 0 && value != 1) return fail(p, SUBADMM_E_ARG, "FACTOR_FP64 takes 0 or 1");
      p->factor_fp64 = (int32_t)value;
      plan_factor(p);
      // the factorisation order is a device table: a bound problem gets the new one now,
      // and the kept host staging of the tables is refreshed on its next use
      p->upload_keep.clear();
      if (p->bound) {
        hipError_t e = hipMemcpyAsync(p->ws + p->o.fac_order, p->fac_order.data(), sizeof(int32_t) * p->n_sub,
                                      hipMemcpyHostToDevice, p->stream);
        if (e == hipSuccess) e = hipStreamSynchronize(p->stream);
        if (e != hipSuccess) return dev_err(p, e, "factorisation order upload");
      }
      return SUBADMM_OK;
    case SUBADMM_OPT_TEAM_KERNEL:
      if (value < 0 || value > 2) return fail(p, SUBADMM_E_ARG, "TEAM_KERNEL takes 0, 1 or 2");
      if (value != 0 && p->max_members > 2)
        return fail(p, SUBADMM_E_ARG, "the team and wave forms take interfaces of one or two members");
      if (value == 2) {
        const size_t lds = 16 * (size_t)p->max_hq_scene +
                           p->rsize() * ((size_t)p->max_wq_scene + 2 * (size_t)std::max<int32_t>(p->max_slot_scene, 1)) + 64;
        if (!p->small_ok || p->max_slot_scene > 256 || p->max_if_scene > 64 || lds > 150 * 1024)
          return fail(p, SUBADMM_E_ARG, "the wave form needs scenes of at most 256 slot rows and 64 interfaces "
                                        "whose operators fit in LDS");
      }
      p->use_team = (int32_t)value;
      return SUBADMM_OK;
    case SUBADMM_OPT_FACTOR_STREAMS:
      if (value != 0 && value != 1) return fail(p, SUBADMM_E_ARG, "FACTOR_STREAMS takes 0 or 1");
      p->factor_streams = (int32_t)value;
      return SUBADMM_OK;
    case SUBADMM_OPT_FEM_RESIDENT:
      if (value != 0 && value != 1) return fail(p, SUBADMM_E_ARG, "FEM_RESIDENT takes 0 or 1");
      p->fem_resident = (int32_t)value;
      return SUBADMM_OK;
    case SUBADMM_OPT_IMPULSE_OUTPUT:
      if (value != 0 && value != 1) return fail(p, SUBADMM_E_ARG, "IMPULSE_OUTPUT takes 0 or 1");
      p->impulse = (int32_t)value;
      return SUBADMM_OK;
    case SUBADMM_OPT_FEM_KAPPA_MAX:
      if (value < 0 || value > ((int64_t)1 << 52)) return fail(p, SUBADMM_E_ARG, "FEM_KAPPA_MAX out of range");
      p->fem_kappa_max = value;
      return SUBADMM_OK;
    case SUBADMM_OPT_SPLIT_ROWS:
      if (value < 0 || value > 2) return fail(p, SUBADMM_E_ARG, "SPLIT_ROWS takes 0, 1 or 2");
      p->split_rows = (int32_t)value;
      return SUBADMM_OK;
    case SUBADMM_OPT_CONTACT_MODEL:
      if (value != 0 && value != 1) return fail(p, SUBADMM_E_ARG, "CONTACT_MODEL takes 0 or 1");
      p->contact_model = (int32_t)value;
      return SUBADMM_OK;
    case SUBADMM_OPT_LARGE_PATH:
      if (value < 0 || value > 2) return fail(p, SUBADMM_E_ARG, "LARGE_PATH takes 0, 1 or 2");
      p->force_large = (int32_t)value;
      return SUBADMM_OK;
    case SUBADMM_OPT_BOYD_RESIDUALS:
      if (value != 0 && value != 1) return fail(p, SUBADMM_E_ARG, "BOYD_RESIDUALS takes 0 or 1");
      p->boyd = (int32_t)value;
      return SUBADMM_OK;
    case SUBADMM_OPT_LEARNED_BUDGET:
      if (value < 0 || value > (1 << 30)) return fail(p, SUBADMM_E_ARG, "LEARNED_BUDGET out of range");
      p->learned_budget = (int32_t)value;
      return SUBADMM_OK;
    default:
      return fail(p, SUBADMM_E_ARG, "unknown option");
  }
}
}  // namespace

SUBADMM_API int subadmm_set_option(subadmm_problem* p, int32_t option, int64_t value) {
  if (!p) return fail(nullptr, SUBADMM_E_ARG, "null problem");
  const int rc = set_option(p, option, value);
  if (rc == SUBADMM_OK) ++p->cfg_gen;
  return rc;
}

SUBADMM_API int subadmm_get_sizes(const subadmm_problem* p, subadmm_sizes* out) {
  if (!p || !out) return SUBADMM_E_ARG;
  out->n_dof = p->n_dof;
  out->n_slot = p->n_slot;
  out->n_rows = p->n_rows;
  out->n_A = p->n_A;
  out->n_J = p->n_J;
  out->n_sub = p->n_sub;
  out->n_if = p->n_if;
  out->n_scene = p->n_scene;
  out->max_dof = p->max_n;
  out->max_slot_sub = p->max_nc;
  out->max_slot_scene = p->max_slot_scene;
  return SUBADMM_OK;
}

SUBADMM_API int subadmm_rigid_set_links(subadmm_problem* p, int32_t nl, const int32_t* link_type,
                                        const int32_t* link_body, const double* link_anchor, const double* link_frame,
                                        const int32_t* link_if, const int32_t* link_dim, const double* link_k,
                                        const double* link_alpha) {
  if (!p) return fail(nullptr, SUBADMM_E_ARG, "null problem");
  if (p->has_rigid || p->has_fem || p->bound) return fail(p, SUBADMM_E_STATE, "links come before the model");
  if (nl < 0 || (nl > 0 && (!link_type || !link_body || !link_anchor || !link_frame || !link_if)))
    return fail(p, SUBADMM_E_ARG, "bad link arrays");
  std::vector<int32_t> dims(nl);
  std::vector<double> ks(nl, 0.0), als(nl, 0.0);
  for (int32_t q = 0; q < nl; ++q) {
    const int32_t j = link_if[q];
    if (link_type[q] < 0 || link_type[q] > 2) return fail(p, SUBADMM_E_ARG, "link type must be 0, 1 or 2");
    if (j < 0 && link_type[q] == 2) return fail(p, SUBADMM_E_ARG, "a sphere contact link needs its interface");
    if (j < 0) {
      // a soft link folded into its subsystem's dynamics
      if (!link_dim || !link_k || !link_alpha) return fail(p, SUBADMM_E_ARG, "folded links need dim, k and alpha");
      if (link_dim[q] < 1 || link_dim[q] > 3) return fail(p, SUBADMM_E_ARG, "links have 1 to 3 rows");
      if (!(link_k[q] >= 0.0) || !std::isfinite(link_k[q]) || !(link_alpha[q] > 0.0) || !std::isfinite(link_alpha[q]))
        return fail(p, SUBADMM_E_ARG, "a folded soft link needs k >= 0 and alpha > 0");
      dims[q] = link_dim[q];
      ks[q] = link_k[q];
      als[q] = link_alpha[q];
    } else {
      if (j >= p->n_if) return fail(p, SUBADMM_E_ARG, "link interface out of range");
      const int32_t kind = p->if_kind[j], dim = p->if_dim[j];
      if (dim < 1 || dim > 3) return fail(p, SUBADMM_E_ARG, "link interfaces have 1 to 3 rows");
      if (kind == SUBADMM_IF_CONTACT && (dim != 3 || link_type[q] == 1))
        return fail(p, SUBADMM_E_ARG, "a contact link has three linear rows (normal, two tangents)");
      if (link_type[q] == 2 && kind != SUBADMM_IF_CONTACT)
        return fail(p, SUBADMM_E_ARG, "a sphere link is a contact interface");
      dims[q] = dim;
    }
    for (int c = 0; c < 6; ++c)
      if (!std::isfinite(link_anchor[6 * q + c])) return fail(p, SUBADMM_E_ARG, "non-finite link anchor");
    for (int c = 0; c < 9; ++c)
      if (!std::isfinite(link_frame[9 * q + c])) return fail(p, SUBADMM_E_ARG, "non-finite link frame");
  }
  p->nl = nl;
  p->link_type.assign(link_type, link_type + nl);
  p->link_body.assign(link_body, link_body + 2 * (size_t)nl);
  p->link_if.assign(link_if, link_if + nl);
  p->link_anchor.assign(link_anchor, link_anchor + 6 * (size_t)nl);
  p->link_frame.assign(link_frame, link_frame + 9 * (size_t)nl);
  p->link_dim = dims;
  p->link_k = ks;
  p->link_alpha = als;
  return SUBADMM_OK;
}

SUBADMM_API int subadmm_rigid_set_model(subadmm_problem* p, int32_t nb, const int32_t* body_sub,
                                        const int32_t* body_local, const double* mass, const double* inertia,
                                        int32_t nj, const int32_t* joint_body, const double* joint_anchor,
                                        const double* joint_frame_a, const double* joint_axis_b,
                                        const int32_t* joint_if, int32_t ncon, const int32_t* contact_body,
                                        const double* contact_point, const int32_t* contact_if, double gravity,
                                        double baumgarte) {
  if (!p) return fail(nullptr, SUBADMM_E_ARG, "null problem");
  if (nb < 1 || nj < 0 || ncon < 0 || !body_sub || !body_local || !mass || !inertia)
    return fail(p, SUBADMM_E_ARG, "bad body arrays");
  if ((nj > 0 && (!joint_body || !joint_anchor || !joint_frame_a || !joint_axis_b || !joint_if)) ||
      (ncon > 0 && (!contact_body || !contact_point || !contact_if)))
    return fail(p, SUBADMM_E_ARG, "bad joint/contact arrays");
  if (!std::isfinite(gravity) || !std::isfinite(baumgarte)) return fail(p, SUBADMM_E_ARG, "bad constants");
  if (p->bound) return fail(p, SUBADMM_E_STATE, "the model must be set before bind");
  if (p->has_fem) return fail(p, SUBADMM_E_STATE, "problem already has a FEM model");
  if (p->max_n > kMaxDof) return fail(p, SUBADMM_E_ARG, "rigid subsystems have at most 64 DOF");
  std::vector<int32_t> src(p->n_if, INT32_MIN);
  std::vector<int32_t> used(p->n_dof, 0);
  for (int32_t k = 0; k < nb; ++k) {
    const int32_t i = body_sub[k];
    if (i < 0 || i >= p->n_sub) return fail(p, SUBADMM_E_ARG, "body subsystem out of range");
    const int32_t c0 = 6 * body_local[k];
    if (body_local[k] < 0 || c0 + 6 > p->sub_n[i]) return fail(p, SUBADMM_E_ARG, "body block outside its subsystem");
    for (int c = 0; c < 6; ++c)
      if (used[p->sub_dof[i] + c0 + c]++) return fail(p, SUBADMM_E_ARG, "two bodies share a DOF block");
    if (!(mass[k] > 0.0) || !(inertia[3 * k] > 0.0) || !(inertia[3 * k + 1] > 0.0) || !(inertia[3 * k + 2] > 0.0))
      return fail(p, SUBADMM_E_ARG, "mass and inertia must be positive");
  }
  for (int64_t d = 0; d < p->n_dof; ++d)
    if (!used[d]) return fail(p, SUBADMM_E_ARG, "a subsystem DOF belongs to no body");
  for (int32_t q = 0; q < nj; ++q) {
    const int32_t j = joint_if[q], a = joint_body[2 * q], b = joint_body[2 * q + 1];
    if (j < 0 || j >= p->n_if || src[j] != INT32_MIN) return fail(p, SUBADMM_E_ARG, "bad joint interface index");
    if (a < 0 || a >= nb || b < 0 || b >= nb || a == b) return fail(p, SUBADMM_E_ARG, "bad joint bodies");
    if (p->if_kind[j] != SUBADMM_IF_EQUALITY || p->if_dim[j] != 5)
      return fail(p, SUBADMM_E_ARG, "joint interface must be an equality of dim 5");
    const bool same = body_sub[a] == body_sub[b];
    if (same ? (p->if_nsub[j] != 1 || p->if_sub0[j] != body_sub[a])
             : (p->if_nsub[j] != 2 || p->if_sub0[j] != body_sub[a] || p->if_sub1[j] != body_sub[b]))
      return fail(p, SUBADMM_E_ARG, "joint interface members do not match the bodies' subsystems");
    src[j] = q;
  }
  for (int32_t q = 0; q < ncon; ++q) {
    const int32_t j = contact_if[q], k = contact_body[q];
    if (j < 0 || j >= p->n_if || src[j] != INT32_MIN) return fail(p, SUBADMM_E_ARG, "bad contact interface index");
    if (k < 0 || k >= nb) return fail(p, SUBADMM_E_ARG, "bad contact body");
    if (p->if_kind[j] != SUBADMM_IF_CONTACT || p->if_nsub[j] != 1 || p->if_sub0[j] != body_sub[k])
      return fail(p, SUBADMM_E_ARG, "contact interface must be a one-member contact on the body's subsystem");
    src[j] = -1 - q;
  }
  std::vector<int32_t> ilink_off(p->n_sub + 1, 0), ilink;
  for (int32_t q = 0; q < p->nl; ++q) {
    const int32_t j = p->link_if[q], a = p->link_body[2 * q], b = p->link_body[2 * q + 1];
    if (a < 0 || a >= nb || b < -1 || b >= nb || a == b) return fail(p, SUBADMM_E_ARG, "bad link bodies");
    if (j < 0) {
      if (b < 0 || body_sub[a] != body_sub[b])
        return fail(p, SUBADMM_E_ARG, "a folded soft link joins two bodies of one subsystem");
      ilink_off[body_sub[a] + 1]++;
      continue;
    }
    if (src[j] != INT32_MIN) return fail(p, SUBADMM_E_ARG, "interface of a link used twice");
    const bool same = b < 0 || body_sub[a] == body_sub[b];
    if (same ? (p->if_nsub[j] != 1 || p->if_sub0[j] != body_sub[a])
             : (p->if_nsub[j] != 2 || p->if_sub0[j] != body_sub[a] || p->if_sub1[j] != body_sub[b]))
      return fail(p, SUBADMM_E_ARG, "link interface members do not match the bodies' subsystems");
    if (p->if_kind[j] == SUBADMM_IF_CONTACT && b < 0 && p->link_type[q] != 2)
      return fail(p, SUBADMM_E_ARG, "a contact link needs two bodies (ground contacts are contacts)");
    src[j] = nj + q;
  }
  for (int32_t j = 0; j < p->n_if; ++j) {
    if (src[j] == INT32_MIN) return fail(p, SUBADMM_E_ARG, "interface without a joint, link or contact");
    if (p->if_kind[j] == SUBADMM_IF_SOFT && !(src[j] >= nj))
      return fail(p, SUBADMM_E_ARG, "soft interfaces of the rigid model come from links");
  }
  p->has_rigid = true;
  p->nb = nb;
  p->nj = nj;
  p->ncon = ncon;
  p->body_sub.assign(body_sub, body_sub + nb);
  p->body_local.assign(body_local, body_local + nb);
  p->mass.assign(mass, mass + nb);
  p->inertia.assign(inertia, inertia + 3 * (size_t)nb);
  p->joint_body.assign(joint_body, joint_body + 2 * (size_t)nj);
  p->joint_anchor.assign(joint_anchor, joint_anchor + 6 * (size_t)nj);
  p->joint_frame.assign(joint_frame_a, joint_frame_a + 9 * (size_t)nj);
  p->joint_axis_b.assign(joint_axis_b, joint_axis_b + 3 * (size_t)nj);
  p->contact_body.assign(contact_body, contact_body + ncon);
  p->contact_point.assign(contact_point, contact_point + 3 * (size_t)ncon);
  p->if_src = src;
  for (int32_t i = 0; i < p->n_sub; ++i) ilink_off[i + 1] += ilink_off[i];
  ilink.assign(ilink_off[p->n_sub], 0);
  {
    std::vector<int32_t> put(ilink_off.begin(), ilink_off.end() - 1);
    for (int32_t q = 0; q < p->nl; ++q)
      if (p->link_if[q] < 0) ilink[put[body_sub[p->link_body[2 * q]]]++] = q;
  }
  p->sub_ilink_off = ilink_off;
  p->sub_ilink = ilink;
  p->sub_body_off.assign(p->n_sub + 1, 0);
  for (int32_t k = 0; k < nb; ++k) p->sub_body_off[body_sub[k] + 1]++;
  for (int32_t i = 0; i < p->n_sub; ++i) p->sub_body_off[i + 1] += p->sub_body_off[i];
  p->sub_body.assign(nb, 0);
  std::vector<int32_t> fill(p->n_sub, 0);
  for (int32_t k = 0; k < nb; ++k) p->sub_body[p->sub_body_off[body_sub[k]] + fill[body_sub[k]]++] = k;
  p->gravity = gravity;
  p->baumgarte = baumgarte;
  p->bound = false;  // layout changed: bind again
  plan_workspace(p);
  return SUBADMM_OK;
}

SUBADMM_API size_t subadmm_workspace_bytes(const subadmm_problem* p) { return p ? p->o.total : 0; }

namespace {

// Stages every table into one host buffer laid out like the workspace prefix
// (p->upload_keep, static_end bytes).
template <typename T>
void stage_tables_t(subadmm_problem* p) {
  auto& o = p->o;
  std::vector<char>& h = p->upload_keep;
  h.assign(o.static_end, 0);
  auto put = [&](size_t off, const void* src, size_t bytes) {
    if (bytes) std::memcpy(h.data() + off, src, bytes);
  };
  auto puti = [&](size_t off, const std::vector<int32_t>& v) { put(off, v.data(), v.size() * sizeof(int32_t)); };
  auto putl = [&](size_t off, const std::vector<int64_t>& v) { put(off, v.data(), v.size() * sizeof(int64_t)); };
  auto putr = [&](size_t off, const std::vector<double>& v) {
    std::vector<T> tmp(v.begin(), v.end());
    put(off, tmp.data(), tmp.size() * sizeof(T));
  };
  puti(o.sub_n, p->sub_n);
  puti(o.sub_nc, p->sub_nc);
  puti(o.sub_dof, p->sub_dof);
  puti(o.sub_slot, p->sub_slot);
  putl(o.sub_A, p->sub_A);
  putl(o.sub_J, p->sub_J);
  putl(o.sub_H, p->sub_H);
  puti(o.slot_sub, p->slot_sub);
  puti(o.slot_loc, p->slot_loc);
  puti(o.slot_if, p->slot_if);
  puti(o.slot_mk, p->slot_mk);
  puti(o.if_kind, p->if_kind);
  puti(o.if_dim, p->if_dim);
  puti(o.if_nsub, p->if_nsub);
  puti(o.if_sub0, p->if_sub0);
  puti(o.if_sub1, p->if_sub1);
  puti(o.if_slot0, p->if_slot0);
  puti(o.if_subx, p->if_subx);
  puti(o.if_slotx, p->if_slotx);
  puti(o.if_slot1, p->if_slot1);
  puti(o.if_row, p->if_row);
  puti(o.sc_sub, p->sc_sub);
  puti(o.sc_slot, p->sc_slot);
  puti(o.sc_if, p->sc_if);
  puti(o.sc_dof, p->sc_dof);
  puti(o.sub_hq, p->sub_hq);
  puti(o.sub_wq, p->sub_wq);
  puti(o.sc_hq, p->sc_hq);
  puti(o.sc_wq, p->sc_wq);
  puti(o.lane_code, p->lane_code);
  puti(o.zmap, p->zmap);
  puti(o.rmap, p->rmap);
  puti(o.rmap_in, p->rmap_in);
  puti(o.if_class, p->if_class);
  puti(o.if_krow, p->if_krow);
  puti(o.if_scene, p->if_scene);
  puti(o.fac_order, p->fac_order);
  putl(o.big_off, p->big_off);
  putl(o.sc_fscr, p->sc_fscr);
  puti(o.sc_order, p->sc_order);
  puti(o.sub_scene, p->sub_scene);
  putr(o.mu, p->if_mu);
  putr(o.ksoft, p->if_k);
  putr(o.asoft, p->if_alpha);
  if (p->has_rigid) {
    puti(o.r_body_sub, p->body_sub);
    puti(o.r_body_local, p->body_local);
    putr(o.r_mass, p->mass);
    putr(o.r_inertia, p->inertia);
    puti(o.r_sub_body, p->sub_body);
    puti(o.r_sub_body_off, p->sub_body_off);
    puti(o.r_if_src, p->if_src);
    puti(o.r_joint_body, p->joint_body);
    putr(o.r_joint_anchor, p->joint_anchor);
    putr(o.r_joint_frame, p->joint_frame);
    putr(o.r_joint_axis_b, p->joint_axis_b);
    puti(o.r_contact_body, p->contact_body);
    putr(o.r_contact_point, p->contact_point);
    puti(o.r_link_type, p->link_type);
    puti(o.r_link_body, p->link_body);
    putr(o.r_link_anchor, p->link_anchor);
    putr(o.r_link_frame, p->link_frame);
    puti(o.r_link_dim, p->link_dim);
    putr(o.r_link_k, p->link_k);
    putr(o.r_link_alpha, p->link_alpha);
    puti(o.r_sub_ilink_off, p->sub_ilink_off);
    puti(o.r_sub_ilink, p->sub_ilink);
  }
  if (p->has_fem) {
    puti(o.f_node_off, p->f_node_off);
    puti(o.f_tet_off, p->f_tet_off);
    puti(o.f_tet_node, p->f_tet_node);
    puti(o.f_pair_off, p->f_pair_off);
    puti(o.f_pair_ab, p->f_pair_ab);
    puti(o.f_pent_off, p->f_pent_off);
    puti(o.f_pent, p->f_pent);
    puti(o.f_node_diag, p->f_node_diag);
    puti(o.f_m, p->f_m);
    puti(o.f_dkey_off, p->f_dkey_off);
    puti(o.f_perm, p->f_perm);
    puti(o.f_jtj, p->f_jtj);
    puti(o.f_slot_dk, p->f_slot_dk);
    puti(o.f_slot_dof, p->f_slot_dof);
    puti(o.f_dk_off, p->f_dk_off);
    puti(o.f_dk_slot, p->f_dk_slot);
    puti(o.f_if_node0, p->f_if_node0);
    puti(o.f_if_node1, p->f_if_node1);
    put(o.f_slot_sgn, p->f_slot_sgn.data(), p->f_slot_sgn.size() * sizeof(float));
    auto putd = [&](size_t off, const std::vector<double>& v) { put(off, v.data(), v.size() * sizeof(double)); };
    putd(o.f_tet_g, p->f_tet_g);
    putd(o.f_tet_vol, p->f_tet_vol);
    putd(o.f_rest, p->f_rest);
    putd(o.f_mass, p->f_mass);
    putd(o.f_lame_l, p->f_lame_l);
    putd(o.f_lame_m, p->f_lame_m);
    putl(o.f_sq_off, p->f_sq_off);
  }
}

int stage_tables(subadmm_problem* p) {
  if (p->dtype == SUBADMM_F64) stage_tables_t<double>(p);
  else stage_tables_t<float>(p);
  return SUBADMM_OK;
}

int upload_all(subadmm_problem* p) {
  auto& o = p->o;
  stage_tables(p);
  // the tables in one copy; warm buffers, statistics and flags start at zero.  The staging
  // buffer is kept for later uploads of the same tables (subadmm_solve_scratch).
  hipError_t e = hipMemcpyAsync(p->ws, p->upload_keep.data(), o.static_end, hipMemcpyHostToDevice, p->stream);
  if (e == hipSuccess && o.total > o.static_end)
    e = hipMemsetAsync(p->ws + o.static_end, 0, o.total - o.static_end, p->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(p->stream);
  return dev_err(p, e, "bind upload");
}

}  // namespace

namespace {
void release_graph(subadmm_problem* p) {
  if (p->graph_exec) (void)hipGraphExecDestroy(p->graph_exec);
  if (p->graph) (void)hipGraphDestroy(p->graph);
  p->graph_exec = nullptr;
  p->graph = nullptr;
}

void release_cap_stream(subadmm_problem* p) {
  if (p->cap_stream) (void)hipStreamDestroy(p->cap_stream);
  p->cap_stream = nullptr;
}

void release_side(subadmm_problem* p) {
  if (!p->side.empty() || !p->side_ev.empty() || p->fork_ev) (void)hipDeviceSynchronize();
  for (auto s : p->side) (void)hipStreamDestroy(s);
  for (auto e : p->side_ev) (void)hipEventDestroy(e);
  if (p->fork_ev) (void)hipEventDestroy(p->fork_ev);
  p->side.clear();
  p->side_ev.clear();
  p->fork_ev = nullptr;
}
}  // namespace

SUBADMM_API int subadmm_bind(subadmm_problem* p, void* dev_workspace, size_t bytes, void* hip_stream) {
  if (!p) return fail(nullptr, SUBADMM_E_ARG, "null problem");
  if (!dev_workspace) return fail(p, SUBADMM_E_ARG, "null workspace");
  if ((reinterpret_cast<uintptr_t>(dev_workspace) & 255) != 0) return fail(p, SUBADMM_E_ARG, "workspace must be 256-byte aligned");
  if (bytes < p->o.total) return fail(p, SUBADMM_E_WORKSPACE, "workspace too small");
  p->ws = static_cast<char*>(dev_workspace);
  p->ws_bytes = bytes;
  p->stream = static_cast<hipStream_t>(hip_stream);
  int rc = upload_all(p);
  p->bound = rc == SUBADMM_OK;
  if (rc) return rc;
  release_graph(p);
  release_side(p);
  if (p->sub_ok && p->buckets.size() > 1) {
    const size_t ns = std::min<size_t>(p->buckets.size() - 1, 3);
    hipError_t e = hipEventCreateWithFlags(&p->fork_ev, hipEventDisableTiming);
    for (size_t k = 0; k < ns && e == hipSuccess; ++k) {
      hipStream_t st = nullptr;
      e = hipStreamCreateWithFlags(&st, hipStreamNonBlocking);
      if (e == hipSuccess) p->side.push_back(st);
    }
    for (size_t k = 0; k + 1 < p->buckets.size() && e == hipSuccess; ++k) {
      hipEvent_t ev = nullptr;
      e = hipEventCreateWithFlags(&ev, hipEventDisableTiming);
      if (e == hipSuccess) p->side_ev.push_back(ev);
    }
    if (e != hipSuccess) {
      release_side(p);
      (void)hipGetLastError();  // fall back to one stream
    }
  }
  return SUBADMM_OK;
}

SUBADMM_API int subadmm_solve(subadmm_problem* p, const void* A, const void* b, const void* J, const void* e,
                              int32_t max_iters, double tol, int32_t warm, const void* z0, const void* u0,
                              void* v_hat, void* lambda, void* z_out, void* u_out) {
  int rc = check_solve_args(p, max_iters, tol, warm, z0, u0);
  if (rc) return rc;
  if (!A || !b || (p->n_J > 0 && !J) || (p->n_rows > 0 && !e)) return fail(p, SUBADMM_E_ARG, "null input array");
  if (!p->sub_ok) return fail(p, SUBADMM_E_ARG, "problem exceeds the per-subsystem solver: " + p->sub_why);
  if (p->dtype == SUBADMM_F64)
    rc = run_solve<double>(p, (const double*)A, (const double*)b, (const double*)J, (const double*)e, max_iters, tol,
                           warm, (const double*)z0, (const double*)u0, (double*)v_hat, (double*)lambda);
  else
    rc = run_solve<float>(p, (const float*)A, (const float*)b, (const float*)J, (const float*)e, max_iters, tol,
                          warm, (const float*)z0, (const float*)u0, (float*)v_hat, (float*)lambda);
  if (rc) return rc;
  const size_t R = p->rsize();
  if (z_out) rc = dev_err(p, hipMemcpyAsync(z_out, p->ws + p->o.zw, R * p->n_slot, hipMemcpyDeviceToDevice, p->stream), "copy z");
  if (!rc && u_out) rc = dev_err(p, hipMemcpyAsync(u_out, p->ws + p->o.uw, R * p->n_slot, hipMemcpyDeviceToDevice, p->stream), "copy u");
  return rc;
}

// ------------------------------------------------------------------------------------
// Solve without a caller workspace (subadmm_solve_scratch): the problem's tables and
// per-step arrays are placed in a file-scope device array instead of the bound
// workspace.  The array's host-side name is not a device address; every use goes
// through the per-device address obtained with hipGetSymbolAddress.
// ------------------------------------------------------------------------------------
namespace {

constexpr size_t kScratchBytes = SUBADMM_SCRATCH_BYTES;
constexpr int kScratchDevices = 64;
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

int read_stats_now(subadmm_problem* p, subadmm_stats* host_out);

std::mutex g_scratch_mu;
char* g_scratch_ptr[kScratchDevices] = {};

// Device address of this device's copy of the scratch array (looked up once per device,
// with that device current).
int scratch_address(subadmm_problem* p, char** out) {
  int dev = -1;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return dev_err(p, e, "scratch: current device");
  if (dev < 0 || dev >= kScratchDevices) return fail(p, SUBADMM_E_DEVICE, "scratch: device index out of range");
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* ptr = nullptr;
    e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !ptr) return dev_err(p, e != hipSuccess ? e : hipErrorInvalidSymbol, "scratch: symbol address");
    g_scratch_ptr[dev] = static_cast<char*>(ptr);
  }
  *out = g_scratch_ptr[dev];
  return SUBADMM_OK;
}

// Zero fill of [p, p + n16 * 16): a kernel, so that callers capturing the stream record no
// memset node.
__global__ void scratch_zero_kernel(uint4* p, size_t n16) {
  const uint4 z = make_uint4(0u, 0u, 0u, 0u);
  for (size_t k = (size_t)blockIdx.x * blockDim.x + threadIdx.x; k < n16; k += (size_t)gridDim.x * blockDim.x)
    p[k] = z;
}

}  // namespace

SUBADMM_API int subadmm_solve_scratch(subadmm_problem* p, void* hip_stream, const void* A, const void* b,
                                      const void* J, const void* e, int32_t max_iters, double tol, int32_t warm,
                                      const void* z0, const void* u0, void* v_hat, void* lambda, void* z_out,
                                      void* u_out, subadmm_stats* stats_out) {
  if (!p) return fail(nullptr, SUBADMM_E_ARG, "null problem");
  if (max_iters < 1) return fail(p, SUBADMM_E_ARG, "max_iters must be >= 1");
  if (!(tol >= 0.0) || !std::isfinite(tol)) return fail(p, SUBADMM_E_ARG, "tol must be finite and >= 0");
  if (warm != SUBADMM_WARM_COLD && warm != SUBADMM_WARM_GIVEN)
    return fail(p, SUBADMM_E_ARG, "the scratch solve starts cold or from given z0, u0 only");
  if (warm == SUBADMM_WARM_GIVEN && (!z0 || !u0)) return fail(p, SUBADMM_E_ARG, "warm GIVEN needs z0 and u0");
  if (!A || !b || (p->n_J > 0 && !J) || (p->n_rows > 0 && !e)) return fail(p, SUBADMM_E_ARG, "null input array");
  if (!p->sub_ok) return fail(p, SUBADMM_E_ARG, "problem exceeds the per-subsystem solver: " + p->sub_why);
  if (p->o.total > kScratchBytes)
    return fail(p, SUBADMM_E_WORKSPACE, "problem needs " + std::to_string(p->o.total) +
                                            " bytes of scratch; the static scratch holds " +
                                            std::to_string(kScratchBytes));
  if (p->capturing || p->timing) return fail(p, SUBADMM_E_STATE, "scratch solve during capture or timing");
  char* ptr = nullptr;
  int rc = scratch_address(p, &ptr);
  if (rc) return rc;
  // the problem's own binding is kept and restored around the call
  char* const ws0 = p->ws;
  const size_t bytes0 = p->ws_bytes;
  const hipStream_t stream0 = p->stream;
  const bool bound0 = p->bound;
  const int32_t streams0 = p->factor_streams;
  p->ws = ptr;
  p->ws_bytes = kScratchBytes;
  p->stream = static_cast<hipStream_t>(hip_stream);
  p->bound = true;
  p->in_scratch = true;
  p->factor_streams = 0;  // factorisation classes one after another on the caller's stream
  // tables from the host staging kept in the problem (a copy from pageable host memory
  // returns once the source has been read); everything after them starts at zero
  if (p->upload_keep.size() != p->o.static_end) rc = stage_tables(p);
  hipError_t he = hipSuccess;
  if (!rc) he = hipMemcpyAsync(ptr, p->upload_keep.data(), p->o.static_end, hipMemcpyHostToDevice, p->stream);
  if (!rc && he == hipSuccess && p->o.total > p->o.static_end) {
    const size_t n16 = (p->o.total - p->o.static_end) / 16;  // both offsets are 256-byte aligned
    const unsigned blocks = (unsigned)std::min<size_t>((n16 + 255) / 256, 4096);
    hipLaunchKernelGGL(scratch_zero_kernel, dim3(blocks), dim3(256), 0, p->stream,
                       reinterpret_cast<uint4*>(ptr + p->o.static_end), n16);
    he = hipGetLastError();
  }
  if (!rc) rc = dev_err(p, he, "scratch upload");
  if (!rc) {
    if (p->dtype == SUBADMM_F64)
      rc = run_solve<double>(p, (const double*)A, (const double*)b, (const double*)J, (const double*)e, max_iters, tol,
                             warm, (const double*)z0, (const double*)u0, (double*)v_hat, (double*)lambda);
    else
      rc = run_solve<float>(p, (const float*)A, (const float*)b, (const float*)J, (const float*)e, max_iters, tol,
                            warm, (const float*)z0, (const float*)u0, (float*)v_hat, (float*)lambda);
  }
  const size_t R = p->rsize();
  if (!rc && z_out)
    rc = dev_err(p, hipMemcpyAsync(z_out, ptr + p->o.zw, R * p->n_slot, hipMemcpyDeviceToDevice, p->stream), "copy z");
  if (!rc && u_out)
    rc = dev_err(p, hipMemcpyAsync(u_out, ptr + p->o.uw, R * p->n_slot, hipMemcpyDeviceToDevice, p->stream), "copy u");
  if (!rc && stats_out) rc = read_stats_now(p, stats_out);
  p->ws = ws0;
  p->ws_bytes = bytes0;
  p->stream = stream0;
  p->bound = bound0;
  p->factor_streams = streams0;
  p->in_scratch = false;
  return rc;
}

namespace {

template <typename T>
int run_rigid_assemble(subadmm_problem* p, const T* pos, const T* rot, const T* vel, const T* omega, double dt,
                       T* A, T* b, T* J, T* e) {
  const Topo t = make_topo(p);
  const RigidModel<T> m = make_rigid<T>(p);
  return dev_err(p, timed(p, SUBADMM_K_ASSEMBLE, [&] {
                   // scenes of up to 32 subsystems: one workgroup constructs a whole scene
                   const bool per_scene = p->small_ok && p->max_sub_scene <= 32;
                   return launch_rigid_assemble<T>(t, m, pos, rot, vel, omega, (T)dt, A, b, J, e, per_scene,
                                                   p->stream);
                 }),
                 "rigid assemble kernel");
}

template <typename T>
WarmArgs<T> make_warm(subadmm_problem* p, const T* z_prev, const T* u_prev) {
  auto& o = p->o;
  WarmArgs<T> w;
  w.t = make_topo(p);
  w.if_class = at<int32_t>(p, o.if_class);
  w.if_krow = at<int32_t>(p, o.if_krow);
  w.beta = at<T>(p, o.beta);
  w.e = at<T>(p, o.se);
  w.J = at<T>(p, o.sJ);
  w.v_dof = at<T>(p, o.vdof);
  w.mu = at<T>(p, o.mu);
  w.z_prev = z_prev;
  w.u_prev = u_prev;
  w.xc = at<float>(p, o.xc);
  w.xj = at<float>(p, o.xj);
  w.yc = nullptr;
  w.yj = nullptr;
  w.z0 = at<T>(p, o.zl);
  w.u0 = at<T>(p, o.ul);
  w.if_scene = at<int32_t>(p, o.if_scene);
  w.conv = at<int32_t>(p, o.st_cv);
  w.z_fin = at<T>(p, o.zw);
  w.u_fin = at<T>(p, o.uw);
  w.tc = p->rec_tc;
  w.tj = p->rec_tj;
  w.wc = p->rec_wc;
  w.wj = p->rec_wj;
  return w;
}

// Features of every learned-class interface for the current step (after construction
// and factorisation), from the previous step's (z, u); copied out when recording.
template <typename T>
int run_features(subadmm_problem* p, const T* vel, const T* omega, WarmArgs<T>& w) {
  const Topo t = make_topo(p);
  const RigidModel<T> m = make_rigid<T>(p);
  int rc = dev_err(p, launch_dof_velocity<T>(t, m, vel, omega, at<T>(p, p->o.vdof), p->stream), "dof velocity");
  if (!rc) rc = dev_err(p, launch_features<T>(w, p->stream), "features");
  if (rc) return rc;
  if (p->rec_xc && p->n_class[0])
    rc = dev_err(p, hipMemcpyAsync(p->rec_xc, w.xc, sizeof(float) * kContactIn * p->n_class[0], hipMemcpyDeviceToDevice,
                                   p->stream), "record contact features");
  if (!rc && p->rec_xj && p->n_class[1])
    rc = dev_err(p, hipMemcpyAsync(p->rec_xj, w.xj, sizeof(float) * kJointIn * p->n_class[1], hipMemcpyDeviceToDevice,
                                   p->stream), "record joint features");
  return rc;
}

// lambda -> t lambda, the impulse over the step (option SUBADMM_OPT_IMPULSE_OUTPUT).
template <typename T>
__global__ void impulse_kernel(T* lambda, long n, T dt) {
  const long k = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (k < n) lambda[k] *= dt;
}

template <typename T>
int impulse_out(subadmm_problem* p, T* lambda, double dt) {
  if (!p->impulse || !lambda || p->n_rows == 0) return SUBADMM_OK;
  hipLaunchKernelGGL(impulse_kernel<T>, dim3((unsigned)((p->n_rows + 255) / 256)), dim3(256), 0, p->stream, lambda,
                     (long)p->n_rows, (T)dt);
  return dev_err(p, hipGetLastError(), "impulse output");
}

template <typename T>
int run_rigid_step(subadmm_problem* p, T* pos, T* rot, T* vel, T* omega, double dt, int32_t max_iters, double tol,
                   int32_t warm, T* v_hat, T* lambda) {
  auto& o = p->o;
  p->boyd_valid = false;
  T* A = at<T>(p, o.sA);
  T* b = at<T>(p, o.sb);
  T* J = at<T>(p, o.sJ);
  T* e = at<T>(p, o.se);
  T* vh = at<T>(p, o.svh);
  int rc = run_rigid_assemble<T>(p, pos, rot, vel, omega, dt, A, b, J, e);
  if (!rc) rc = run_factor<T>(p, A, b, J);
  if (rc) return rc;
  T* zw = at<T>(p, o.zw);
  T* uw = at<T>(p, o.uw);
  T* zp = at<T>(p, o.zp);
  T* up = at<T>(p, o.up);
  const bool learned = warm == SUBADMM_WARM_LEARNED;
  const bool rec = p->recording();
  WarmArgs<T> w = make_warm<T>(p, zp, up);
  const int span = (learned || rec) ? timing_begin_span(p) : -1;
  if (learned || rec) {
    // keep the previous step's (z, u) for the features, the fallback and the targets
    rc = dev_err(p, hipMemcpyAsync(zp, zw, sizeof(T) * p->n_slot, hipMemcpyDeviceToDevice, p->stream), "keep z");
    if (!rc) rc = dev_err(p, hipMemcpyAsync(up, uw, sizeof(T) * p->n_slot, hipMemcpyDeviceToDevice, p->stream), "keep u");
    if (!rc) rc = run_features<T>(p, vel, omega, w);
    if (rc) return rc;
  }
  if (learned) {
    if (p->net[0] && p->n_class[0]) {
      rc = mlp_infer_on(p->net[0], p->stream, p->n_class[0], w.xc, at<float>(p, o.yc));
      if (rc) return fail(p, rc, std::string("contact network: ") + subadmm_mlp_last_error(p->net[0]));
      w.yc = at<float>(p, o.yc);
    }
    if (p->net[1] && p->n_class[1]) {
      rc = mlp_infer_on(p->net[1], p->stream, p->n_class[1], w.xj, at<float>(p, o.yj));
      if (rc) return fail(p, rc, std::string("joint network: ") + subadmm_mlp_last_error(p->net[1]));
      w.yj = at<float>(p, o.yj);
    }
    rc = dev_err(p, launch_warm_apply<T>(w, p->stream), "warm apply");
    timing_end_span(p, span, SUBADMM_K_WARM);
    const int32_t budget = p->learned_budget > 0 && p->learned_budget < max_iters ? p->learned_budget : max_iters;
    if (!rc) rc = run_loop<T>(p, e, budget, tol, w.z0, w.u0, vh, lambda, nullptr, nullptr);
    // plain ADMM from the previous step's values wherever the learned start did not reach tol
    if (!rc)
      rc = run_loop<T>(p, e, max_iters, tol, zp, up, vh, lambda, at<int32_t>(p, o.st_cv), at<long long>(p, o.st_fb));
  } else {
    timing_end_span(p, span, SUBADMM_K_WARM);  // recording only: the features
    const bool prev = warm == SUBADMM_WARM_PREV;
    rc = run_loop<T>(p, e, max_iters, tol, prev ? zw : nullptr, prev ? uw : nullptr, vh, lambda, nullptr, nullptr);
  }
  if (!rc && (p->rec_tc || p->rec_tj || p->rec_wc || p->rec_wj))
    rc = dev_err(p, launch_targets<T>(w, p->stream), "targets");
  if (!rc) rc = run_boyd<T>(p, e);
  if (rc) return rc;
  RigidState<T> st{pos, rot, vel, omega};
  const Topo t = make_topo(p);
  const RigidModel<T> m = make_rigid<T>(p);
  rc = dev_err(p, timed(p, SUBADMM_K_ADVANCE, [&] { return launch_rigid_advance<T>(t, m, st, vh, (T)dt, p->stream); }),
               "rigid advance kernel");
  if (!rc) rc = impulse_out<T>(p, lambda, dt);
  if (rc) return rc;
  if (v_hat) rc = dev_err(p, hipMemcpyAsync(v_hat, vh, sizeof(T) * p->n_dof, hipMemcpyDeviceToDevice, p->stream), "copy v_hat");
  return rc;
}

}  // namespace

SUBADMM_API int subadmm_rigid_assemble(subadmm_problem* p, const void* pos, const void* rot, const void* vel,
                                       const void* omega, double dt, void* A, void* b, void* J, void* e) {
  if (!p) return fail(nullptr, SUBADMM_E_ARG, "null problem");
  if (!p->has_rigid) return fail(p, SUBADMM_E_STATE, "no rigid model set");
  if (!p->bound) return fail(p, SUBADMM_E_WORKSPACE, "problem has no bound workspace");
  if (!(dt > 0.0) || !std::isfinite(dt)) return fail(p, SUBADMM_E_ARG, "dt must be positive");
  if (!pos || !rot || !vel || !omega || !A || !b || (p->n_J > 0 && !J) || (p->n_rows > 0 && !e))
    return fail(p, SUBADMM_E_ARG, "null array");
  if (p->dtype == SUBADMM_F64)
    return run_rigid_assemble<double>(p, (const double*)pos, (const double*)rot, (const double*)vel,
                                      (const double*)omega, dt, (double*)A, (double*)b, (double*)J, (double*)e);
  return run_rigid_assemble<float>(p, (const float*)pos, (const float*)rot, (const float*)vel, (const float*)omega, dt,
                                   (float*)A, (float*)b, (float*)J, (float*)e);
}

SUBADMM_API int subadmm_rigid_step(subadmm_problem* p, void* pos, void* rot, void* vel, void* omega, double dt,
                                   int32_t max_iters, double tol, int32_t warm, void* v_hat, void* lambda) {
  int rc = check_solve_args(p, max_iters, tol, warm == SUBADMM_WARM_LEARNED ? SUBADMM_WARM_PREV
                                               : warm == SUBADMM_WARM_GIVEN ? -1 : warm,
                            nullptr, nullptr);
  if (rc) return rc;
  if (!p->has_rigid) return fail(p, SUBADMM_E_STATE, "no rigid model set");
  if (!(dt > 0.0) || !std::isfinite(dt)) return fail(p, SUBADMM_E_ARG, "dt must be positive");
  if (!pos || !rot || !vel || !omega) return fail(p, SUBADMM_E_ARG, "null state array");
  if (!p->sub_ok) return fail(p, SUBADMM_E_ARG, "problem exceeds the per-subsystem solver: " + p->sub_why);
  if (warm == SUBADMM_WARM_LEARNED && (!p->small_ok || p->force_large))
    return fail(p, SUBADMM_E_ARG, "the learned start needs scenes that fit the per-scene kernel");
  if (p->dtype == SUBADMM_F64)
    return run_rigid_step<double>(p, (double*)pos, (double*)rot, (double*)vel, (double*)omega, dt, max_iters, tol,
                                  warm, (double*)v_hat, (double*)lambda);
  return run_rigid_step<float>(p, (float*)pos, (float*)rot, (float*)vel, (float*)omega, dt, max_iters, tol, warm,
                               (float*)v_hat, (float*)lambda);
}


namespace {

template <typename T>
int run_rigid_steps(subadmm_problem* p, T* pos, T* rot, T* vel, T* omega, double dt, int32_t n_steps,
                    int32_t max_iters, double tol, int32_t warm, T* v_hat, T* lambda) {
  auto& o = p->o;
  p->boyd_valid = false;
  // the thread-per-row form, its rows split within the default block when that option is
  // set (SPLIT_ROWS = 2), else unsplit; the interface map is the one built for that block
  Topo t = make_topo(p);
  t.rmap = nullptr;
  t.rmap_block = 0;
  if (p->split_rows == 2 && !p->rmap_in.empty()) {
    t.rmap = at<int32_t>(p, o.rmap_in);
    t.rmap_block = p->zmap_block;
  }
  t.zmap = p->zmap.empty() ? nullptr : at<int32_t>(p, o.zmap);
  t.zmap_block = p->zmap_block;
  StepsArgs<T> a;
  a.A = at<T>(p, o.sA);
  a.b = at<T>(p, o.sb);
  a.J = at<T>(p, o.sJ);
  a.e = at<T>(p, o.se);
  FactorArgs<T>& f = a.f;
  f.t = t;
  f.A = a.A;
  f.b = a.b;
  f.J = a.J;
  f.rho = p->rho;
  f.beta = at<T>(p, o.beta);
  f.H = at<T>(p, o.H);
  f.d = at<T>(p, o.d);
  f.G = at<T>(p, o.G);
  f.cvec = at<T>(p, o.cvec);
  f.flags = at<int32_t>(p, o.flags);
  f.order = nullptr;
  f.first = 0;
  LoopArgs<T>& la = a.l;
  la.t = t;
  la.beta = f.beta;
  la.H = f.H;
  la.d = f.d;
  la.G = f.G;
  la.cvec = f.cvec;
  la.e = a.e;
  la.mu = at<T>(p, o.mu);
  la.ksoft = at<T>(p, o.ksoft);
  la.asoft = at<T>(p, o.asoft);
  const bool prev = warm == SUBADMM_WARM_PREV;
  la.z_in = prev ? at<T>(p, o.zw) : nullptr;
  la.u_in = prev ? at<T>(p, o.uw) : nullptr;
  la.z_out = at<T>(p, o.zw);
  la.u_out = at<T>(p, o.uw);
  la.v_hat = at<T>(p, o.svh);
  la.lambda = lambda;
  la.st_iters = at<int32_t>(p, o.st_it);
  la.st_total = at<long long>(p, o.st_tot);
  la.st_unconv = at<long long>(p, o.st_unc);
  la.st_conv = at<int32_t>(p, o.st_cv);
  la.st_theta = at<double>(p, o.st_th);
  la.st_rtheta = at<double>(p, o.st_rt);
  la.flags = f.flags;
  la.max_iters = max_iters;
  la.tol = tol;
  la.contact_model = p->contact_model;
  la.skip_converged = nullptr;
  la.st_fallback = nullptr;
  a.m = make_rigid<T>(p);
  a.st = RigidState<T>{pos, rot, vel, omega};
  a.dt = (T)dt;
  a.n_steps = n_steps;
  a.lds_factor = (int32_t)p->steps_lds;
  a.fscr = at<double>(p, o.sfscr);
  a.sc_fscr = at<int64_t>(p, o.sc_fscr);
  a.sc_order = at<int32_t>(p, o.sc_order);
  // the kernel reads its arguments from the workspace (a copy from pageable host memory
  // returns once the source has been read)
  auto* dev_args = at<StepsArgs<T>>(p, o.steps_args);
  int rc = dev_err(p, hipMemcpyAsync(dev_args, &a, sizeof(a), hipMemcpyHostToDevice, p->stream), "steps arguments");
  if (rc) return rc;
  rc = dev_err(p, timed(p, SUBADMM_K_STEPS, [&] {
                 return launch_steps<T>(a, dev_args, p->max_slot_scene, p->max_if_scene, p->max_hq_scene,
                                        p->max_wq_scene, p->factor_fp64 != 0, p->steps_lds, p->stream);
               }),
               "multi-step kernel");
  if (!rc) rc = run_boyd<T>(p, a.e);
  if (!rc) rc = impulse_out<T>(p, lambda, dt);
  if (rc) return rc;
  if (v_hat)
    rc = dev_err(p, hipMemcpyAsync(v_hat, la.v_hat, sizeof(T) * p->n_dof, hipMemcpyDeviceToDevice, p->stream),
                 "copy v_hat");
  return rc;
}

}  // namespace

SUBADMM_API int subadmm_set_scene_order(subadmm_problem* p, const int32_t* order) {
  if (!p) return fail(nullptr, SUBADMM_E_ARG, "null problem");
  std::vector<int32_t> ord(p->n_scene);
  if (order) {
    std::vector<char> seen(p->n_scene, 0);
    for (int32_t k = 0; k < p->n_scene; ++k) {
      const int32_t s = order[k];
      if (s < 0 || s >= p->n_scene || seen[s]) return fail(p, SUBADMM_E_ARG, "order is not a permutation of the scenes");
      seen[s] = 1;
      ord[k] = s;
    }
  } else {
    for (int32_t k = 0; k < p->n_scene; ++k) ord[k] = k;
  }
  p->sc_order.swap(ord);
  if (!p->upload_keep.empty()) std::memcpy(p->upload_keep.data() + p->o.sc_order, p->sc_order.data(),
                                           sizeof(int32_t) * p->n_scene);
  if (p->bound) {
    hipError_t e = hipMemcpyAsync(p->ws + p->o.sc_order, p->sc_order.data(), sizeof(int32_t) * p->n_scene,
                                  hipMemcpyHostToDevice, p->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(p->stream);
    if (e != hipSuccess) return dev_err(p, e, "scene order upload");
  }
  ++p->cfg_gen;
  return SUBADMM_OK;
}

SUBADMM_API int subadmm_rigid_steps(subadmm_problem* p, void* pos, void* rot, void* vel, void* omega, double dt,
                                    int32_t n_steps, int32_t max_iters, double tol, int32_t warm, void* v_hat,
                                    void* lambda) {
  int rc = check_solve_args(p, max_iters, tol, warm, nullptr, nullptr);
  if (rc) return rc;
  if (warm != SUBADMM_WARM_COLD && warm != SUBADMM_WARM_PREV)
    return fail(p, SUBADMM_E_ARG, "the multi-step call starts every step cold or from the previous step's values");
  if (n_steps < 1) return fail(p, SUBADMM_E_ARG, "n_steps must be >= 1");
  if (!p->has_rigid) return fail(p, SUBADMM_E_STATE, "no rigid model set");
  if (!(dt > 0.0) || !std::isfinite(dt)) return fail(p, SUBADMM_E_ARG, "dt must be positive");
  if (!pos || !rot || !vel || !omega) return fail(p, SUBADMM_E_ARG, "null state array");
  if (!p->small_ok) return fail(p, SUBADMM_E_ARG, "problem exceeds the per-scene solver: " + p->small_why);
  if (p->dtype == SUBADMM_F64)
    return run_rigid_steps<double>(p, (double*)pos, (double*)rot, (double*)vel, (double*)omega, dt, n_steps, max_iters,
                                   tol, warm, (double*)v_hat, (double*)lambda);
  return run_rigid_steps<float>(p, (float*)pos, (float*)rot, (float*)vel, (float*)omega, dt, n_steps, max_iters, tol,
                                warm, (float*)v_hat, (float*)lambda);
}

// ------------------------------------------------------------------------------------
// FEM blocks
// ------------------------------------------------------------------------------------
SUBADMM_API int subadmm_fem_set_model(subadmm_problem* p, int32_t n_nodes, const double* rest, int32_t n_tets,
                                      const int32_t* tets, const double* young, const double* poisson,
                                      double density, const int32_t* if_node, double gravity, double baumgarte) {
  if (!p) return fail(nullptr, SUBADMM_E_ARG, "null problem");
  if (p->bound) return fail(p, SUBADMM_E_STATE, "the model must be set before bind");
  if (p->has_rigid) return fail(p, SUBADMM_E_STATE, "problem already has a rigid model");
  for (int32_t j = 0; j < p->n_if; ++j)
    if (p->if_kind[j] == SUBADMM_IF_SOFT) return fail(p, SUBADMM_E_ARG, "soft interfaces need an assembled problem");
  if (n_nodes < 1 || !rest || n_tets < 1 || !tets || !young || !poisson || (p->n_if > 0 && !if_node))
    return fail(p, SUBADMM_E_ARG, "bad FEM arrays");
  if (!(density > 0.0) || !std::isfinite(density) || !std::isfinite(gravity) || !std::isfinite(baumgarte))
    return fail(p, SUBADMM_E_ARG, "bad constants");
  const int32_t ns = p->n_sub;
  std::vector<int32_t> node_off(ns + 1, 0);
  for (int32_t i = 0; i < ns; ++i) {
    if (p->sub_n[i] % 3 != 0) return fail(p, SUBADMM_E_ARG, "FEM subsystems have 3 DOF per node");
    node_off[i + 1] = node_off[i] + p->sub_n[i] / 3;
  }
  if (node_off[ns] != n_nodes) return fail(p, SUBADMM_E_ARG, "node count does not match the subsystems' DOF");
  if (p->max_nc > 512) return fail(p, SUBADMM_E_ARG, "a FEM block has more than 512 slot rows");
  if (p->n_scene > 256) return fail(p, SUBADMM_E_ARG, "the FEM path takes at most 256 scenes");
  std::vector<int32_t> node_sub(n_nodes);
  for (int32_t i = 0; i < ns; ++i)
    for (int32_t k = node_off[i]; k < node_off[i + 1]; ++k) node_sub[k] = i;
  for (int32_t i = 0; i < ns; ++i) {
    if (!(young[i] > 0.0) || !std::isfinite(young[i]) || !(poisson[i] >= 0.0) || !(poisson[i] < 0.5))
      return fail(p, SUBADMM_E_ARG, "Young's modulus must be positive and Poisson's ratio in [0, 0.5)");
  }
  // tetrahedra grouped by subsystem (stable)
  std::vector<int32_t> tsub(n_tets);
  for (int32_t e = 0; e < n_tets; ++e) {
    for (int a = 0; a < 4; ++a)
      if (tets[4 * e + a] < 0 || tets[4 * e + a] >= n_nodes) return fail(p, SUBADMM_E_ARG, "tetrahedron node out of range");
    tsub[e] = node_sub[tets[4 * e]];
    for (int a = 1; a < 4; ++a)
      if (node_sub[tets[4 * e + a]] != tsub[e]) return fail(p, SUBADMM_E_ARG, "a tetrahedron spans two subsystems");
  }
  std::vector<int32_t> order(n_tets);
  for (int32_t e = 0; e < n_tets; ++e) order[e] = e;
  std::stable_sort(order.begin(), order.end(), [&](int32_t a, int32_t b) { return tsub[a] < tsub[b]; });
  p->f_tet_off.assign(ns + 1, 0);
  for (int32_t e = 0; e < n_tets; ++e) p->f_tet_off[tsub[e] + 1]++;
  for (int32_t i = 0; i < ns; ++i) p->f_tet_off[i + 1] += p->f_tet_off[i];
  p->f_tet_node.resize(4 * (size_t)n_tets);
  p->f_tet_g.resize(12 * (size_t)n_tets);
  p->f_tet_vol.resize(n_tets);
  p->f_mass.assign(n_nodes, 0.0);
  for (int32_t k = 0; k < n_tets; ++k) {
    const int32_t e = order[k];
    const int32_t* v = tets + 4 * (size_t)e;
    double Dm[9];
    for (int r = 0; r < 3; ++r)
      for (int a = 1; a < 4; ++a) Dm[r * 3 + a - 1] = rest[3 * (size_t)v[a] + r] - rest[3 * (size_t)v[0] + r];
    const double det = Dm[0] * (Dm[4] * Dm[8] - Dm[5] * Dm[7]) - Dm[1] * (Dm[3] * Dm[8] - Dm[5] * Dm[6]) +
                       Dm[2] * (Dm[3] * Dm[7] - Dm[4] * Dm[6]);
    if (!(det > 0.0) || !std::isfinite(det))
      return fail(p, SUBADMM_E_ARG, "tetrahedron " + std::to_string(e) + " has non-positive rest volume");
    double inv[9];
    inv[0] = (Dm[4] * Dm[8] - Dm[5] * Dm[7]) / det;
    inv[1] = (Dm[2] * Dm[7] - Dm[1] * Dm[8]) / det;
    inv[2] = (Dm[1] * Dm[5] - Dm[2] * Dm[4]) / det;
    inv[3] = (Dm[5] * Dm[6] - Dm[3] * Dm[8]) / det;
    inv[4] = (Dm[0] * Dm[8] - Dm[2] * Dm[6]) / det;
    inv[5] = (Dm[2] * Dm[3] - Dm[0] * Dm[5]) / det;
    inv[6] = (Dm[3] * Dm[7] - Dm[4] * Dm[6]) / det;
    inv[7] = (Dm[1] * Dm[6] - Dm[0] * Dm[7]) / det;
    inv[8] = (Dm[0] * Dm[4] - Dm[1] * Dm[3]) / det;
    double* g = p->f_tet_g.data() + 12 * (size_t)k;
    for (int a = 1; a < 4; ++a)
      for (int c = 0; c < 3; ++c) g[3 * a + c] = inv[(a - 1) * 3 + c];
    for (int c = 0; c < 3; ++c) g[c] = -(g[3 + c] + g[6 + c] + g[9 + c]);
    const double V = det / 6.0;
    p->f_tet_vol[k] = V;
    for (int a = 0; a < 4; ++a) {
      p->f_tet_node[4 * (size_t)k + a] = v[a];
      p->f_mass[v[a]] += density * V / 4.0;
    }
  }
  for (int32_t k = 0; k < n_nodes; ++k)
    if (!(p->f_mass[k] > 0.0)) return fail(p, SUBADMM_E_ARG, "node " + std::to_string(k) + " belongs to no tetrahedron");
  // node pairs per subsystem: for each (a, b) the tetrahedra holding both (gather form of A)
  p->f_pair_off.assign(ns + 1, 0);
  p->f_pair_ab.clear();
  p->f_pent_off.assign(1, 0);
  p->f_pent.clear();
  p->f_node_diag.assign(n_nodes, -1);
  for (int32_t i = 0; i < ns; ++i) {
    std::vector<std::pair<int64_t, int32_t>> ent;
    for (int32_t k = p->f_tet_off[i]; k < p->f_tet_off[i + 1]; ++k) {
      const int32_t lt = k - p->f_tet_off[i];
      for (int a = 0; a < 4; ++a)
        for (int b = 0; b < 4; ++b) {
          const int64_t na = p->f_tet_node[4 * (size_t)k + a] - node_off[i];
          const int64_t nb = p->f_tet_node[4 * (size_t)k + b] - node_off[i];
          ent.push_back({(na << 16) | nb, (lt << 4) | (a << 2) | b});
        }
    }
    std::stable_sort(ent.begin(), ent.end(),
                     [](const std::pair<int64_t, int32_t>& x, const std::pair<int64_t, int32_t>& y) { return x.first < y.first; });
    for (size_t q = 0; q < ent.size(); ++q) {
      if (q == 0 || ent[q].first != ent[q - 1].first) {
        if (q > 0) p->f_pent_off.push_back((int32_t)p->f_pent.size());
        const int32_t na = (int32_t)(ent[q].first >> 16), nb = (int32_t)(ent[q].first & 0xffff);
        if (na == nb) p->f_node_diag[node_off[i] + na] = (int32_t)p->f_pair_ab.size();
        p->f_pair_ab.push_back(na | (nb << 16));
      }
      p->f_pent.push_back(ent[q].second);
    }
    if (!ent.empty()) p->f_pent_off.push_back((int32_t)p->f_pent.size());
    p->f_pair_off[i + 1] = (int32_t)p->f_pair_ab.size();
  }
  // interfaces: nodal equality (dim 3, two members) or ground contact (dim 3, one member)
  p->f_if_node0.assign(p->n_if, 0);
  p->f_if_node1.assign(p->n_if, 0);
  for (int32_t j = 0; j < p->n_if; ++j) {
    const bool eq = p->if_kind[j] == SUBADMM_IF_EQUALITY && p->if_nsub[j] == 2;
    const bool ct = p->if_kind[j] == SUBADMM_IF_CONTACT && p->if_nsub[j] == 1;
    if (p->if_dim[j] != 3 || !(eq || ct))
      return fail(p, SUBADMM_E_ARG, "FEM interfaces are nodal equalities (dim 3, two members) or contacts");
    for (int m = 0; m < p->if_nsub[j]; ++m) {
      const int32_t nd = if_node[2 * j + m];
      const int32_t i = m == 0 ? p->if_sub0[j] : p->if_sub1[j];
      if (nd < 0 || nd >= n_nodes || node_sub[nd] != i)
        return fail(p, SUBADMM_E_ARG, "interface node outside its member subsystem");
      (m == 0 ? p->f_if_node0 : p->f_if_node1)[j] = nd;
    }
    if (ct) p->f_if_node1[j] = p->f_if_node0[j];
  }
  // slot selection, constrained DOFs and the permutation (constrained DOFs last)
  p->f_slot_dof.assign(p->n_slot, 0);
  p->f_slot_sgn.assign(p->n_slot, 1.0f);
  p->f_slot_dk.assign(p->n_slot, 0);
  p->f_jtj.assign(p->n_dof, 0);
  for (int32_t g = 0; g < p->n_slot; ++g) {
    const int32_t i = p->slot_sub[g], j = p->slot_if[g], mk = p->slot_mk[g];
    const int m = mk >> 3, k = mk & 7;
    const int32_t nd = (m == 0 ? p->f_if_node0 : p->f_if_node1)[j] - node_off[i];
    int32_t dof;
    if (p->if_kind[j] == SUBADMM_IF_CONTACT) dof = 3 * nd + (k == 0 ? 2 : k - 1);  // rows (e_z, e_x, e_y)
    else dof = 3 * nd + k;
    p->f_slot_dof[g] = dof;
    p->f_slot_sgn[g] = (p->if_kind[j] == SUBADMM_IF_EQUALITY && m == 1) ? -1.0f : 1.0f;
    p->f_jtj[p->sub_dof[i] + dof] += 1;
  }
  p->f_m.assign(ns, 0);
  p->f_dkey_off.assign(ns + 1, 0);
  p->f_perm.assign(p->n_dof, 0);
  p->f_sq_off.assign(ns + 1, 0);
  p->f_dk_off.assign(1, 0);
  p->f_dk_slot.clear();
  p->f_max_m = 0;
  p->f_max_ng = 0;
  for (int32_t i = 0; i < ns; ++i) {
    const int32_t n = p->sub_n[i], d0 = p->sub_dof[i];
    std::vector<int32_t> key(n, -1);
    int32_t m = 0;
    for (int32_t r = 0; r < n; ++r)
      if (p->f_jtj[d0 + r] > 0) key[r] = m++;
    int32_t pos = 0;
    for (int32_t r = 0; r < n; ++r)
      if (key[r] < 0) p->f_perm[d0 + pos++] = r;
    for (int32_t r = 0; r < n; ++r)
      if (key[r] >= 0) p->f_perm[d0 + pos++] = r;
    std::vector<std::vector<int32_t>> sl(m);
    for (int32_t g = p->sub_slot[i]; g < p->sub_slot[i + 1]; ++g) {
      p->f_slot_dk[g] = key[p->f_slot_dof[g]];
      sl[key[p->f_slot_dof[g]]].push_back(g);
    }
    for (int32_t k = 0; k < m; ++k) {
      for (int32_t g : sl[k]) p->f_dk_slot.push_back(g);
      p->f_dk_off.push_back((int32_t)p->f_dk_slot.size());
    }
    p->f_m[i] = m;
    p->f_dkey_off[i + 1] = p->f_dkey_off[i] + m;
    const int64_t mt = (m + 15) / 16;
    p->f_sq_off[i + 1] = p->f_sq_off[i] + mt * (mt + 1) / 2 * 256;
    p->f_max_m = std::max(p->f_max_m, m);
    int32_t ng = 0;  // interfaces touching the block: the first slot row of each
    for (int32_t g = p->sub_slot[i]; g < p->sub_slot[i + 1]; ++g) ng += (p->slot_mk[g] & 7) == 0;
    p->f_max_ng = std::max(p->f_max_ng, ng);
  }
  p->f_lame_l.resize(ns);
  p->f_lame_m.resize(ns);
  for (int32_t i = 0; i < ns; ++i) {
    p->f_lame_l[i] = young[i] * poisson[i] / ((1.0 + poisson[i]) * (1.0 - 2.0 * poisson[i]));
    p->f_lame_m[i] = young[i] / (2.0 * (1.0 + poisson[i]));
  }
  p->f_rest.assign(rest, rest + 3 * (size_t)n_nodes);
  p->f_node_off = node_off;
  p->f_n_nodes = n_nodes;
  p->f_n_tets = n_tets;
  p->f_n_sq = p->f_sq_off[ns];
  p->f_n_dkey = p->f_dkey_off[ns];
  p->f_n_pairs = (int64_t)p->f_pair_ab.size();
  p->f_n_pent = (int64_t)p->f_pent.size();
  p->gravity = gravity;
  p->baumgarte = baumgarte;
  p->has_fem = true;
  if (p->n_big > 0) {
    // the FEM path factorises its blocks itself; the assembled solve's device-memory class
    // (and its operators) is not kept for FEM-model problems
    p->sub_ok = p->small_ok = false;
    p->sub_why = p->small_why = "FEM blocks beyond the LDS factorisation are solved by subadmm_fem_step";
  }
  plan_workspace(p);
  return SUBADMM_OK;
}

namespace {

FemModel make_fem(subadmm_problem* p) {
  auto& o = p->o;
  FemModel f;
  f.n_tets = p->f_n_tets;
  f.node_off = at<int32_t>(p, o.f_node_off);
  f.tet_off = at<int32_t>(p, o.f_tet_off);
  f.tet_node = at<int32_t>(p, o.f_tet_node);
  f.tet_g = at<double>(p, o.f_tet_g);
  f.tet_vol = at<double>(p, o.f_tet_vol);
  f.rest = at<double>(p, o.f_rest);
  f.mass = at<double>(p, o.f_mass);
  f.lame_l = at<double>(p, o.f_lame_l);
  f.lame_m = at<double>(p, o.f_lame_m);
  f.pair_off = at<int32_t>(p, o.f_pair_off);
  f.pair_ab = at<int32_t>(p, o.f_pair_ab);
  f.pent_off = at<int32_t>(p, o.f_pent_off);
  f.pent = at<int32_t>(p, o.f_pent);
  f.node_diag = at<int32_t>(p, o.f_node_diag);
  f.m = at<int32_t>(p, o.f_m);
  f.dkey_off = at<int32_t>(p, o.f_dkey_off);
  f.sq_off = at<int64_t>(p, o.f_sq_off);
  f.perm = at<int32_t>(p, o.f_perm);
  f.jtj = at<int32_t>(p, o.f_jtj);
  f.slot_dk = at<int32_t>(p, o.f_slot_dk);
  f.slot_dof = at<int32_t>(p, o.f_slot_dof);
  f.slot_sgn = at<float>(p, o.f_slot_sgn);
  f.dk_off = at<int32_t>(p, o.f_dk_off);
  f.dk_slot = at<int32_t>(p, o.f_dk_slot);
  f.if_node0 = at<int32_t>(p, o.f_if_node0);
  f.if_node1 = at<int32_t>(p, o.f_if_node1);
  f.gravity = p->gravity;
  f.baumgarte = p->baumgarte;
  return f;
}

template <typename T>
int run_fem_assemble(subadmm_problem* p, const T* pos, const T* vel, double dt, T* e) {
  const Topo t = make_topo(p);
  const FemModel f = make_fem(p);
  auto& o = p->o;
  return dev_err(p, timed(p, SUBADMM_K_ASSEMBLE, [&] {
                   hipError_t r = launch_fem_assemble<T>(t, f, pos, vel, dt, at<double>(p, o.fA), at<double>(p, o.fb),
                                                         at<double>(p, o.fscr), at<int32_t>(p, o.flags), p->stream);
                   if (r == hipSuccess) r = launch_fem_rows<T>(t, f, pos, dt, e, p->stream);
                   return r;
                 }),
                 "FEM assembly");
}

template <typename T>
int run_fem_step(subadmm_problem* p, T* pos, T* vel, double dt, int32_t max_iters, double tol, int32_t warm, T* v_hat,
                 T* lambda) {
  auto& o = p->o;
  const Topo t = make_topo(p);
  const FemModel f = make_fem(p);
  T* e = at<T>(p, o.fe);
  int rc = run_fem_assemble<T>(p, pos, vel, dt, e);
  if (rc) return rc;
  rc = dev_err(p, timed(p, SUBADMM_K_FACTOR, [&] {
                 return launch_fem_factor<T>(t, f, at<double>(p, o.fA), at<double>(p, o.fb), p->rho, at<T>(p, o.beta),
                                             at<double>(p, o.fL), at<double>(p, o.fA), at<T>(p, o.fS), at<T>(p, o.fcd),
                                             at<int32_t>(p, o.flags), at<int32_t>(p, o.fprec),
                                             at<double>(p, o.fkest), (double)p->fem_kappa_max, p->max_n, p->f_max_m,
                                             p->stream);
               }),
               "FEM factorisation");
  if (rc) return rc;
  p->fem_factored = true;
  FemLoopArgs<T> a;
  a.t = t;
  a.f = f;
  a.S = at<T>(p, o.fS);
  a.cd = at<T>(p, o.fcd);
  a.beta = at<T>(p, o.beta);
  a.e = e;
  a.mu = at<T>(p, o.mu);
  const bool prev = warm == SUBADMM_WARM_PREV;
  a.z_in = prev ? at<T>(p, o.zw) : nullptr;
  a.u_in = prev ? at<T>(p, o.uw) : nullptr;
  a.z_out = at<T>(p, o.zw);
  a.u_out = at<T>(p, o.uw);
  a.w_out = at<T>(p, o.fw);
  a.ybuf = at<T>(p, o.fy);
  a.lambda = lambda;
  a.part = at<double>(p, o.fpart);
  a.st_iters = at<int32_t>(p, o.st_it);
  a.st_total = at<long long>(p, o.st_tot);
  a.st_unconv = at<long long>(p, o.st_unc);
  a.st_conv = at<int32_t>(p, o.st_cv);
  a.st_theta = at<double>(p, o.st_th);
  a.st_rtheta = at<double>(p, o.st_rt);
  a.flags = at<int32_t>(p, o.flags);
  a.max_iters = max_iters;
  a.tol = tol;
  a.contact_model = p->contact_model;
  a.max_m = p->f_max_m;
  a.max_mt16 = (p->f_max_m + 15) / 16 * 16;
  a.max_nc = p->max_nc;
  a.max_ng = p->f_max_ng;
  a.n_slot = p->n_slot;
  a.resident = p->fem_resident;
  rc = dev_err(p, timed(p, SUBADMM_K_LOOP, [&] {
                 int form = 0;
                 const hipError_t r = launch_fem_loop<T>(a, &form, p->stream);
                 p->fem_form = form;
                 return r;
               }), "FEM iteration kernel");
  if (rc) return rc;
  T* vh = at<T>(p, o.fvh);
  rc = dev_err(p, timed(p, SUBADMM_K_ADVANCE, [&] {
                 hipError_t r = launch_fem_vhat<T>(t, f, at<double>(p, o.fL), at<double>(p, o.fA), at<double>(p, o.fb),
                                                   at<int32_t>(p, o.fprec), at<T>(p, o.fw), vh, p->max_n, p->stream);
                 if (r == hipSuccess) r = launch_fem_advance<T>(p->n_dof, vh, (T)dt, pos, vel, p->stream);
                 return r;
               }),
               "FEM state update");
  if (!rc) rc = impulse_out<T>(p, lambda, dt);
  if (rc) return rc;
  if (v_hat) rc = dev_err(p, hipMemcpyAsync(v_hat, vh, sizeof(T) * p->n_dof, hipMemcpyDeviceToDevice, p->stream), "copy v_hat");
  return rc;
}

}  // namespace

SUBADMM_API int subadmm_fem_assemble(subadmm_problem* p, const void* pos, const void* vel, double dt, void* A, void* b,
                                     void* J, void* e) {
  if (!p) return fail(nullptr, SUBADMM_E_ARG, "null problem");
  if (!p->has_fem) return fail(p, SUBADMM_E_STATE, "no FEM model set");
  if (!p->bound) return fail(p, SUBADMM_E_WORKSPACE, "problem has no bound workspace");
  if (!(dt > 0.0) || !std::isfinite(dt)) return fail(p, SUBADMM_E_ARG, "dt must be positive");
  if (!pos || !vel || !A || !b || (p->n_J > 0 && !J) || (p->n_rows > 0 && !e)) return fail(p, SUBADMM_E_ARG, "null array");
  const Topo t = make_topo(p);
  const FemModel f = make_fem(p);
  auto& o = p->o;
  int rc;
  if (p->dtype == SUBADMM_F64) {
    rc = run_fem_assemble<double>(p, (const double*)pos, (const double*)vel, dt, (double*)e);
    if (!rc)
      rc = dev_err(p, launch_fem_export<double>(t, f, at<double>(p, o.fA), at<double>(p, o.fb), (double*)A, (double*)b,
                                                (double*)J, p->stream),
                   "FEM export");
  } else {
    rc = run_fem_assemble<float>(p, (const float*)pos, (const float*)vel, dt, (float*)e);
    if (!rc)
      rc = dev_err(p, launch_fem_export<float>(t, f, at<double>(p, o.fA), at<double>(p, o.fb), (float*)A, (float*)b,
                                               (float*)J, p->stream),
                   "FEM export");
  }
  return rc;
}

SUBADMM_API int subadmm_fem_step(subadmm_problem* p, void* pos, void* vel, double dt, int32_t max_iters, double tol,
                                 int32_t warm, void* v_hat, void* lambda) {
  int rc = check_solve_args(p, max_iters, tol, warm == SUBADMM_WARM_GIVEN ? -1 : warm, nullptr, nullptr);
  if (rc) return rc;
  if (!p->has_fem) return fail(p, SUBADMM_E_STATE, "no FEM model set");
  if (!(dt > 0.0) || !std::isfinite(dt)) return fail(p, SUBADMM_E_ARG, "dt must be positive");
  if (!pos || !vel) return fail(p, SUBADMM_E_ARG, "null state array");
  p->boyd_valid = false;
  if (p->dtype == SUBADMM_F64)
    return run_fem_step<double>(p, (double*)pos, (double*)vel, dt, max_iters, tol, warm, (double*)v_hat,
                                (double*)lambda);
  return run_fem_step<float>(p, (float*)pos, (float*)vel, dt, max_iters, tol, warm, (float*)v_hat, (float*)lambda);
}

SUBADMM_API int subadmm_fem_loop_form(const subadmm_problem* p, int32_t* tiles) {
  if (!p || !tiles) return SUBADMM_E_ARG;
  *tiles = p->fem_form;
  return SUBADMM_OK;
}

SUBADMM_API int subadmm_fem_block_precision(subadmm_problem* p, void* kappa_est, void* fp64) {
  if (!p) return fail(nullptr, SUBADMM_E_ARG, "null problem");
  if (!p->has_fem) return fail(p, SUBADMM_E_STATE, "no FEM model set");
  if (!p->bound) return fail(p, SUBADMM_E_WORKSPACE, "problem has no bound workspace");
  if (!p->fem_factored) return fail(p, SUBADMM_E_STATE, "no FEM factorisation has run");
  if (!kappa_est && !fp64) return fail(p, SUBADMM_E_ARG, "null array");
  auto& o = p->o;
  if (kappa_est) {
    const int rc = dev_err(p, hipMemcpyAsync(kappa_est, at<double>(p, o.fkest), sizeof(double) * p->n_sub,
                                             hipMemcpyDeviceToDevice, p->stream), "copy kappa_est");
    if (rc) return rc;
  }
  if (fp64)
    return dev_err(p, hipMemcpyAsync(fp64, at<int32_t>(p, o.fprec), sizeof(int32_t) * p->n_sub,
                                     hipMemcpyDeviceToDevice, p->stream), "copy block precision");
  return SUBADMM_OK;
}

namespace {
// A step replayed from a HIP graph: captured (stream capture on a private stream, so that
// forked factorisation streams are captured too) on the first call with `key` or after
// any change of it, then launched into the bound stream.
template <typename F>
int graph_step(subadmm_problem* p, const subadmm_problem::GraphKey& key, F&& run) {
  if (!p->graph_exec || !(key == p->graph_key)) {
    release_graph(p);
    hipError_t e = hipSuccess;
    if (!p->cap_stream) e = hipStreamCreateWithFlags(&p->cap_stream, hipStreamNonBlocking);
    if (e != hipSuccess) return dev_err(p, e, "capture stream");
    // everything queued on the bound stream so far completes before the capture's first
    // launch when the graph is launched into the bound stream, so no fork is needed here
    e = hipStreamBeginCapture(p->cap_stream, hipStreamCaptureModeThreadLocal);
    if (e != hipSuccess) return dev_err(p, e, "begin capture");
    hipStream_t bound = p->stream;
    p->stream = p->cap_stream;
    p->capturing = true;
    const int rc = run();
    p->capturing = false;
    p->stream = bound;
    hipGraph_t g = nullptr;
    e = hipStreamEndCapture(p->cap_stream, &g);
    if (rc) {
      if (g) (void)hipGraphDestroy(g);
      return rc;
    }
    if (e != hipSuccess) return dev_err(p, e, "end capture");
    p->graph = g;
    e = hipGraphInstantiate(&p->graph_exec, p->graph, nullptr, nullptr, 0);
    if (e != hipSuccess) {
      release_graph(p);
      return dev_err(p, e, "instantiate graph");
    }
    p->graph_key = key;
  }
  return dev_err(p, hipGraphLaunch(p->graph_exec, p->stream), "launch graph");
}
}  // namespace

SUBADMM_API int subadmm_rigid_step_graph(subadmm_problem* p, void* pos, void* rot, void* vel, void* omega,
                                         double dt, int32_t max_iters, double tol, int32_t warm, void* v_hat,
                                         void* lambda) {
  int rc = check_solve_args(p, max_iters, tol, warm == SUBADMM_WARM_LEARNED ? SUBADMM_WARM_PREV
                                               : warm == SUBADMM_WARM_GIVEN ? -1 : warm,
                            nullptr, nullptr);
  if (rc) return rc;
  if (!p->has_rigid) return fail(p, SUBADMM_E_STATE, "no rigid model set");
  if (!(dt > 0.0) || !std::isfinite(dt)) return fail(p, SUBADMM_E_ARG, "dt must be positive");
  if (!pos || !rot || !vel || !omega) return fail(p, SUBADMM_E_ARG, "null state array");
  if (!p->sub_ok) return fail(p, SUBADMM_E_ARG, "problem exceeds the per-subsystem solver: " + p->sub_why);
  if (warm == SUBADMM_WARM_LEARNED && (!p->small_ok || p->force_large))
    return fail(p, SUBADMM_E_ARG, "the learned start needs scenes that fit the per-scene kernel");
  const subadmm_problem::GraphKey key{pos,
                                      rot,
                                      vel,
                                      omega,
                                      v_hat,
                                      lambda,
                                      dt,
                                      tol,
                                      max_iters,
                                      warm,
                                      p->cfg_gen,
                                      p->net[0],
                                      p->net[1],
                                      p->net[0] ? mlp_generation(p->net[0]) : 0,
                                      p->net[1] ? mlp_generation(p->net[1]) : 0};
  rc = graph_step(p, key, [&] {
    if (p->dtype == SUBADMM_F64)
      return run_rigid_step<double>(p, (double*)pos, (double*)rot, (double*)vel, (double*)omega, dt, max_iters, tol,
                                    warm, (double*)v_hat, (double*)lambda);
    return run_rigid_step<float>(p, (float*)pos, (float*)rot, (float*)vel, (float*)omega, dt, max_iters, tol, warm,
                                 (float*)v_hat, (float*)lambda);
  });
  // the graph holds the residual pair's kernel when the option was on at capture (an option
  // change captures again)
  if (!rc) p->boyd_valid = p->boyd != 0;
  return rc;
}

SUBADMM_API int subadmm_fem_step_graph(subadmm_problem* p, void* pos, void* vel, double dt, int32_t max_iters,
                                       double tol, int32_t warm, void* v_hat, void* lambda) {
  int rc = check_solve_args(p, max_iters, tol, warm == SUBADMM_WARM_GIVEN ? -1 : warm, nullptr, nullptr);
  if (rc) return rc;
  if (warm == SUBADMM_WARM_LEARNED) return fail(p, SUBADMM_E_ARG, "the FEM step starts cold or from the previous step");
  if (!p->has_fem) return fail(p, SUBADMM_E_STATE, "no FEM model set");
  if (!(dt > 0.0) || !std::isfinite(dt)) return fail(p, SUBADMM_E_ARG, "dt must be positive");
  if (!pos || !vel) return fail(p, SUBADMM_E_ARG, "null state array");
  p->boyd_valid = false;
  const subadmm_problem::GraphKey key{pos, nullptr, vel, nullptr, v_hat, lambda, dt, tol, max_iters, warm,
                                      p->cfg_gen, nullptr, nullptr, 0, 0};
  return graph_step(p, key, [&] {
    if (p->dtype == SUBADMM_F64)
      return run_fem_step<double>(p, (double*)pos, (double*)vel, dt, max_iters, tol, warm, (double*)v_hat,
                                  (double*)lambda);
    return run_fem_step<float>(p, (float*)pos, (float*)vel, dt, max_iters, tol, warm, (float*)v_hat, (float*)lambda);
  });
}

namespace {
// Blocking copy of the per-scene statistics from the current workspace.
int read_stats_now(subadmm_problem* p, subadmm_stats* host_out) {
  const size_t n = p->n_scene;
  std::vector<int32_t> it(n), cv(n);
  std::vector<double> th(n), rt(n), rp(n, std::nan("")), rd(n, std::nan(""));
  std::vector<long long> tot(n), unc(n), fb(n);
  hipError_t e = hipMemcpyAsync(it.data(), p->ws + p->o.st_it, 4 * n, hipMemcpyDeviceToHost, p->stream);
  if (e == hipSuccess) e = hipMemcpyAsync(cv.data(), p->ws + p->o.st_cv, 4 * n, hipMemcpyDeviceToHost, p->stream);
  if (e == hipSuccess) e = hipMemcpyAsync(th.data(), p->ws + p->o.st_th, 8 * n, hipMemcpyDeviceToHost, p->stream);
  if (e == hipSuccess) e = hipMemcpyAsync(rt.data(), p->ws + p->o.st_rt, 8 * n, hipMemcpyDeviceToHost, p->stream);
  if (e == hipSuccess) e = hipMemcpyAsync(tot.data(), p->ws + p->o.st_tot, 8 * n, hipMemcpyDeviceToHost, p->stream);
  if (e == hipSuccess) e = hipMemcpyAsync(unc.data(), p->ws + p->o.st_unc, 8 * n, hipMemcpyDeviceToHost, p->stream);
  if (e == hipSuccess) e = hipMemcpyAsync(fb.data(), p->ws + p->o.st_fb, 8 * n, hipMemcpyDeviceToHost, p->stream);
  if (e == hipSuccess && p->boyd_valid)
    e = hipMemcpyAsync(rp.data(), p->ws + p->o.st_rp, 8 * n, hipMemcpyDeviceToHost, p->stream);
  if (e == hipSuccess && p->boyd_valid)
    e = hipMemcpyAsync(rd.data(), p->ws + p->o.st_rd, 8 * n, hipMemcpyDeviceToHost, p->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(p->stream);
  if (e != hipSuccess) return dev_err(p, e, "read stats");
  for (size_t s = 0; s < n; ++s)
    host_out[s] = subadmm_stats{it[s], cv[s], th[s], rt[s], (int64_t)tot[s], (int64_t)unc[s], (int64_t)fb[s], rp[s], rd[s]};
  return SUBADMM_OK;
}
}  // namespace

namespace {
template <typename T>
int run_constraint_error(subadmm_problem* p, const T* J, const T* e, const T* v_hat, const T* lambda, int kinds,
                         double* out) {
  auto& o = p->o;
  ErrorArgs<T> a;
  a.t = make_topo(p);
  a.J = J;
  a.e = e;
  a.slot_dof = nullptr;
  a.slot_sgn = nullptr;
  if (!J && p->has_rigid) {
    a.J = at<T>(p, o.sJ);
    a.e = at<T>(p, o.se);
  } else if (!J && p->has_fem) {
    a.slot_dof = at<int32_t>(p, o.f_slot_dof);
    a.slot_sgn = at<float>(p, o.f_slot_sgn);
    a.e = at<T>(p, o.fe);
  }
  a.v_hat = v_hat;
  a.lambda = lambda;
  a.beta = at<T>(p, o.beta);
  a.mu = at<T>(p, o.mu);
  a.ksoft = at<T>(p, o.ksoft);
  a.asoft = at<T>(p, o.asoft);
  a.out = at<double>(p, o.err);
  a.kinds = kinds;
  hipError_t he = launch_constraint_error<T>(a, p->stream);
  if (he == hipSuccess)
    he = hipMemcpyAsync(out, a.out, sizeof(double) * p->n_scene, hipMemcpyDeviceToHost, p->stream);
  if (he == hipSuccess) he = hipStreamSynchronize(p->stream);
  return dev_err(p, he, "constraint error");
}
}  // namespace

SUBADMM_API int subadmm_constraint_error(subadmm_problem* p, const void* J, const void* e, const void* v_hat,
                                         const void* lambda, int kinds, double* host_out) {
  if (!p) return fail(nullptr, SUBADMM_E_ARG, "null problem");
  if (!p->bound) return fail(p, SUBADMM_E_WORKSPACE, "problem has no bound workspace");
  if (!v_hat || !lambda || !host_out) return fail(p, SUBADMM_E_ARG, "null argument");
  if (!J != !e) return fail(p, SUBADMM_E_ARG, "J and e are given together or not at all");
  if (!J && !p->has_rigid && !p->has_fem) return fail(p, SUBADMM_E_ARG, "an assembled problem needs J and e");
  if (kinds <= 0 || kinds > 15) return fail(p, SUBADMM_E_ARG, "kinds is a non-empty mask of bits 0..3");
  if (p->dtype == SUBADMM_F64)
    return run_constraint_error<double>(p, (const double*)J, (const double*)e, (const double*)v_hat,
                                        (const double*)lambda, kinds, host_out);
  return run_constraint_error<float>(p, (const float*)J, (const float*)e, (const float*)v_hat, (const float*)lambda,
                                     kinds, host_out);
}

SUBADMM_API int subadmm_read_stats(subadmm_problem* p, subadmm_stats* host_out) {
  if (!p || !host_out) return fail(p, SUBADMM_E_ARG, "null argument");
  if (!p->bound) return fail(p, SUBADMM_E_WORKSPACE, "problem has no bound workspace");
  return read_stats_now(p, host_out);
}

SUBADMM_API int subadmm_reset_totals(subadmm_problem* p) {
  if (!p) return fail(nullptr, SUBADMM_E_ARG, "null problem");
  if (!p->bound) return fail(p, SUBADMM_E_WORKSPACE, "problem has no bound workspace");
  hipError_t e = hipMemsetAsync(p->ws + p->o.st_tot, 0, sizeof(long long) * p->n_scene, p->stream);
  if (e == hipSuccess) e = hipMemsetAsync(p->ws + p->o.st_unc, 0, sizeof(long long) * p->n_scene, p->stream);
  if (e == hipSuccess) e = hipMemsetAsync(p->ws + p->o.st_fb, 0, sizeof(long long) * p->n_scene, p->stream);
  return dev_err(p, e, "reset totals");
}

SUBADMM_API int subadmm_timing_begin(subadmm_problem* p, int32_t max_launches) {
  if (!p) return fail(nullptr, SUBADMM_E_ARG, "null problem");
  if (!p->bound) return fail(p, SUBADMM_E_WORKSPACE, "problem has no bound workspace");
  if (max_launches < 1 || max_launches > (1 << 20)) return fail(p, SUBADMM_E_ARG, "max_launches out of range");
  if (p->timing) return fail(p, SUBADMM_E_STATE, "timing already active");
  p->ev0.assign(max_launches, nullptr);
  p->ev1.assign(max_launches, nullptr);
  p->ev_kernel.assign(max_launches, -1);
  for (int32_t k = 0; k < max_launches; ++k) {
    hipError_t e = hipEventCreate(&p->ev0[k]);
    if (e == hipSuccess) e = hipEventCreate(&p->ev1[k]);
    if (e != hipSuccess) {
      for (auto ev : p->ev0) if (ev) (void)hipEventDestroy(ev);
      for (auto ev : p->ev1) if (ev) (void)hipEventDestroy(ev);
      p->ev0.clear();
      p->ev1.clear();
      return dev_err(p, e, "event create");
    }
  }
  p->timing = true;
  p->timing_max = max_launches;
  p->timing_used = 0;
  p->timing_dropped = 0;
  return SUBADMM_OK;
}

SUBADMM_API int subadmm_timing_end(subadmm_problem* p, double* ms_out, int32_t* count_out) {
  if (!p || !ms_out || !count_out) return fail(p, SUBADMM_E_ARG, "null argument");
  if (!p->timing) return fail(p, SUBADMM_E_STATE, "timing not active");
  for (int k = 0; k < SUBADMM_NUM_KERNELS; ++k) {
    ms_out[k] = 0.0;
    count_out[k] = 0;
  }
  hipError_t e = hipStreamSynchronize(p->stream);
  for (int32_t k = 0; e == hipSuccess && k < p->timing_used; ++k) {
    float ms = 0.f;
    e = hipEventElapsedTime(&ms, p->ev0[k], p->ev1[k]);
    if (e == hipSuccess && p->ev_kernel[k] >= 0) {
      ms_out[p->ev_kernel[k]] += ms;
      count_out[p->ev_kernel[k]] += 1;
    }
  }
  for (auto ev : p->ev0) (void)hipEventDestroy(ev);
  for (auto ev : p->ev1) (void)hipEventDestroy(ev);
  p->ev0.clear();
  p->ev1.clear();
  p->timing = false;
  if (e != hipSuccess) return dev_err(p, e, "timing end");
  if (p->timing_dropped) return fail(p, SUBADMM_E_ARG, "more launches than max_launches were made");
  return SUBADMM_OK;
}

SUBADMM_API int subadmm_copy_beta(subadmm_problem* p, void* dev_out) {
  if (!p || !dev_out) return fail(p, SUBADMM_E_ARG, "null argument");
  if (!p->bound) return fail(p, SUBADMM_E_WORKSPACE, "problem has no bound workspace");
  return dev_err(p, hipMemcpyAsync(dev_out, p->ws + p->o.beta, p->rsize() * p->n_sub, hipMemcpyDeviceToDevice, p->stream),
                 "copy beta");
}

SUBADMM_API int subadmm_check(subadmm_problem* p) {
  if (!p) return fail(nullptr, SUBADMM_E_ARG, "null problem");
  if (!p->bound) return fail(p, SUBADMM_E_WORKSPACE, "problem has no bound workspace");
  int32_t flags = 0;
  hipError_t e = hipMemcpyAsync(&flags, p->ws + p->o.flags, 4, hipMemcpyDeviceToHost, p->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(p->stream);
  if (e != hipSuccess) return dev_err(p, e, "check");
  if (flags) {
    const int32_t zero = 0;
    e = hipMemcpyAsync(p->ws + p->o.flags, &zero, 4, hipMemcpyHostToDevice, p->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(p->stream);
    if (e != hipSuccess) return dev_err(p, e, "check reset");
  }
  if (flags & FLAG_NOT_SPD) return fail(p, SUBADMM_E_NOT_SPD, "a factorised matrix had a non-positive pivot");
  if (flags & FLAG_NONFINITE) return fail(p, SUBADMM_E_NONFINITE, "non-finite residual");
  if (flags & FLAG_BARRIER) return fail(p, SUBADMM_E_DEVICE, "grid barrier of the FEM iteration timed out");
  return SUBADMM_OK;
}

SUBADMM_API int subadmm_set_warm_model(subadmm_problem* p, int32_t cls, subadmm_mlp* net) {
  if (!p) return fail(nullptr, SUBADMM_E_ARG, "null problem");
  if (cls != 0 && cls != 1) return fail(p, SUBADMM_E_ARG, "class must be 0 (contacts) or 1 (joints)");
  if (net) {
    const int32_t in = cls == 0 ? kContactIn : kJointIn, out = cls == 0 ? kContactOut : kJointOut;
    if (mlp_input_width(net) != in || mlp_output_width(net) != out)
      return fail(p, SUBADMM_E_ARG, "network widths do not match the class's features and outputs");
    if (mlp_max_batch(net) < p->n_class[cls]) return fail(p, SUBADMM_E_ARG, "network max_batch below the class size");
    if (p->bound && mlp_stream(net) != p->stream) return fail(p, SUBADMM_E_ARG, "network bound to another stream");
  }
  p->net[cls] = net;
  ++p->cfg_gen;
  return SUBADMM_OK;
}

SUBADMM_API int subadmm_warm_class_counts(const subadmm_problem* p, int32_t* n_contact, int32_t* n_joint) {
  if (!p || !n_contact || !n_joint) return SUBADMM_E_ARG;
  *n_contact = p->n_class[0];
  *n_joint = p->n_class[1];
  return SUBADMM_OK;
}

SUBADMM_API int subadmm_set_recording(subadmm_problem* p, float* xc, float* xj, float* tc, float* tj, float* wc,
                                      float* wj) {
  if (!p) return fail(nullptr, SUBADMM_E_ARG, "null problem");
  if (!p->has_rigid) return fail(p, SUBADMM_E_STATE, "no rigid model set");
  p->rec_xc = xc;
  p->rec_xj = xj;
  p->rec_tc = tc;
  p->rec_tj = tj;
  p->rec_wc = wc;
  p->rec_wj = wj;
  ++p->cfg_gen;
  return SUBADMM_OK;
}

SUBADMM_API int subadmm_get_warm(subadmm_problem* p, void* z_out, void* u_out) {
  if (!p || !z_out || !u_out) return fail(p, SUBADMM_E_ARG, "null argument");
  if (!p->bound) return fail(p, SUBADMM_E_WORKSPACE, "problem has no bound workspace");
  const size_t bytes = p->rsize() * p->n_slot;
  hipError_t e = hipMemcpyAsync(z_out, p->ws + p->o.zw, bytes, hipMemcpyDeviceToDevice, p->stream);
  if (e == hipSuccess) e = hipMemcpyAsync(u_out, p->ws + p->o.uw, bytes, hipMemcpyDeviceToDevice, p->stream);
  return dev_err(p, e, "get warm");
}

SUBADMM_API int subadmm_set_warm(subadmm_problem* p, const void* z, const void* u) {
  if (!p || !z || !u) return fail(p, SUBADMM_E_ARG, "null argument");
  if (!p->bound) return fail(p, SUBADMM_E_WORKSPACE, "problem has no bound workspace");
  const size_t bytes = p->rsize() * p->n_slot;
  hipError_t e = hipMemcpyAsync(p->ws + p->o.zw, z, bytes, hipMemcpyDeviceToDevice, p->stream);
  if (e == hipSuccess) e = hipMemcpyAsync(p->ws + p->o.uw, u, bytes, hipMemcpyDeviceToDevice, p->stream);
  return dev_err(p, e, "set warm");
}

SUBADMM_API void subadmm_destroy(subadmm_problem* p) {
  if (!p) return;
  release_graph(p);
  release_side(p);
  release_cap_stream(p);
  for (auto ev : p->ev0) if (ev) (void)hipEventDestroy(ev);
  for (auto ev : p->ev1) if (ev) (void)hipEventDestroy(ev);
  delete p;
}

SUBADMM_API const char* subadmm_last_error(const subadmm_problem* p) {
  return p ? p->err.c_str() : g_setup_error.c_str();
}
