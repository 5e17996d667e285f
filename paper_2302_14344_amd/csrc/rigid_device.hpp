// Device functions of the rigid-box model in maximal coordinates: the construction steps
// of Algorithm 1 (Eq. (2)-(5)) for one subsystem and the state update of Eq. (2) for one
// body.  Used by the per-step kernels and by the multi-step kernel.
//
// Generalised velocity of a body: (v in the world frame, omega in the body frame),
// M = diag(m I3, I_b) with I_b the principal inertia.  A body point r (body frame)
// moves with v + R (omega x r); along a world direction d its Jacobian row is
// (d, r x R^T d).  The world angular velocity along a world direction n has the row
// (0, R^T n).
#pragma once

#include "internal.hpp"

namespace subadmm {

template <typename T>
__device__ inline void rt_vec(const T* R, const T* d, T* o) {  // R^T d
  o[0] = R[0] * d[0] + R[3] * d[1] + R[6] * d[2];
  o[1] = R[1] * d[0] + R[4] * d[1] + R[7] * d[2];
  o[2] = R[2] * d[0] + R[5] * d[1] + R[8] * d[2];
}
template <typename T>
__device__ inline void r_vec(const T* R, const T* v, T* o) {  // R v
  o[0] = R[0] * v[0] + R[1] * v[1] + R[2] * v[2];
  o[1] = R[3] * v[0] + R[4] * v[1] + R[5] * v[2];
  o[2] = R[6] * v[0] + R[7] * v[1] + R[8] * v[2];
}
template <typename T>
__device__ inline void cross(const T* a, const T* b, T* o) {
  o[0] = a[1] * b[2] - a[2] * b[1];
  o[1] = a[2] * b[0] - a[0] * b[2];
  o[2] = a[0] * b[1] - a[1] * b[0];
}

// Row k (0..4) of a revolute joint for one body: k < 3 the anchor velocity along
// world axis k, else the world angular velocity along n.
template <typename T>
__device__ inline void joint_row(const T* R, const T* anchor, const T* n, int k, T* row) {
  if (k < 3) {
    T d[3] = {(T)0, (T)0, (T)0};
    d[k] = (T)1;
    T a[3];
    rt_vec(R, d, a);
    row[0] = d[0]; row[1] = d[1]; row[2] = d[2];
    cross(anchor, a, row + 3);
  } else {
    row[0] = row[1] = row[2] = (T)0;
    rt_vec(R, n, row + 3);
  }
}

// Rotation vector of the rotation matrix Q (row-major), FP64: angle acos((tr Q - 1)/2) about
// vee(Q - Q^T) / (2 sin angle), the factor angle / sin(angle) from its series for small
// angles.
__device__ inline void so3_log_d(const double* Q, double* th) {
  double c = 0.5 * (Q[0] + Q[4] + Q[8] - 1.0);
  c = c > 1.0 ? 1.0 : (c < -1.0 ? -1.0 : c);
  const double ang = acos(c);
  const double f = ang < 1e-4 ? 1.0 + ang * ang / 6.0 : ang / sin(ang);
  th[0] = 0.5 * f * (Q[7] - Q[5]);
  th[1] = 0.5 * f * (Q[2] - Q[6]);
  th[2] = 0.5 * f * (Q[3] - Q[1]);
}

// Row k of link q for member mem of interface j, added into row (the slot row of this
// subsystem, length n), and e_j,k for member 0.  Directions d_k = R_a f_k with f_k fixed in
// body a's frame.  Linear links: anchor-point velocity of a minus that of b along d_k,
// phi_k = (x_a - x_b) . d_k.  Angular links: world angular velocity of a minus that of b
// along d_k, phi_k = -f_k . log(R_a^T R_b).  One-body links have a's rows only and no error.
// Errors by interface kind: soft e = phi (Eq. 3 with the spring's position error),
// contact (phi_0 / t, 0, 0), equality and hard gamma phi / t (Baumgarte).  phi is formed in
// FP64 from the stored state (differences of positions or rotations of similar size).
// Separation phi of row k of a two-body link, in FP64 from the stored state: the anchor
// separation along d = R_a f (linear), or minus f . log(R_a^T R_b) (angular).
template <typename T>
__device__ inline double rigid_link_phi(const RigidModel<T>& m, const int q, const int k, const T* pos,
                                        const T* rot) {
  const int ba = m.link_body[2 * q], bb = m.link_body[2 * q + 1];
  const T* Ra = rot + 9 * ba;
  const T* Rb = rot + 9 * bb;
  const T* f = m.link_frame + 9 * q + 3 * k;
  const T* ra = m.link_anchor + 6 * q;
  const T* rb = ra + 3;
  double phi = 0.0;
  if (m.link_type[q] == 1) {
    double Q[9], th[3];
    for (int r = 0; r < 3; ++r)
      for (int c = 0; c < 3; ++c)
        Q[3 * r + c] = (double)Ra[r] * (double)Rb[c] + (double)Ra[3 + r] * (double)Rb[3 + c] +
                       (double)Ra[6 + r] * (double)Rb[6 + c];
    so3_log_d(Q, th);
    phi = -((double)f[0] * th[0] + (double)f[1] * th[1] + (double)f[2] * th[2]);
  } else {
    for (int r = 0; r < 3; ++r) {
      const double dd =
          (double)Ra[3 * r] * (double)f[0] + (double)Ra[3 * r + 1] * (double)f[1] + (double)Ra[3 * r + 2] * (double)f[2];
      double xa = (double)pos[3 * ba + r], xb = (double)pos[3 * bb + r];
      for (int c = 0; c < 3; ++c) {
        xa += (double)Ra[3 * r + c] * (double)ra[c];
        xb += (double)Rb[3 * r + c] * (double)rb[c];
      }
      phi += (xa - xb) * dd;
    }
  }
  return phi;
}

template <typename T>
__device__ __attribute__((noinline)) double rigid_link_phi_outlined(const RigidModel<T>& m, const int q, const int k,
                                                                    const T* pos, const T* rot) {
  return rigid_link_phi<T>(m, q, k, pos, rot);
}

template <typename T, bool kOutline>
__device__ inline double link_phi(const RigidModel<T>& m, const int q, const int k, const T* pos, const T* rot) {
  if constexpr (kOutline)
    return rigid_link_phi_outlined<T>(m, q, k, pos, rot);
  else
    return rigid_link_phi<T>(m, q, k, pos, rot);
}

// Soft links between two bodies of subsystem i folded into its dynamics (the option of the
// remark after Eq. 6): lambda = -k (phi + alpha J v_hat) is linear in v_hat, so A_i gains
// k alpha J^T J and b_i loses k J^T phi, J the link's rows over the two bodies' columns
// (body a's row minus body b's).  Whole workgroup; links one after another (two links may
// share a body).
template <typename T, bool kOutline = false>
__device__ __attribute__((always_inline)) inline void rigid_fold_links(const Topo& t, const RigidModel<T>& m,
                                                                       const int i, const T* pos, const T* rot,
                                                                       T* Ai, T* bi) {
  const int l0 = m.sub_ilink_off[i], l1 = m.sub_ilink_off[i + 1];
  if (l1 <= l0) return;
  // the link's rows (3 x 12: body a's 6 columns, then body b's) and phi, staged in LDS
  __shared__ double s_row[3][12];
  __shared__ double s_phi[3];
  const int tid = threadIdx.x, bd = blockDim.x;
  const int n = t.sub_n[i];
  __syncthreads();
  for (int li = l0; li < l1; ++li) {
    const int q = m.sub_ilink[li];
    const int ba = m.link_body[2 * q], bb = m.link_body[2 * q + 1];
    const int dim = m.link_dim[q];
    for (int w = tid; w < 39; w += bd) {
      if (w >= 36) {
        const int k = w - 36;
        s_phi[k] = k < dim ? link_phi<T, kOutline>(m, q, k, pos, rot) : 0.0;
        continue;
      }
      const int k = w / 12, c = w % 12;
      double v = 0.0;
      if (k < dim) {
        const T* f = m.link_frame + 9 * q + 3 * k;
        const T* Ra = rot + 9 * ba;
        const T* Rb = rot + 9 * bb;
        T d[3], db[3], x[3];
        r_vec(Ra, f, d);
        rt_vec(Rb, d, db);
        const int part = c / 3, cc = c % 3;  // a linear, a angular, b linear, b angular
        if (m.link_type[q] == 1) {
          v = part == 1 ? (double)f[cc] : part == 3 ? -(double)db[cc] : 0.0;
        } else if (part == 0 || part == 2) {
          v = part == 0 ? (double)d[cc] : -(double)d[cc];
        } else if (part == 1) {
          cross(m.link_anchor + 6 * q, f, x);
          v = (double)x[cc];
        } else {
          cross(m.link_anchor + 6 * q + 3, db, x);
          v = -(double)x[cc];
        }
      }
      s_row[k][c] = v;
    }
    __syncthreads();
    const int ca = 6 * m.body_local[ba], cb = 6 * m.body_local[bb];
    const double kk = (double)m.link_k[q], ka = kk * (double)m.link_alpha[q];
    for (int w = tid; w < 144 + 12; w += bd) {
      if (w < 144) {
        const int r = w / 12, c = w % 12;
        double s = 0.0;
        for (int k = 0; k < dim; ++k) s += s_row[k][r] * s_row[k][c];
        const int gr = (r < 6 ? ca : cb - 6) + r, gc = (c < 6 ? ca : cb - 6) + c;
        Ai[gr * n + gc] += (T)(ka * s);
      } else {
        const int r = w - 144;
        double s = 0.0;
        for (int k = 0; k < dim; ++k) s += s_phi[k] * s_row[k][r];
        bi[(r < 6 ? ca : cb - 6) + r] -= (T)(kk * s);
      }
    }
    __syncthreads();
  }
}

// Sphere contact link (link type 2, a contact interface): row k of body a (and b) along the
// contact frame.  Two bodies: the normal n = (x_a - x_b)/|x_a - x_b| from the centres, gap
// |x_a - x_b| - r_a - r_b (radii in the first anchor entries), tangents from the world axis
// least aligned with n; one body: a plane with world normal and tangents in the link frame
// rows and offset in b's first anchor entry, gap n . x_a - offset - r_a.  Contact points on
// the spheres along n (-r_a n, +r_b n); rows (d, R^T (p x d)) for a, minus that for b;
// e = (gap/t, 0, 0).  Geometry in FP64.
template <typename T>
__device__ inline void rigid_sphere_row(const Topo& t, const RigidModel<T>& m, const int q, const int j,
                                        const int mem, const int k, const T* pos, const T* rot, const T dt,
                                        T* row, T* e) {
  const int ba = m.link_body[2 * q], bb = m.link_body[2 * q + 1];
  const T* an = m.link_anchor + 6 * q;
  const double rad_a = (double)an[0];
  double n[3], tg[2][3], gap;
  if (bb >= 0) {
    double len2 = 0.0;
    for (int c = 0; c < 3; ++c) {
      n[c] = (double)pos[3 * ba + c] - (double)pos[3 * bb + c];
      len2 += n[c] * n[c];
    }
    const double len = __builtin_sqrt(len2);
    for (int c = 0; c < 3; ++c) n[c] /= len;
    gap = len - rad_a - (double)an[3];
    int ax = 0;
    for (int c = 1; c < 3; ++c)
      if (__builtin_fabs(n[c]) < __builtin_fabs(n[ax])) ax = c;
    double l1 = 0.0;
    for (int c = 0; c < 3; ++c) {
      tg[0][c] = (c == ax ? 1.0 : 0.0) - n[ax] * n[c];
      l1 += tg[0][c] * tg[0][c];
    }
    l1 = __builtin_sqrt(l1);
    for (int c = 0; c < 3; ++c) tg[0][c] /= l1;
    tg[1][0] = n[1] * tg[0][2] - n[2] * tg[0][1];
    tg[1][1] = n[2] * tg[0][0] - n[0] * tg[0][2];
    tg[1][2] = n[0] * tg[0][1] - n[1] * tg[0][0];
  } else {
    const T* f = m.link_frame + 9 * q;
    for (int c = 0; c < 3; ++c) {
      n[c] = (double)f[c];
      tg[0][c] = (double)f[3 + c];
      tg[1][c] = (double)f[6 + c];
    }
    gap = n[0] * (double)pos[3 * ba] + n[1] * (double)pos[3 * ba + 1] + n[2] * (double)pos[3 * ba + 2] -
          (double)an[3] - rad_a;
  }
  const double* d = k == 0 ? n : tg[k - 1];
  auto body_row = [&](const int b, const double rad, T* out) {
    // p = rad n (signed radius: -r_a for a, +r_b for b); angular part R^T (p x d)
    double p[3] = {rad * n[0], rad * n[1], rad * n[2]};
    double cr[3] = {p[1] * d[2] - p[2] * d[1], p[2] * d[0] - p[0] * d[2], p[0] * d[1] - p[1] * d[0]};
    const T* R = rot + 9 * b;
    for (int c = 0; c < 3; ++c) {
      out[c] = (T)d[c];
      out[3 + c] = (T)((double)R[c] * cr[0] + (double)R[3 + c] * cr[1] + (double)R[6 + c] * cr[2]);
    }
  };
  T rowa[6], rowb[6];
  body_row(ba, -rad_a, rowa);
  if (bb >= 0) body_row(bb, (double)an[3], rowb);
  const int ca = 6 * m.body_local[ba];
  if (t.if_nsub[j] == 1) {
    for (int c = 0; c < 6; ++c) row[ca + c] += rowa[c];
    if (bb >= 0) {
      const int cb = 6 * m.body_local[bb];
      for (int c = 0; c < 6; ++c) row[cb + c] -= rowb[c];
    }
  } else if (mem == 0) {
    for (int c = 0; c < 6; ++c) row[ca + c] = rowa[c];
  } else {
    const int cb = 6 * m.body_local[bb];
    for (int c = 0; c < 6; ++c) row[cb + c] = -rowb[c];
  }
  if (mem == 0) e[t.if_row[j] + k] = (T)(k == 0 ? gap / (double)dt : 0.0);
}

template <typename T, bool kOutline = false>
__device__ inline void rigid_link_row(const Topo& t, const RigidModel<T>& m, const int q, const int j, const int mem,
                                      const int k, const T* pos, const T* rot, const T dt, T* row, T* e) {
  if (m.link_type[q] == 2) {
    rigid_sphere_row<T>(t, m, q, j, mem, k, pos, rot, dt, row, e);
    return;
  }
  const int ba = m.link_body[2 * q], bb = m.link_body[2 * q + 1];
  const bool ang = m.link_type[q] == 1;
  const T* Ra = rot + 9 * ba;
  const T* f = m.link_frame + 9 * q + 3 * k;
  const T* ra = m.link_anchor + 6 * q;
  const T* rb = ra + 3;
  T d[3];
  r_vec(Ra, f, d);
  T rowa[6], rowb[6];
  // a: R_a^T d = f
  if (ang) {
    rowa[0] = rowa[1] = rowa[2] = (T)0;
    rowa[3] = f[0]; rowa[4] = f[1]; rowa[5] = f[2];
  } else {
    rowa[0] = d[0]; rowa[1] = d[1]; rowa[2] = d[2];
    cross(ra, f, rowa + 3);
  }
  if (bb >= 0) {
    const T* Rb = rot + 9 * bb;
    T db[3];
    rt_vec(Rb, d, db);
    if (ang) {
      rowb[0] = rowb[1] = rowb[2] = (T)0;
      rowb[3] = db[0]; rowb[4] = db[1]; rowb[5] = db[2];
    } else {
      rowb[0] = d[0]; rowb[1] = d[1]; rowb[2] = d[2];
      cross(rb, db, rowb + 3);
    }
  }
  const int ca = 6 * m.body_local[ba];
  if (t.if_nsub[j] == 1) {
    for (int c = 0; c < 6; ++c) row[ca + c] += rowa[c];
    if (bb >= 0) {
      const int cb = 6 * m.body_local[bb];
      for (int c = 0; c < 6; ++c) row[cb + c] -= rowb[c];
    }
  } else if (mem == 0) {
    for (int c = 0; c < 6; ++c) row[ca + c] = rowa[c];
  } else {
    const int cb = 6 * m.body_local[bb];
    for (int c = 0; c < 6; ++c) row[cb + c] = -rowb[c];
  }
  if (mem != 0) return;
  const double phi = bb >= 0 ? link_phi<T, kOutline>(m, q, k, pos, rot) : 0.0;
  const int kind = t.if_kind[j];
  double ek;
  if (kind == KIND_SOFT) ek = phi;
  else if (kind == KIND_CONTACT) ek = k == 0 ? phi / (double)dt : 0.0;
  else ek = (double)m.baumgarte * phi / (double)dt;
  e[t.if_row[j] + k] = (T)ek;
}

// Construction of subsystem i by the whole workgroup: A_i = (2/t) M_i,
// b_i = (2/t) M_i v - C v + f (Eq. (2) solved for the midpoint velocity; C v =
// (0, omega x I omega) at the start of the step, f = (m g, 0)), the slot rows J_c,i, and e_j
// for interfaces whose first member is this subsystem.
// Out-of-line copies of the link code for the multi-step kernel, where inlining it (never
// executed on scenes without links) costs the iteration registers.
template <typename T>
__device__ __attribute__((noinline)) void rigid_link_row_outlined(const Topo& t, const RigidModel<T>& m, const int q,
                                                                  const int j, const int mem, const int k,
                                                                  const T* pos, const T* rot, const T dt, T* row,
                                                                  T* e) {
  rigid_link_row<T, true>(t, m, q, j, mem, k, pos, rot, dt, row, e);
}

template <typename T>
__device__ __attribute__((noinline)) void rigid_fold_links_outlined(const Topo& t, const RigidModel<T>& m, const int i,
                                                                    const T* pos, const T* rot, T* Ai, T* bi) {
  rigid_fold_links<T, true>(t, m, i, pos, rot, Ai, bi);
}

// Mass terms of body k (Eq. 2): its diagonal of A_i and its entries of b_i.
template <typename T>
__device__ __attribute__((always_inline)) inline void rigid_body_terms(const RigidModel<T>& m, const int k, const int n,
                                                                       const T* vel, const T* omega, const T dt, T* Ai,
                                                                       T* bi) {
  const T two_dt = (T)2 / dt;
  const int c0 = 6 * m.body_local[k];
  const T mk = m.mass[k];
  const T* I = m.inertia + 3 * k;
  const T* wk = omega + 3 * k;
  T Iw[3] = {I[0] * wk[0], I[1] * wk[1], I[2] * wk[2]};
  T gy[3];
  cross(wk, Iw, gy);
  for (int c = 0; c < 3; ++c) {
    Ai[(c0 + c) * n + c0 + c] = two_dt * mk;
    Ai[(c0 + 3 + c) * n + c0 + 3 + c] = two_dt * I[c];
    bi[c0 + c] = two_dt * mk * vel[3 * k + c] + (c == 2 ? -mk * m.gravity : (T)0);
    bi[c0 + 3 + c] = two_dt * Iw[c] - gy[c];
  }
}

// Slot row loc of subsystem i (its row of J_c,i, zeroed before) and, for the interface's
// first member, the row's e.
template <typename T, bool kOutline = false>
__device__ __attribute__((always_inline)) inline void rigid_slot_row(const Topo& t, const RigidModel<T>& m, const int i,
                                                                     const int loc, const T* pos, const T* rot,
                                                                     const T dt, T* Ji, T* e) {
  const int n = t.sub_n[i];
  const int g = t.sub_slot[i] + loc;
  const int j = t.slot_if[g];
  const int mem = t.slot_mk[g] >> 3;
  const int k = t.slot_mk[g] & 7;
  const int src = m.if_src[j];
  T* row = Ji + (size_t)loc * n;
  if (src >= m.nj) {
    if constexpr (kOutline)
      rigid_link_row_outlined<T>(t, m, src - m.nj, j, mem, k, pos, rot, dt, row, e);
    else
      rigid_link_row<T>(t, m, src - m.nj, j, mem, k, pos, rot, dt, row, e);
  } else if (src >= 0) {
    // revolute joint
    const int q = src;
    const int ba = m.joint_body[2 * q], bb = m.joint_body[2 * q + 1];
    const T* Ra = rot + 9 * ba;
    const T* Rb = rot + 9 * bb;
    const T* F = m.joint_frame + 9 * q;
    T nv[3] = {(T)0, (T)0, (T)0};
    if (k >= 3) r_vec(Ra, F + 3 * (k - 2), nv);  // k = 3 -> u, k = 4 -> v
    T ra[6], rb[6];
    joint_row(Ra, m.joint_anchor + 6 * q, nv, k, ra);
    joint_row(Rb, m.joint_anchor + 6 * q + 3, nv, k, rb);
    if (t.if_nsub[j] == 1) {
      const int ca = 6 * m.body_local[ba], cb = 6 * m.body_local[bb];
      for (int c = 0; c < 6; ++c) {
        row[ca + c] += ra[c];
        row[cb + c] -= rb[c];
      }
    } else if (mem == 0) {
      const int ca = 6 * m.body_local[ba];
      for (int c = 0; c < 6; ++c) row[ca + c] = ra[c];
    } else {
      const int cb = 6 * m.body_local[bb];
      for (int c = 0; c < 6; ++c) row[cb + c] = -rb[c];
    }
    if (mem == 0) {
      T val;
      if (k < 3) {
        // Anchor separation: a difference of two positions of similar size, formed in
        // FP64 from the stored state so that it carries no cancellation error.
        const T* aa = m.joint_anchor + 6 * q;
        const T* ab = aa + 3;
        double xa = (double)pos[3 * ba + k], xb = (double)pos[3 * bb + k];
        for (int c = 0; c < 3; ++c) {
          xa += (double)Ra[3 * k + c] * (double)aa[c];
          xb += (double)Rb[3 * k + c] * (double)ab[c];
        }
        val = (T)(xa - xb);
      } else {
        // axis misalignment n . (h_b x h_a): a small difference of unit vectors, also
        // formed in FP64
        double ha[3], hb[3], nn[3], c3[3];
        const T* hbb = m.joint_axis_b + 3 * q;
        const T* uv = F + 3 * (k - 2);
        for (int r = 0; r < 3; ++r) {
          ha[r] = hb[r] = nn[r] = 0.0;
          for (int c = 0; c < 3; ++c) {
            ha[r] += (double)Ra[3 * r + c] * (double)F[c];
            hb[r] += (double)Rb[3 * r + c] * (double)hbb[c];
            nn[r] += (double)Ra[3 * r + c] * (double)uv[c];
          }
        }
        cross(hb, ha, c3);
        val = (T)(nn[0] * c3[0] + nn[1] * c3[1] + nn[2] * c3[2]);
      }
      e[t.if_row[j] + k] = m.baumgarte * val / dt;
    }
  } else {
    // ground contact, rows (e_z, e_x, e_y)
    const int q = -1 - src;
    const int kb = m.contact_body[q];
    const T* R = rot + 9 * kb;
    const T* r = m.contact_point + 3 * q;
    const int axis = k == 0 ? 2 : k - 1;
    T d[3] = {(T)0, (T)0, (T)0};
    d[axis] = (T)1;
    T av[3], rr[3];
    rt_vec(R, d, av);
    cross(r, av, rr);
    const int c0 = 6 * m.body_local[kb];
    row[c0 + axis] = (T)1;
    row[c0 + 3] = rr[0];
    row[c0 + 4] = rr[1];
    row[c0 + 5] = rr[2];
    if (k == 0) {
      // gap above the plane, formed in FP64 like the joint separations
      const double gap = (double)pos[3 * kb + 2] + (double)R[6] * (double)r[0] + (double)R[7] * (double)r[1] +
                         (double)R[8] * (double)r[2];
      e[t.if_row[j]] = (T)(gap / (double)dt);
    } else {
      e[t.if_row[j] + k] = (T)0;
    }
  }
}

template <typename T, bool kOutline = false>
__device__ __attribute__((always_inline)) inline void rigid_assemble_sub(const Topo& t, const RigidModel<T>& m, const int i, const T* pos,
                                          const T* rot, const T* vel, const T* omega, const T dt, T* A, T* b,
                                          T* J, T* e) {
  const int tid = threadIdx.x, bd = blockDim.x;
  const int n = t.sub_n[i], nc = t.sub_nc[i];
  T* Ai = A + t.sub_A[i];
  T* Ji = J + t.sub_J[i];
  T* bi = b + t.sub_dof[i];
  for (int q = tid; q < n * n; q += bd) Ai[q] = (T)0;
  for (int q = tid; q < nc * n; q += bd) Ji[q] = (T)0;
  __syncthreads();
  for (int q = m.sub_body_off[i] + tid; q < m.sub_body_off[i + 1]; q += bd)
    rigid_body_terms<T>(m, m.sub_body[q], n, vel, omega, dt, Ai, bi);
  if constexpr (kOutline) {
    if (m.sub_ilink_off[i + 1] > m.sub_ilink_off[i]) rigid_fold_links_outlined<T>(t, m, i, pos, rot, Ai, bi);
  } else {
    rigid_fold_links<T>(t, m, i, pos, rot, Ai, bi);
  }
  for (int loc = tid; loc < nc; loc += bd) rigid_slot_row<T, kOutline>(t, m, i, loc, pos, rot, dt, Ji, e);
}

// Construction of all subsystems sb..se-1 of one scene by the workgroup at once (their A,
// J blocks and bodies are contiguous): the entries of rigid_assemble_sub, with the scene's
// bodies and slot rows spread over the threads instead of one subsystem after another.
template <typename T, bool kOutline = false>
__device__ __attribute__((always_inline)) inline void rigid_assemble_scene(const Topo& t, const RigidModel<T>& m,
                                                                           const int sb, const int se, const T* pos,
                                                                           const T* rot, const T* vel, const T* omega,
                                                                           const T dt, T* A, T* b, T* J, T* e) {
  const int tid = threadIdx.x, bd = blockDim.x;
  for (long long q = t.sub_A[sb] + tid; q < t.sub_A[se]; q += bd) A[q] = (T)0;
  for (long long q = t.sub_J[sb] + tid; q < t.sub_J[se]; q += bd) J[q] = (T)0;
  __syncthreads();
  for (int q = m.sub_body_off[sb] + tid; q < m.sub_body_off[se]; q += bd) {
    const int k = m.sub_body[q];
    const int i = m.body_sub[k];
    rigid_body_terms<T>(m, k, t.sub_n[i], vel, omega, dt, A + t.sub_A[i], b + t.sub_dof[i]);
  }
  if (m.sub_ilink_off[se] > m.sub_ilink_off[sb]) {
    for (int i = sb; i < se; ++i) {
      if constexpr (kOutline) {
        if (m.sub_ilink_off[i + 1] > m.sub_ilink_off[i])
          rigid_fold_links_outlined<T>(t, m, i, pos, rot, A + t.sub_A[i], b + t.sub_dof[i]);
      } else {
        rigid_fold_links<T>(t, m, i, pos, rot, A + t.sub_A[i], b + t.sub_dof[i]);
      }
    }
  }
  for (int g = t.sub_slot[sb] + tid; g < t.sub_slot[se]; g += bd) {
    const int i = t.slot_sub[g];
    rigid_slot_row<T, kOutline>(t, m, i, g - t.sub_slot[i], pos, rot, dt, J + t.sub_J[i], e);
  }
}

// exp([phi]x) by Rodrigues' formula, E = I + (sin th/th) X + ((1 - cos th)/th^2) X^2, with
// 1 - cos th written as 2 sin^2(th/2) (no cancellation) and Taylor coefficients for tiny
// angles.
template <typename T>
__device__ inline void so3_exp(const T* phi, T* E) {
  const T th2 = phi[0] * phi[0] + phi[1] * phi[1] + phi[2] * phi[2];
  T s, c;
  if (th2 < (T)1e-8) {
    s = (T)1 - th2 / (T)6;
    c = (T)0.5 - th2 / (T)24;
  } else {
    const T th = sqrt(th2);
    const T hs = sin((T)0.5 * th) / th;
    s = sin(th) / th;
    c = (T)2 * hs * hs;
  }
  const T X[9] = {(T)0, -phi[2], phi[1], phi[2], (T)0, -phi[0], -phi[1], phi[0], (T)0};
  for (int r = 0; r < 3; ++r)
    for (int q = 0; q < 3; ++q) {
      T x2 = X[r * 3 + 0] * X[0 * 3 + q] + X[r * 3 + 1] * X[1 * 3 + q] + X[r * 3 + 2] * X[2 * 3 + q];
      E[r * 3 + q] = (r == q ? (T)1 : (T)0) + s * X[r * 3 + q] + c * x2;
    }
}

// State update of Eq. (2) for body k.
template <typename T>
__device__ __attribute__((always_inline)) inline void rigid_advance_body(const Topo& t, const RigidModel<T>& m, const RigidState<T>& st,
                                          const T* v_hat, const T dt, const int k) {
  const T* vh = v_hat + t.sub_dof[m.body_sub[k]] + 6 * m.body_local[k];
  T phi[3], E[9], R[9], Rn[9];
  for (int c = 0; c < 3; ++c) {
    st.vel[3 * k + c] = (T)2 * vh[c] - st.vel[3 * k + c];
    st.omega[3 * k + c] = (T)2 * vh[3 + c] - st.omega[3 * k + c];
    st.pos[3 * k + c] += dt * vh[c];
    phi[c] = dt * vh[3 + c];
  }
  so3_exp(phi, E);
  for (int q = 0; q < 9; ++q) R[q] = st.rot[9 * k + q];
  for (int r = 0; r < 3; ++r)
    for (int q = 0; q < 3; ++q) Rn[r * 3 + q] = R[r * 3] * E[q] + R[r * 3 + 1] * E[3 + q] + R[r * 3 + 2] * E[6 + q];
  for (int q = 0; q < 9; ++q) st.rot[9 * k + q] = Rn[q];
}

}  // namespace subadmm
