/* FP64 oracle: per-step assembly of co-rotated linear-tetrahedron elastic blocks and
 * their state update.  TEST INFRASTRUCTURE ONLY (see oracle/__init__.py).
 *
 * Eq. (2) with the elastic potential psi of the blocks (Sec. II, soft constraints folded
 * into A_i, b_i as the remark after Eq. (6) allows):
 *   (2/t) M (v_hat - v) + d psi(x + (t/2) v_hat)^T = f + J^T lambda
 * and d psi linearised about x: d psi(x + (t/2) v_hat) ~ d psi(x) + (t/2) K(x) v_hat, so
 *   A = (2/t) M + (t/2) K,    b = (2/t) M v - d psi(x)^T + M g.
 * M is the lumped mass (density x volume / 4 to each vertex of a tetrahedron).
 *
 * Co-rotated linear elasticity per tetrahedron e with rest edge matrix D_m and current
 * D_s: F = D_s D_m^-1, R = orthogonal polar factor of F (Newton iteration
 * R <- (R + R^-T) / 2 from R = F, Higham's method), shape-function gradients g_1..g_3 =
 * rows of D_m^-1, g_0 = -(g_1 + g_2 + g_3), volume V.  The rest stiffness block of
 * vertices (a, b) is the Hessian of V (mu |eps|^2 + lambda/2 tr(eps)^2) for the small
 * strain eps:
 *   K0_ab = V (lambda g_a g_b^T + mu g_b g_a^T + mu (g_a . g_b) I)
 * with the Lame constants of (E, nu); co-rotated: K_ab = R K0_ab R^T and the elastic
 * force on vertex a is -sum_b R K0_ab (R^T x_b - X_b).
 *
 * Interfaces: a nodal equality between member nodes p (member 0) and q (member 1),
 * x_p = x_q, has rows +I on p's DOFs and -I on q's, error e = gamma (x_p - x_q) / t
 * (Baumgarte); a ground contact of node p (plane z = 0, normal +z) has rows
 * (e_z, e_x, e_y) on p's DOFs and error e = (z_p / t, 0, 0).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#include "subadmm_oracle.h"

enum { K_EQUALITY = 0, K_CONTACT = 1 };

static double det3(const double* m) {
  return m[0] * (m[4] * m[8] - m[5] * m[7]) - m[1] * (m[3] * m[8] - m[5] * m[6]) + m[2] * (m[3] * m[7] - m[4] * m[6]);
}

static int inv3(const double* m, double* out) {
  double d = det3(m);
  if (d == 0.0 || !isfinite(d)) return -1;
  out[0] = (m[4] * m[8] - m[5] * m[7]) / d;
  out[1] = (m[2] * m[7] - m[1] * m[8]) / d;
  out[2] = (m[1] * m[5] - m[2] * m[4]) / d;
  out[3] = (m[5] * m[6] - m[3] * m[8]) / d;
  out[4] = (m[0] * m[8] - m[2] * m[6]) / d;
  out[5] = (m[2] * m[3] - m[0] * m[5]) / d;
  out[6] = (m[3] * m[7] - m[4] * m[6]) / d;
  out[7] = (m[1] * m[6] - m[0] * m[7]) / d;
  out[8] = (m[0] * m[4] - m[1] * m[3]) / d;
  return 0;
}

static void matmul3(const double* a, const double* b, double* out) {
  for (int r = 0; r < 3; ++r)
    for (int c = 0; c < 3; ++c) out[r * 3 + c] = a[r * 3 + 0] * b[0 * 3 + c] + a[r * 3 + 1] * b[1 * 3 + c] + a[r * 3 + 2] * b[2 * 3 + c];
}

/* Orthogonal polar factor by Newton's iteration R <- (R + R^-T) / 2. */
int oracle_polar(const double* F, double* R) {
  double X[9], Xi[9];
  memcpy(X, F, sizeof(X));
  for (int it = 0; it < 100; ++it) {
    if (inv3(X, Xi) != 0) return -1;
    double N[9], diff = 0.0, nrm = 0.0;
    for (int r = 0; r < 3; ++r)
      for (int c = 0; c < 3; ++c) {
        N[r * 3 + c] = 0.5 * (X[r * 3 + c] + Xi[c * 3 + r]);
        double d = N[r * 3 + c] - X[r * 3 + c];
        diff += d * d;
        nrm += N[r * 3 + c] * N[r * 3 + c];
      }
    memcpy(X, N, sizeof(X));
    if (diff <= 1e-30 * nrm) break;
  }
  memcpy(R, X, sizeof(X));
  return 0;
}

/* Rest data of one tetrahedron: gradients g (4x3, rows) and volume. */
static int tet_rest(const double* X0, const double* X1, const double* X2, const double* X3, double* g, double* vol) {
  double Dm[9], Dmi[9];
  for (int r = 0; r < 3; ++r) {
    Dm[r * 3 + 0] = X1[r] - X0[r];
    Dm[r * 3 + 1] = X2[r] - X0[r];
    Dm[r * 3 + 2] = X3[r] - X0[r];
  }
  double d = det3(Dm);
  if (!(d > 0.0)) return -1;
  *vol = d / 6.0;
  if (inv3(Dm, Dmi) != 0) return -1;
  for (int a = 1; a < 4; ++a)
    for (int c = 0; c < 3; ++c) g[a * 3 + c] = Dmi[(a - 1) * 3 + c];
  for (int c = 0; c < 3; ++c) g[c] = -(g[3 + c] + g[6 + c] + g[9 + c]);
  return 0;
}

/* K0_ab (3x3, row-major) of the rest configuration. */
static void k0_block(const double* ga, const double* gb, double vol, double lam, double mu, double* K) {
  double dot = ga[0] * gb[0] + ga[1] * gb[1] + ga[2] * gb[2];
  for (int r = 0; r < 3; ++r)
    for (int c = 0; c < 3; ++c)
      K[r * 3 + c] = vol * (lam * ga[r] * gb[c] + mu * gb[r] * ga[c] + (r == c ? mu * dot : 0.0));
}

int oracle_fem_element(const double* X, const double* x, double young, double poisson, double* K, double* f) {
  /* X, x: 4x3 rest and current vertex positions; K: 12x12 co-rotated stiffness;
     f: 12 elastic forces. */
  double g[12], vol;
  if (tet_rest(X, X + 3, X + 6, X + 9, g, &vol) != 0) return -1;
  double lam = young * poisson / ((1.0 + poisson) * (1.0 - 2.0 * poisson));
  double mu = young / (2.0 * (1.0 + poisson));
  double Ds[9], Dm[9], Dmi[9], F[9], R[9];
  for (int r = 0; r < 3; ++r)
    for (int a = 1; a < 4; ++a) {
      Ds[r * 3 + a - 1] = x[a * 3 + r] - x[r];
      Dm[r * 3 + a - 1] = X[a * 3 + r] - X[r];
    }
  if (inv3(Dm, Dmi) != 0) return -1;
  matmul3(Ds, Dmi, F);
  if (oracle_polar(F, R) != 0) return -1;
  /* unrotated displacement R^T x_b - X_b */
  double du[12];
  for (int b = 0; b < 4; ++b)
    for (int c = 0; c < 3; ++c)
      du[b * 3 + c] = R[0 * 3 + c] * x[b * 3 + 0] + R[1 * 3 + c] * x[b * 3 + 1] + R[2 * 3 + c] * x[b * 3 + 2] - X[b * 3 + c];
  for (int i = 0; i < 12; ++i) f[i] = 0.0;
  for (int a = 0; a < 4; ++a)
    for (int b = 0; b < 4; ++b) {
      double K0[9], T[9], Kab[9];
      k0_block(g + 3 * a, g + 3 * b, vol, lam, mu, K0);
      /* Kab = R K0 R^T */
      matmul3(R, K0, T);
      for (int r = 0; r < 3; ++r)
        for (int c = 0; c < 3; ++c)
          Kab[r * 3 + c] = T[r * 3 + 0] * R[c * 3 + 0] + T[r * 3 + 1] * R[c * 3 + 1] + T[r * 3 + 2] * R[c * 3 + 2];
      for (int r = 0; r < 3; ++r)
        for (int c = 0; c < 3; ++c) K[(3 * a + r) * 12 + 3 * b + c] = Kab[r * 3 + c];
      /* f_a -= R K0 du_b */
      double k0du[3];
      for (int r = 0; r < 3; ++r) k0du[r] = K0[r * 3 + 0] * du[b * 3 + 0] + K0[r * 3 + 1] * du[b * 3 + 1] + K0[r * 3 + 2] * du[b * 3 + 2];
      for (int r = 0; r < 3; ++r) f[3 * a + r] -= R[r * 3 + 0] * k0du[0] + R[r * 3 + 1] * k0du[1] + R[r * 3 + 2] * k0du[2];
    }
  return 0;
}

int oracle_fem_assemble(int32_t n_sub, const int32_t* sub_nodes, int32_t n_tets, const int32_t* tets,
                        const int32_t* tet_sub, const double* rest, const double* pos, const double* vel,
                        const double* young, const double* poisson, double density, int32_t n_if,
                        const int32_t* if_kind, const int32_t* if_dim, const int32_t* if_nsub,
                        const int32_t* if_sub, const int32_t* if_node, double dt, double gravity, double baumgarte,
                        double* A, double* b, double* J, double* e) {
  if (n_sub <= 0 || !(dt > 0.0)) return -1;
  int64_t* node_off = malloc(sizeof(int64_t) * (size_t)(n_sub + 1));
  int64_t* A_off = malloc(sizeof(int64_t) * (size_t)(n_sub + 1));
  int64_t* J_off = malloc(sizeof(int64_t) * (size_t)(n_sub + 1));
  int64_t* nc = calloc((size_t)n_sub, sizeof(int64_t));
  int64_t* loc = malloc(sizeof(int64_t) * (size_t)(2 * (n_if > 0 ? n_if : 1)));
  double* mass = NULL;
  int rc = 0;
  if (!node_off || !A_off || !J_off || !nc || !loc) { rc = -1; goto done; }
  node_off[0] = A_off[0] = 0;
  for (int32_t i = 0; i < n_sub; ++i) {
    node_off[i + 1] = node_off[i] + sub_nodes[i];
    int64_t n = 3 * (int64_t)sub_nodes[i];
    A_off[i + 1] = A_off[i] + n * n;
  }
  /* slot layout: per subsystem, its interfaces in ascending order */
  for (int32_t j = 0; j < n_if; ++j)
    for (int m = 0; m < if_nsub[j]; ++m) {
      int32_t i = if_sub[2 * j + m];
      loc[2 * j + m] = nc[i];
      nc[i] += if_dim[j];
    }
  J_off[0] = 0;
  for (int32_t i = 0; i < n_sub; ++i) J_off[i + 1] = J_off[i] + nc[i] * 3 * (int64_t)sub_nodes[i];
  int64_t nn = node_off[n_sub];
  mass = calloc((size_t)nn, sizeof(double));
  if (!mass) { rc = -1; goto done; }
  memset(A, 0, sizeof(double) * (size_t)A_off[n_sub]);
  memset(J, 0, sizeof(double) * (size_t)(J_off[n_sub] > 0 ? J_off[n_sub] : 0));
  for (int64_t k = 0; k < 3 * nn; ++k) b[k] = 0.0;

  for (int32_t t = 0; t < n_tets; ++t) {
    const int32_t i = tet_sub[t];
    const int32_t* v = tets + 4 * t;
    double X[12], x[12], K[144], f[12], g[12], vol;
    for (int a = 0; a < 4; ++a)
      for (int c = 0; c < 3; ++c) {
        X[3 * a + c] = rest[3 * (int64_t)v[a] + c];
        x[3 * a + c] = pos[3 * (int64_t)v[a] + c];
      }
    if (tet_rest(X, X + 3, X + 6, X + 9, g, &vol) != 0) { rc = -2; goto done; }
    if (oracle_fem_element(X, x, young[i], poisson[i], K, f) != 0) { rc = -2; goto done; }
    const int64_t n = 3 * (int64_t)sub_nodes[i];
    double* Ai = A + A_off[i];
    for (int a = 0; a < 4; ++a) {
      mass[v[a]] += density * vol / 4.0;
      const int64_t ra = 3 * (v[a] - node_off[i]);
      for (int c = 0; c < 3; ++c) b[3 * (int64_t)v[a] + c] += f[3 * a + c];
      for (int bb = 0; bb < 4; ++bb) {
        const int64_t rb = 3 * (v[bb] - node_off[i]);
        for (int r = 0; r < 3; ++r)
          for (int c = 0; c < 3; ++c) Ai[(ra + r) * n + rb + c] += 0.5 * dt * K[(3 * a + r) * 12 + 3 * bb + c];
      }
    }
  }
  for (int32_t i = 0; i < n_sub; ++i) {
    const int64_t n = 3 * (int64_t)sub_nodes[i];
    double* Ai = A + A_off[i];
    for (int64_t p = node_off[i]; p < node_off[i + 1]; ++p) {
      const int64_t r0 = 3 * (p - node_off[i]);
      for (int c = 0; c < 3; ++c) {
        Ai[(r0 + c) * n + r0 + c] += 2.0 / dt * mass[p];
        b[3 * p + c] += 2.0 / dt * mass[p] * vel[3 * p + c];
      }
      b[3 * p + 2] -= mass[p] * gravity;
    }
  }
  /* interface rows */
  int64_t eo = 0;
  for (int32_t j = 0; j < n_if; ++j) {
    for (int m = 0; m < if_nsub[j]; ++m) {
      const int32_t i = if_sub[2 * j + m];
      const int64_t n = 3 * (int64_t)sub_nodes[i];
      const int64_t col = 3 * ((int64_t)if_node[2 * j + m] - node_off[i]);
      double* Ji = J + J_off[i] + loc[2 * j + m] * n;
      if (if_kind[j] == K_CONTACT) {
        Ji[0 * n + col + 2] = 1.0;  /* normal e_z */
        Ji[1 * n + col + 0] = 1.0;  /* tangent e_x */
        Ji[2 * n + col + 1] = 1.0;  /* tangent e_y */
      } else {
        const double sgn = m == 0 ? 1.0 : -1.0;
        for (int c = 0; c < 3; ++c) Ji[c * n + col + c] = sgn;
      }
    }
    const int64_t p = if_node[2 * j];
    if (if_kind[j] == K_CONTACT) {
      e[eo + 0] = pos[3 * p + 2] / dt;
      e[eo + 1] = 0.0;
      e[eo + 2] = 0.0;
    } else {
      const int64_t q = if_node[2 * j + 1];
      for (int c = 0; c < 3; ++c) e[eo + c] = baumgarte * (pos[3 * p + c] - pos[3 * q + c]) / dt;
    }
    eo += if_dim[j];
  }
done:
  free(node_off); free(A_off); free(J_off); free(nc); free(loc); free(mass);
  return rc;
}

int oracle_fem_advance(int64_t n_nodes, const double* v_hat, double dt, const double* pos, const double* vel,
                       double* pos_out, double* vel_out) {
  /* Eq. (2): v+ = 2 v_hat - v, x+ = x + t v_hat. */
  for (int64_t k = 0; k < 3 * n_nodes; ++k) {
    pos_out[k] = pos[k] + dt * v_hat[k];
    vel_out[k] = 2.0 * v_hat[k] - vel[k];
  }
  return 0;
}
