/*
 * FP64 CPU oracle for the per-step subsystem-based ADMM solve (arXiv 2302.14344).
 *
 * TEST INFRASTRUCTURE ONLY: the independent reference the HIP path is checked against.
 * Only the test suite, the smoke check and the benchmark's CPU-baseline leg use it.
 *
 * The code follows the paper's equations in their own order and notation, keeping the
 * ADMM variables x, z, u explicit, in plain loops with no blocking or fusion:
 *   Eq. (2)   midpoint-rule discrete dynamics, A_i = (2/t) M_i, b_i = (2/t) M_i v - C v + f
 *   Eq. (15)  x-update: (A_i + beta_i J_c,i^T J_c,i) v_hat_i = b_i + J_c,i^T (beta_i z_i - u_i)
 *   Eq. (18)  y_i,j = beta_i x_i,j + u_i,j ;  beta_i z_i,j = y_i,j + lambda_j
 *   Eq. (19)/(21)  lambda_j = Pi(-(sum_i y_i,j / beta_i + e_j) / sum_i 1/beta_i)
 *   Eq. (14)  u_i <- u_i + beta_i (x_i - z_i)
 *   Eq. (22)  theta = sum_i || y_i^{l+1} - y_i^l ||^2
 *   Eq. (23)  beta_i = Tr(A_i) / Tr(J_c,i^T J_c,i)
 * Readings of points the paper leaves open are stated where they are used.
 */
#include "subadmm_oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

enum { K_EQUALITY = 0, K_CONTACT = 1, K_HARD_INEQ = 2, K_SOFT = 3 };

/* Members an interface may have in the solve (|S_j| <= MEMB, Sec. III-B: S_j is the set of
 * subsystems a constraint touches; one for intra-subsystem rows, two or more for couplings).
 * The solve entry points take MEMB member entries per interface; the rigid and FEM
 * constructions, whose interfaces have one or two members, take two. */
#define MEMB 4

/* ------------------------------------------------------------------------------------ */
/* Layout bookkeeping (slot rows, offsets)                                               */
/* ------------------------------------------------------------------------------------ */

typedef struct {
  int32_t n_sub, n_if;
  int64_t *dof_off, *A_off, *J_off, *slot_off, *nc; /* per subsystem (n_sub+1 for offsets) */
  int64_t *e_off;                                   /* per interface (n_if+1) */
  int64_t *if_slot;                                 /* per interface, MEMB entries: first slot row of member m */
} layout_t;

static void layout_free(layout_t* L) {
  free(L->dof_off); free(L->A_off); free(L->J_off); free(L->slot_off); free(L->nc);
  free(L->e_off); free(L->if_slot);
}

/* if_sub holds `stride` entries per interface (members 0..if_nsub-1 used). */
static int layout_build(layout_t* L, int32_t n_sub, const int32_t* sub_ndof, int32_t n_if,
                        const int32_t* if_dim, const int32_t* if_nsub, const int32_t* if_sub, int stride) {
  L->n_sub = n_sub; L->n_if = n_if;
  L->dof_off = calloc((size_t)n_sub + 1, sizeof(int64_t));
  L->A_off = calloc((size_t)n_sub + 1, sizeof(int64_t));
  L->J_off = calloc((size_t)n_sub + 1, sizeof(int64_t));
  L->slot_off = calloc((size_t)n_sub + 1, sizeof(int64_t));
  L->nc = calloc((size_t)n_sub + 1, sizeof(int64_t));
  L->e_off = calloc((size_t)n_if + 1, sizeof(int64_t));
  L->if_slot = calloc(MEMB * (size_t)n_if + MEMB, sizeof(int64_t));
  if (!L->dof_off || !L->A_off || !L->J_off || !L->slot_off || !L->nc || !L->e_off || !L->if_slot)
    return -1;
  for (int32_t j = 0; j < n_if; ++j) {
    if (if_dim[j] <= 0 || if_nsub[j] < 1 || if_nsub[j] > stride || stride > MEMB) return -1;
    for (int m = 0; m < if_nsub[j]; ++m) {
      int32_t i = if_sub[stride * j + m];
      if (i < 0 || i >= n_sub) return -1;
      for (int q = 0; q < m; ++q)
        if (if_sub[stride * j + q] == i) return -1; /* members are distinct subsystems */
      L->nc[i] += if_dim[j];
    }
    L->e_off[j + 1] = L->e_off[j] + if_dim[j];
  }
  for (int32_t i = 0; i < n_sub; ++i) {
    if (sub_ndof[i] <= 0) return -1;
    L->dof_off[i + 1] = L->dof_off[i] + sub_ndof[i];
    L->A_off[i + 1] = L->A_off[i] + (int64_t)sub_ndof[i] * sub_ndof[i];
    L->J_off[i + 1] = L->J_off[i] + L->nc[i] * sub_ndof[i];
    L->slot_off[i + 1] = L->slot_off[i] + L->nc[i];
  }
  /* slot rows of subsystem i: interfaces in ascending order, rows 0..d_j-1 */
  int64_t* cursor = calloc((size_t)n_sub + 1, sizeof(int64_t));
  if (!cursor) return -1;
  for (int32_t i = 0; i < n_sub; ++i) cursor[i] = L->slot_off[i];
  for (int32_t j = 0; j < n_if; ++j)
    for (int m = 0; m < if_nsub[j]; ++m) {
      int32_t i = if_sub[stride * j + m];
      L->if_slot[MEMB * j + m] = cursor[i];
      cursor[i] += if_dim[j];
    }
  free(cursor);
  return 0;
}

/* ------------------------------------------------------------------------------------ */
/* Dense SPD factorisation (textbook Cholesky-Banachiewicz) and triangular solves         */
/* ------------------------------------------------------------------------------------ */

/* K (n x n, row-major) is overwritten by its lower Cholesky factor L, K = L L^T. */
static int cholesky(double* K, int n) {
  for (int r = 0; r < n; ++r) {
    for (int c = 0; c <= r; ++c) {
      double s = K[r * n + c];
      for (int k = 0; k < c; ++k) s -= K[r * n + k] * K[c * n + k];
      if (r == c) {
        if (!(s > 0.0)) return -2;
        K[r * n + r] = sqrt(s);
      } else {
        K[r * n + c] = s / K[c * n + c];
      }
    }
  }
  return 0;
}

/* Solve L L^T x = rhs in place. */
static void chol_solve(const double* L, int n, double* x) {
  for (int r = 0; r < n; ++r) {
    double s = x[r];
    for (int k = 0; k < r; ++k) s -= L[r * n + k] * x[k];
    x[r] = s / L[r * n + r];
  }
  for (int r = n - 1; r >= 0; --r) {
    double s = x[r];
    for (int k = r + 1; k < n; ++k) s -= L[k * n + r] * x[k];
    x[r] = s / L[r * n + r];
  }
}

/* ------------------------------------------------------------------------------------ */
/* z-subproblem projections, Eq. (16)-(21)                                               */
/* ------------------------------------------------------------------------------------ */

/* With the matrix-free relation beta_i z_i,j = y_i,j + lambda_j of Eq. (18), the value
 * of the constraint is sum_i z_i,j + e_j = s + w lambda with s = sum_i y_i,j/beta_i + e_j
 * and the scalar w = sum_i 1/beta_i.  Write p = -s/w, so the constraint value is
 * w (lambda - p).
 *
 * Contact, Eq. (21), with rows (n, t1, t2): the normal pair is the complementarity
 * 0 <= lambda_n  _|_  w (lambda_n - p_n) >= 0, solved by lambda_n = max(0, p_n).  The
 * tangential value is w (lambda_t - p_t).  Stick (zero tangential value) gives
 * lambda_t = p_t, admissible while |p_t| <= mu lambda_n.  Slip requires
 * |lambda_t| = mu lambda_n with lambda_t opposite to w (lambda_t - p_t), i.e. parallel to
 * p_t: lambda_t = mu lambda_n p_t/|p_t|.  Because the metric is a scalar multiple of the
 * identity the normal and tangential conditions decouple and this is the exact
 * Signorini-Coulomb solution (not the Euclidean second-order-cone projection, which
 * belongs to the relaxed convex model).  Ties: p_n <= 0 -> open (lambda = 0);
 * |p_t| <= mu lambda_n -> stick; |p_t| = 0 -> lambda_t = 0. */
/* Relaxed convex contact model (the convexification named in the paper's convergence
 * discussion): the Euclidean projection of p onto the friction cone
 * K = {lambda : |lambda_t| <= mu lambda_n}.  Inside K it is p itself; in the polar cone
 * {q : mu |q_t| <= -q_n} it is 0; otherwise it is the nearest point on the boundary ray
 * through p_t's direction, found by projecting (p_n, |p_t|) onto the line (1, mu). */
static void project_cone(const double* p, double mu, double* lam) {
  double tn = sqrt(p[1] * p[1] + p[2] * p[2]);
  if (tn <= mu * p[0]) {
    lam[0] = p[0]; lam[1] = p[1]; lam[2] = p[2];
  } else if (mu * tn <= -p[0]) {
    lam[0] = 0.0; lam[1] = 0.0; lam[2] = 0.0;
  } else {
    double ln = (p[0] + mu * tn) / (1.0 + mu * mu);
    lam[0] = ln;
    lam[1] = mu * ln * p[1] / tn;
    lam[2] = mu * ln * p[2] / tn;
  }
}

static void project_contact(const double* p, double mu, double* lam) {
  double ln = p[0] > 0.0 ? p[0] : 0.0;
  double pt1 = p[1], pt2 = p[2];
  double tn = sqrt(pt1 * pt1 + pt2 * pt2);
  double cap = mu * ln;
  lam[0] = ln;
  if (tn <= cap) {
    lam[1] = pt1;
    lam[2] = pt2;
  } else {
    lam[1] = cap * pt1 / tn;
    lam[2] = cap * pt2 / tn;
  }
}

/* ------------------------------------------------------------------------------------ */
/* Algorithm 1 on one scene                                                              */
/* ------------------------------------------------------------------------------------ */

typedef struct {
  const int32_t *sub_ndof, *if_kind, *if_dim, *if_nsub, *if_sub;
  const double *if_mu, *A, *b, *J, *e, *z0, *u0;
  double rho, tol;
  int32_t max_iters;
  int32_t contact_model; /* 0: exact Signorini-Coulomb, 1: relaxed convex (Euclidean cone) */
  const double *if_k, *if_alpha; /* soft constraints, Eq. (3): gain k_j and alpha_j */
  double *v_hat, *lambda, *z, *u, *beta;
  double *x, *y, *yprev; /* per slot row, scenes touch disjoint ranges */
  double *zb, *lb;       /* per slot row / per row: the residual pair's z- and lambda-update */
  const layout_t* L;
} solve_args_t;

/* z-update, Eq. (16)-(21), of the interfaces ifs[0..ni) from the slot vector y: lambda_j
 * (row layout) and the members' z (Eq. 18: beta_i z_i,j = y_i,j + lambda_j). */
static void z_update(const solve_args_t* S, const int32_t* ifs, int32_t ni, const double* y, double* z,
                     double* lambda) {
  const layout_t* L = S->L;
  for (int32_t c = 0; c < ni; ++c) {
    int32_t j = ifs[c];
    int d = S->if_dim[j];
    int ms = S->if_nsub[j];
    double w = 0.0;
    for (int m = 0; m < ms; ++m) w += 1.0 / S->beta[S->if_sub[MEMB * j + m]];
    double p[8], lam[8];
    for (int k = 0; k < d; ++k) {
      double s = S->e[L->e_off[j] + k];
      for (int m = 0; m < ms; ++m) s += y[L->if_slot[MEMB * j + m] + k] / S->beta[S->if_sub[MEMB * j + m]];
      p[k] = -s / w;
    }
    if (S->if_kind[j] == K_SOFT) {
      /* Eq. (3) with the sum of the members' z from Eq. (16) substituted (Eq. 20):
       * lambda = -k (e + alpha sum_i y_i / beta_i) / (1 + w alpha k) */
      double kj = S->if_k[j], aj = S->if_alpha[j];
      for (int k = 0; k < d; ++k) {
        double sy = 0.0;
        for (int m = 0; m < ms; ++m) sy += y[L->if_slot[MEMB * j + m] + k] / S->beta[S->if_sub[MEMB * j + m]];
        lam[k] = -kj * (S->e[L->e_off[j] + k] + aj * sy) / (1.0 + w * aj * kj);
      }
    } else if (S->if_kind[j] == K_CONTACT) {
      if (S->contact_model == 1) project_cone(p, S->if_mu[j], lam);
      else project_contact(p, S->if_mu[j], lam);
    } else if (S->if_kind[j] == K_HARD_INEQ) {
      for (int k = 0; k < d; ++k) lam[k] = p[k] > 0.0 ? p[k] : 0.0;  /* Eq. (19) */
    } else {
      for (int k = 0; k < d; ++k) lam[k] = p[k];  /* equality: lambda free */
    }
    for (int k = 0; k < d; ++k) {
      lambda[L->e_off[j] + k] = lam[k];
      for (int m = 0; m < ms; ++m) {
        int32_t i = S->if_sub[MEMB * j + m];
        int64_t s = L->if_slot[MEMB * j + m] + k;
        z[s] = (y[s] + lam[k]) / S->beta[i];  /* Eq. (18) */
      }
    }
  }
}

static int solve_scene(const solve_args_t* S, int32_t max_iters, const int32_t* subs, int32_t ns,
                       const int32_t* ifs, int32_t ni, int32_t* iters_out,
                       int32_t* conv_out, double* theta_out, double* r_theta_out, double* r_prim_out,
                       double* r_dual_out) {
  const layout_t* L = S->L;
  int rc = 0;
  /* scene-local scratch: factors, rhs, x, y_prev */
  int64_t kfac = 0, nslot = 0, nmax = 0;
  for (int32_t a = 0; a < ns; ++a) {
    int32_t i = subs[a];
    kfac += (int64_t)S->sub_ndof[i] * S->sub_ndof[i];
    nslot += L->nc[i];
    if (S->sub_ndof[i] > nmax) nmax = S->sub_ndof[i];
  }
  double* K = malloc(sizeof(double) * (size_t)(kfac > 0 ? kfac : 1));
  int64_t* koff = malloc(sizeof(int64_t) * (size_t)(ns + 1));
  double* x = S->x;
  double* yprev = S->yprev;
  double* y = S->y;
  /* one right-hand side per subsystem, so that large scenes can spread their
     subsystems over threads (the arithmetic of each subsystem is unchanged) */
  double* rhs_all = malloc(sizeof(double) * (size_t)ns * (size_t)(nmax + 1));
  int* frc = calloc((size_t)ns + 1, sizeof(int));
  (void)nslot;
  if (!K || !koff || !rhs_all || !frc) { rc = -1; goto done; }
  const int par = ns >= 16 && !omp_in_parallel();

  /* Alg. 1: factorise A_i + beta_i J_c,i^T J_c,i once per step. */
  koff[0] = 0;
  for (int32_t a = 0; a < ns; ++a) koff[a + 1] = koff[a] + (int64_t)S->sub_ndof[subs[a]] * S->sub_ndof[subs[a]];
#pragma omp parallel for schedule(dynamic) if (par)
  for (int32_t a = 0; a < ns; ++a) {
    int32_t i = subs[a];
    int n = S->sub_ndof[i];
    int64_t nc = L->nc[i];
    const double* Ai = S->A + L->A_off[i];
    const double* Ji = S->J + L->J_off[i];
    double trA = 0.0, trJJ = 0.0;
    for (int r = 0; r < n; ++r) trA += Ai[r * n + r];
    for (int64_t k = 0; k < nc * n; ++k) trJJ += Ji[k] * Ji[k];
    /* Eq. (23); rho > 0 overrides with a uniform weight.  A subsystem with no slot
       rows has no augmented term and beta only has to be a positive placeholder. */
    double be;
    if (S->rho > 0.0) be = S->rho;
    else be = trJJ > 0.0 ? trA / trJJ : 1.0;
    S->beta[i] = be;
    double* Ki = K + koff[a];
    for (int r = 0; r < n; ++r)
      for (int c = 0; c < n; ++c) {
        double jj = 0.0;
        for (int64_t k = 0; k < nc; ++k) jj += Ji[k * n + r] * Ji[k * n + c];
        Ki[r * n + c] = Ai[r * n + c] + be * jj;
      }
    if (cholesky(Ki, n) != 0) frc[a] = -2;
  }
  for (int32_t a = 0; a < ns; ++a)
    if (frc[a]) { rc = frc[a]; goto done; }

  /* Initial z^0, u^0 (zero unless given) and y^0 := beta z^0 + u^0 (the relation that
     holds after every z/u-update), used by the first residual. */
  for (int32_t a = 0; a < ns; ++a) {
    int32_t i = subs[a];
    for (int64_t s = L->slot_off[i]; s < L->slot_off[i + 1]; ++s) {
      S->z[s] = S->z0 ? S->z0[s] : 0.0;
      S->u[s] = S->u0 ? S->u0[s] : 0.0;
      yprev[s] = S->beta[i] * S->z[s] + S->u[s];
    }
  }
  /* lambda before any z-update: the one implied by u = -lambda (zero when cold). */
  for (int32_t c = 0; c < ni; ++c) {
    int32_t j = ifs[c];
    for (int k = 0; k < S->if_dim[j]; ++k)
      S->lambda[L->e_off[j] + k] = -S->u[L->if_slot[MEMB * j] + k];
  }

  int32_t l = 0, conv = 0, it = 0;
  double th = 0.0, rth = 0.0;
  for (l = 0; l < max_iters; ++l) {
    it = l + 1;
    /* x-update, Eq. (15), every subsystem. */
#pragma omp parallel for schedule(dynamic) if (par)
    for (int32_t a = 0; a < ns; ++a) {
      int32_t i = subs[a];
      double* rhs = rhs_all + (size_t)a * (size_t)(nmax + 1);
      int n = S->sub_ndof[i];
      int64_t nc = L->nc[i];
      const double* Ji = S->J + L->J_off[i];
      const double* zi = S->z + L->slot_off[i];
      const double* ui = S->u + L->slot_off[i];
      double be = S->beta[i];
      for (int r = 0; r < n; ++r) {
        double s = S->b[L->dof_off[i] + r];
        for (int64_t k = 0; k < nc; ++k) s += Ji[k * n + r] * (be * zi[k] - ui[k]);
        rhs[r] = s;
      }
      chol_solve(K + koff[a], n, rhs);
      for (int r = 0; r < n; ++r) S->v_hat[L->dof_off[i] + r] = rhs[r];
      for (int64_t k = 0; k < nc; ++k) {
        double s = 0.0;
        for (int r = 0; r < n; ++r) s += Ji[k * n + r] * rhs[r];
        x[L->slot_off[i] + k] = s;
        y[L->slot_off[i] + k] = be * s + ui[k];  /* Eq. (18) */
      }
    }
    /* Residual, Eq. (22), and the relative form used as the stopping test:
       r_theta = sqrt(theta) / max(|y^{l+1}|, 1e-12). */
    double ss = 0.0, yy = 0.0;
    for (int32_t a = 0; a < ns; ++a) {
      int32_t i = subs[a];
      for (int64_t s = L->slot_off[i]; s < L->slot_off[i + 1]; ++s) {
        double d = y[s] - yprev[s];
        ss += d * d;
        yy += y[s] * y[s];
      }
    }
    th = ss;
    double yn = sqrt(yy);
    rth = sqrt(ss) / (yn > 1e-12 ? yn : 1e-12);
    if (rth <= S->tol) { conv = 1; break; }
    if (l + 1 == max_iters) break;

    /* z-update, Eq. (16)-(21), every interface. */
    z_update(S, ifs, ni, y, S->z, S->lambda);
    /* u-update, Eq. (14). */
    for (int32_t a = 0; a < ns; ++a) {
      int32_t i = subs[a];
      for (int64_t s = L->slot_off[i]; s < L->slot_off[i + 1]; ++s) {
        S->u[s] = S->u[s] + S->beta[i] * (x[s] - S->z[s]);
        yprev[s] = y[s];
      }
    }
  }
  *iters_out = it;
  *conv_out = conv;
  *theta_out = th;
  *r_theta_out = rth;
  /* Primal and dual residuals of the returned iterate, the stopping pair of ADMM in its
     standard form (Boyd et al. 2011, Sec. 3.3): the z-update (Eq. 16-21) and u-update
     (Eq. 14) that would follow the last x-update, taken aside (the outputs keep the z, u
     that x-update started from): r_prim = |x - z'| / max(|x|, |z'|) and
     r_dual = |beta (z' - z)| / |u'| over the scene's slot rows, each with r_theta's floor
     1e-12.  Reported beside r_theta; the stop stays on r_theta. */
  if (r_prim_out && r_dual_out) {
    z_update(S, ifs, ni, y, S->zb, S->lb);
    double pp = 0.0, xx = 0.0, zz = 0.0, dd = 0.0, uu = 0.0;
    for (int32_t a = 0; a < ns; ++a) {
      int32_t i = subs[a];
      double be = S->beta[i];
      for (int64_t s = L->slot_off[i]; s < L->slot_off[i + 1]; ++s) {
        double zn = S->zb[s];
        double un = S->u[s] + be * (x[s] - zn);
        double dz = be * (zn - S->z[s]);
        pp += (x[s] - zn) * (x[s] - zn);
        xx += x[s] * x[s];
        zz += zn * zn;
        dd += dz * dz;
        uu += un * un;
      }
    }
    double nx = sqrt(xx > zz ? xx : zz), nu = sqrt(uu);
    *r_prim_out = sqrt(pp) / (nx > 1e-12 ? nx : 1e-12);
    *r_dual_out = sqrt(dd) / (nu > 1e-12 ? nu : 1e-12);
  }
done:
  free(K); free(koff); free(rhs_all); free(frc);
  return rc;
}

int oracle_solve(int32_t n_sub, const int32_t* sub_ndof, const int32_t* sub_scene,
                 int32_t n_if, const int32_t* if_kind, const int32_t* if_dim,
                 const int32_t* if_nsub, const int32_t* if_sub, const double* if_mu,
                 const double* A, const double* b, const double* J, const double* e,
                 double rho, int32_t max_iters, double tol,
                 const double* z0, const double* u0,
                 double* v_hat, double* lambda, double* z, double* u, double* beta,
                 int32_t* iters, int32_t* converged, double* theta, double* r_theta,
                 int32_t n_threads) {
  return oracle_solve_model(n_sub, sub_ndof, sub_scene, n_if, if_kind, if_dim, if_nsub, if_sub, if_mu, A, b, J,
                            e, rho, max_iters, tol, z0, u0, v_hat, lambda, z, u, beta, iters, converged, theta,
                            r_theta, NULL, NULL, 0, NULL, NULL, NULL, n_threads);
}

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
                       const int32_t* scene_max_iters, int32_t n_threads) {
  if (n_sub <= 0 || n_if < 0 || max_iters < 1 || !(tol >= 0.0)) return -1;
  if (contact_model != 0 && contact_model != 1) return -1;
  for (int32_t j = 0; j < n_if; ++j)
    if (if_kind[j] == K_SOFT && (!if_k || !if_alpha || !(if_k[j] >= 0.0) || !(if_alpha[j] > 0.0))) return -1;
  layout_t L;
  memset(&L, 0, sizeof(L));
  if (layout_build(&L, n_sub, sub_ndof, n_if, if_dim, if_nsub, if_sub, MEMB) != 0) {
    layout_free(&L);
    return -1;
  }
  int32_t n_scenes = 0;
  for (int32_t i = 0; i < n_sub; ++i) {
    if (sub_scene[i] < 0) { layout_free(&L); return -1; }
    if (sub_scene[i] + 1 > n_scenes) n_scenes = sub_scene[i] + 1;
  }
  for (int32_t j = 0; j < n_if; ++j)
    for (int m = 1; m < if_nsub[j]; ++m)
      if (sub_scene[if_sub[MEMB * j]] != sub_scene[if_sub[MEMB * j + m]]) {
        layout_free(&L);
        return -1;
      }
  /* group subsystems and interfaces by scene (interfaces belong to their member's scene) */
  int32_t* scnt = calloc((size_t)n_scenes + 1, sizeof(int32_t));
  int32_t* icnt = calloc((size_t)n_scenes + 1, sizeof(int32_t));
  int32_t* slist = malloc(sizeof(int32_t) * (size_t)n_sub);
  int32_t* ilist = malloc(sizeof(int32_t) * (size_t)(n_if > 0 ? n_if : 1));
  int32_t* sfill = calloc((size_t)n_scenes + 1, sizeof(int32_t));
  int32_t* ifill = calloc((size_t)n_scenes + 1, sizeof(int32_t));
  for (int32_t i = 0; i < n_sub; ++i) scnt[sub_scene[i] + 1]++;
  for (int32_t j = 0; j < n_if; ++j) icnt[sub_scene[if_sub[MEMB * j]] + 1]++;
  for (int32_t s = 0; s < n_scenes; ++s) { scnt[s + 1] += scnt[s]; icnt[s + 1] += icnt[s]; }
  for (int32_t i = 0; i < n_sub; ++i) { int32_t s = sub_scene[i]; slist[scnt[s] + sfill[s]++] = i; }
  for (int32_t j = 0; j < n_if; ++j) { int32_t s = sub_scene[if_sub[MEMB * j]]; ilist[icnt[s] + ifill[s]++] = j; }

  size_t nslot = (size_t)L.slot_off[n_sub] + 1;
  double* xs = malloc(sizeof(double) * nslot);
  double* ys = malloc(sizeof(double) * nslot);
  double* yps = malloc(sizeof(double) * nslot);
  const int pair = r_prim && r_dual;
  double* zbs = pair ? malloc(sizeof(double) * nslot) : NULL;
  double* lbs = pair ? malloc(sizeof(double) * ((size_t)L.e_off[n_if] + 1)) : NULL;
  solve_args_t S = {sub_ndof, if_kind, if_dim, if_nsub, if_sub, if_mu, A, b, J, e, z0, u0,
                    rho, tol, max_iters, contact_model, if_k, if_alpha, v_hat, lambda, z, u, beta, xs, ys, yps,
                    zbs, lbs, &L};
  int rc = (xs && ys && yps && (!pair || (zbs && lbs))) ? 0 : -1;
  const int32_t n_run = rc == 0 ? n_scenes : 0;
#ifdef _OPENMP
  if (n_threads > 0) omp_set_num_threads(n_threads);
#pragma omp parallel for schedule(dynamic) reduction(min : rc) if (n_run > 1)
#endif
  for (int32_t s = 0; s < n_run; ++s) {
    /* iteration bound of Alg. 1 for this scene: its own cap when given */
    const int32_t cap = scene_max_iters ? scene_max_iters[s] : max_iters;
    int r = cap < 1 ? -1 : solve_scene(&S, cap, slist + scnt[s], scnt[s + 1] - scnt[s], ilist + icnt[s],
                        icnt[s + 1] - icnt[s], iters + s, converged + s, theta + s, r_theta + s,
                        pair ? r_prim + s : NULL, pair ? r_dual + s : NULL);
    if (r < rc) rc = r;
  }
  (void)n_threads;
  free(scnt); free(icnt); free(slist); free(ilist); free(sfill); free(ifill);
  free(xs); free(ys); free(yps); free(zbs); free(lbs);
  layout_free(&L);
  return rc;
}

/* ------------------------------------------------------------------------------------ */
/* Rigid boxes in maximal coordinates: Eq. (2)-(5) per step                               */
/* ------------------------------------------------------------------------------------ */

/* Generalised velocity of a body: (v world frame, omega body frame); M = diag(m I3, I_b)
 * with I_b the principal inertia.  The velocity of a body point r (body frame) is
 * v + R (omega x r); along a world direction d that is d.v + omega.(r x R^T d), so its
 * Jacobian row is (d, r x R^T d).  The body-frame angular velocity seen along a world
 * direction n is omega.(R^T n). */

static void mat_t_vec(const double* R, const double* d, double* out) { /* R^T d */
  for (int c = 0; c < 3; ++c) out[c] = R[0 * 3 + c] * d[0] + R[1 * 3 + c] * d[1] + R[2 * 3 + c] * d[2];
}
static void mat_vec(const double* R, const double* v, double* out) { /* R v */
  for (int r = 0; r < 3; ++r) out[r] = R[r * 3 + 0] * v[0] + R[r * 3 + 1] * v[1] + R[r * 3 + 2] * v[2];
}
static void cross3(const double* a, const double* b, double* out) {
  out[0] = a[1] * b[2] - a[2] * b[1];
  out[1] = a[2] * b[0] - a[0] * b[2];
  out[2] = a[0] * b[1] - a[1] * b[0];
}

/* Jacobian row (6 entries) of a body point's velocity along world direction d. */
static void point_row(const double* R, const double* r, const double* d, double* row) {
  double a[3];
  mat_t_vec(R, d, a);
  row[0] = d[0]; row[1] = d[1]; row[2] = d[2];
  cross3(r, a, row + 3);
}
/* Jacobian row (6 entries) of the world angular velocity along world direction n. */
static void ang_row(const double* R, const double* n, double* row) {
  row[0] = row[1] = row[2] = 0.0;
  mat_t_vec(R, n, row + 3);
}

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
                          double* A, double* b, double* J, double* e) {
  if (!(dt > 0.0)) return -1;
  layout_t L;
  memset(&L, 0, sizeof(L));
  if (layout_build(&L, n_sub, sub_ndof, n_if, if_dim, if_nsub, if_sub, 2) != 0) {
    layout_free(&L);
    return -1;
  }
  memset(A, 0, sizeof(double) * (size_t)L.A_off[n_sub]);
  memset(J, 0, sizeof(double) * (size_t)L.J_off[n_sub]);
  memset(e, 0, sizeof(double) * (size_t)L.e_off[n_if]);
  const double g[3] = {0.0, 0.0, -gravity};
  /* Eq. (2) solved for the midpoint velocity: (2/t) M v_hat = (2/t) M v - C v + f + J^T lambda.
     C v is the gyroscopic term (0, omega x I omega) evaluated at the step's start,
     f the weight (m g, 0). */
  for (int32_t k = 0; k < nb; ++k) {
    int32_t i = body_sub[k];
    int n = sub_ndof[i];
    int c0 = 6 * body_local[k];
    if (c0 + 6 > n) { layout_free(&L); return -1; }
    double* Ai = A + L.A_off[i];
    double* bi = b + L.dof_off[i] + c0;
    const double* I = inertia + 3 * k;
    const double* w = omega + 3 * k;
    double m = mass[k];
    for (int a = 0; a < 3; ++a) {
      Ai[(c0 + a) * n + c0 + a] = 2.0 / dt * m;
      Ai[(c0 + 3 + a) * n + c0 + 3 + a] = 2.0 / dt * I[a];
    }
    double Iw[3] = {I[0] * w[0], I[1] * w[1], I[2] * w[2]}, gyro[3];
    cross3(w, Iw, gyro);
    for (int a = 0; a < 3; ++a) {
      bi[a] = 2.0 / dt * m * vel[3 * k + a] + m * g[a];
      bi[3 + a] = 2.0 / dt * Iw[a] - gyro[a];
    }
  }
  /* Revolute joints: anchor points coincide (3 rows) and the relative world angular
     velocity has no component along u, v (2 rows), where (h,u,v) is the joint frame
     fixed in body a.  Rows of member a carry +J_a, rows of member b carry -J_b; a joint
     inside one subsystem has a single member whose rows carry J_a - J_b.  Errors are
     Baumgarte terms gamma*phi/t: phi = x_a - x_b for the anchors and
     phi_k = n_k . (h_b x h_a) (world frame, n_k = R_a u_a, R_a v_a) for the axes, whose
     rates are exactly the constrained velocities. */
  for (int32_t q = 0; q < nj; ++q) {
    int32_t ba = joint_body[2 * q], bb = joint_body[2 * q + 1];
    int32_t j = joint_if[q];
    if (j < 0 || j >= n_if || if_dim[j] != 5) { layout_free(&L); return -1; }
    const double* Ra = rot + 9 * ba;
    const double* Rb = rot + 9 * bb;
    const double* ra = joint_anchor + 6 * q;
    const double* rb = joint_anchor + 6 * q + 3;
    const double* F = joint_frame_a + 9 * q;
    double xa[3], xb[3], ha[3], hb[3], nrm[2][3], hbxha[3];
    mat_vec(Ra, ra, xa);
    mat_vec(Rb, rb, xb);
    for (int a = 0; a < 3; ++a) { xa[a] += pos[3 * ba + a]; xb[a] += pos[3 * bb + a]; }
    mat_vec(Ra, F, ha);
    mat_vec(Rb, joint_axis_b + 3 * q, hb);
    mat_vec(Ra, F + 3, nrm[0]);
    mat_vec(Ra, F + 6, nrm[1]);
    cross3(hb, ha, hbxha);
    double rowa[5][6], rowb[5][6];
    for (int k = 0; k < 3; ++k) {
      double d[3] = {0.0, 0.0, 0.0};
      d[k] = 1.0;
      point_row(Ra, ra, d, rowa[k]);
      point_row(Rb, rb, d, rowb[k]);
      e[L.e_off[j] + k] = baumgarte * (xa[k] - xb[k]) / dt;
    }
    for (int k = 0; k < 2; ++k) {
      ang_row(Ra, nrm[k], rowa[3 + k]);
      ang_row(Rb, nrm[k], rowb[3 + k]);
      e[L.e_off[j] + 3 + k] = baumgarte * (nrm[k][0] * hbxha[0] + nrm[k][1] * hbxha[1] + nrm[k][2] * hbxha[2]) / dt;
    }
    int32_t sa = body_sub[ba], sb = body_sub[bb];
    int ca = 6 * body_local[ba], cb = 6 * body_local[bb];
    if (if_nsub[j] == 1) {
      int32_t i = if_sub[2 * j];
      if (sa != i || sb != i) { layout_free(&L); return -1; }
      int n = sub_ndof[i];
      double* Ji = J + L.J_off[i];
      int64_t r0 = L.if_slot[MEMB * j] - L.slot_off[i];
      for (int k = 0; k < 5; ++k)
        for (int c = 0; c < 6; ++c) {
          Ji[(r0 + k) * n + ca + c] += rowa[k][c];
          Ji[(r0 + k) * n + cb + c] -= rowb[k][c];
        }
    } else {
      if (if_sub[2 * j] != sa || if_sub[2 * j + 1] != sb) { layout_free(&L); return -1; }
      int na = sub_ndof[sa], nbb = sub_ndof[sb];
      double* Ja = J + L.J_off[sa];
      double* Jb = J + L.J_off[sb];
      int64_t ra0 = L.if_slot[MEMB * j] - L.slot_off[sa];
      int64_t rb0 = L.if_slot[MEMB * j + 1] - L.slot_off[sb];
      for (int k = 0; k < 5; ++k)
        for (int c = 0; c < 6; ++c) {
          Ja[(ra0 + k) * na + ca + c] = rowa[k][c];
          Jb[(rb0 + k) * nbb + cb + c] = -rowb[k][c];
        }
    }
  }
  /* Ground contacts against the plane z = 0: rows along (e_z, e_x, e_y); the normal
     error is the gap over the step, e_n = phi/t, tangential errors zero. */
  for (int32_t q = 0; q < ncon; ++q) {
    int32_t k = contact_body[q];
    int32_t j = contact_if[q];
    if (j < 0 || j >= n_if || if_dim[j] != 3 || if_nsub[j] != 1 || if_sub[2 * j] != body_sub[k]) {
      layout_free(&L);
      return -1;
    }
    const double* R = rot + 9 * k;
    const double* r = contact_point + 3 * q;
    double xw[3];
    mat_vec(R, r, xw);
    double gap = pos[3 * k + 2] + xw[2];
    int32_t i = body_sub[k];
    int n = sub_ndof[i];
    int c0 = 6 * body_local[k];
    double* Ji = J + L.J_off[i];
    int64_t r0 = L.if_slot[MEMB * j] - L.slot_off[i];
    const double dirs[3][3] = {{0, 0, 1}, {1, 0, 0}, {0, 1, 0}};
    for (int a = 0; a < 3; ++a) {
      double row[6];
      point_row(R, r, dirs[a], row);
      for (int c = 0; c < 6; ++c) Ji[(r0 + a) * n + c0 + c] = row[c];
    }
    e[L.e_off[j]] = gap / dt;
    e[L.e_off[j] + 1] = 0.0;
    e[L.e_off[j] + 2] = 0.0;
  }
  layout_free(&L);
  return 0;
}

/* Rotation vector of a rotation matrix Q (the inverse of Rodrigues' formula): angle
 * acos((tr Q - 1)/2) about the axis vee(Q - Q^T)/(2 sin angle); for small angles the
 * factor angle/sin(angle) is taken from its series. */
static void so3_log(const double* Q, double* th) {
  double c = 0.5 * (Q[0] + Q[4] + Q[8] - 1.0);
  if (c > 1.0) c = 1.0;
  if (c < -1.0) c = -1.0;
  double ang = acos(c);
  double f = ang < 1e-4 ? 1.0 + ang * ang / 6.0 : ang / sin(ang);
  th[0] = 0.5 * f * (Q[7] - Q[5]);
  th[1] = 0.5 * f * (Q[2] - Q[6]);
  th[2] = 0.5 * f * (Q[3] - Q[1]);
}

/* Links: rows between two bodies (or on one body) along directions f_k fixed in body a's
 * frame (rows of link_frame, world directions d_k = R_a f_k), for an interface of kind
 * soft (Eq. 3), equality or hard inequality (Eq. 4) or contact (Eq. 5).
 *   type 0 (linear): the velocity of the anchor point of a minus that of b along d_k;
 *     phi_k = (x_a - x_b) . d_k with x = p + R r the anchor points;
 *   type 1 (angular): the world angular velocity of a minus that of b along d_k;
 *     phi_k = -f_k . log(R_a^T R_b), whose rate is that row near the rest pose.
 * A one-body link (link_body[2q+1] = -1) has only a's rows and no error: velocity-level
 * constraints such as the no-slip condition of a wheel (non-holonomic).  Errors: soft
 * e_k = phi_k (so that lambda = -k (phi + alpha J v_hat), the spring force at the step's
 * midpoint for alpha = t/2); equality and hard e_k = gamma phi_k / t (Baumgarte, as the
 * joints); contact e = (phi_0 / t, 0, 0) (the gap closed over the step, as the ground
 * contacts).  Rows of member a carry +J_a, rows of member b carry -J_b; a link inside one
 * subsystem has a single member whose rows carry J_a - J_b.  Called after
 * oracle_rigid_assemble on the same arrays (the link rows are still zero there). */
/* Tangent basis of a unit normal n: the world axis least aligned with n (first of equals),
 * made orthogonal to n and normalised, then n x t1. */
static void sphere_tangents(const double* n, double* t1, double* t2) {
  int ax = 0;
  for (int a = 1; a < 3; ++a)
    if (fabs(n[a]) < fabs(n[ax])) ax = a;
  double dot = n[ax], len = 0.0;
  for (int a = 0; a < 3; ++a) {
    t1[a] = (a == ax ? 1.0 : 0.0) - dot * n[a];
    len += t1[a] * t1[a];
  }
  len = sqrt(len);
  for (int a = 0; a < 3; ++a) t1[a] /= len;
  cross3(n, t1, t2);
}

int oracle_rigid_links(int32_t n_sub, const int32_t* sub_ndof, int32_t n_if, const int32_t* if_kind,
                       const int32_t* if_dim, const int32_t* if_nsub, const int32_t* if_sub,
                       const int32_t* body_sub, const int32_t* body_local, const double* pos,
                       const double* rot, int32_t nl, const int32_t* link_type, const int32_t* link_body,
                       const double* link_anchor, const double* link_frame, const int32_t* link_if,
                       double dt, double baumgarte, double* J, double* e) {
  if (!(dt > 0.0)) return -1;
  layout_t L;
  memset(&L, 0, sizeof(L));
  if (layout_build(&L, n_sub, sub_ndof, n_if, if_dim, if_nsub, if_sub, 2) != 0) {
    layout_free(&L);
    return -1;
  }
  for (int32_t q = 0; q < nl; ++q) {
    const int32_t ba = link_body[2 * q], bb = link_body[2 * q + 1], j = link_if[q], ty = link_type[q];
    if (j < 0) continue; /* folded into its subsystem's dynamics (oracle_rigid_fold_soft) */
    if (j >= n_if || ba < 0 || ty < 0 || ty > 2 || if_dim[j] < 1 || if_dim[j] > 3) {
      layout_free(&L);
      return -1;
    }
    const int dim = if_dim[j], kind = if_kind[j];
    const double* Ra = rot + 9 * ba;
    const double* ra = link_anchor + 6 * q;
    const double* rb = link_anchor + 6 * q + 3;
    double rowa[3][6], rowb[3][6], phi[3] = {0.0, 0.0, 0.0};
    double xa[3], xb[3], th[3] = {0.0, 0.0, 0.0};
    if (ty == 2) {
      /* sphere contact (Eq. 5 between round bodies): the normal follows the centres (or is a
       * plane's world normal), the contact points lie on the spheres along it */
      if (kind != 1 || dim != 3) { layout_free(&L); return -1; }
      double dir[3][3], pa[3], pb[3];
      const double rad_a = ra[0];
      if (bb >= 0) {
        const double rad_b = rb[0];
        double dv[3], len = 0.0;
        for (int a = 0; a < 3; ++a) { dv[a] = pos[3 * ba + a] - pos[3 * bb + a]; len += dv[a] * dv[a]; }
        len = sqrt(len);
        if (!(len > 0.0)) { layout_free(&L); return -1; }
        for (int a = 0; a < 3; ++a) dir[0][a] = dv[a] / len;
        sphere_tangents(dir[0], dir[1], dir[2]);
        phi[0] = len - rad_a - rad_b;
        for (int a = 0; a < 3; ++a) { pa[a] = -rad_a * dir[0][a]; pb[a] = rad_b * dir[0][a]; }
      } else {
        const double* f = link_frame + 9 * q;  /* world frame: plane normal, two tangents */
        for (int r = 0; r < 3; ++r)
          for (int a = 0; a < 3; ++a) dir[r][a] = f[3 * r + a];
        phi[0] = dir[0][0] * pos[3 * ba] + dir[0][1] * pos[3 * ba + 1] + dir[0][2] * pos[3 * ba + 2] - rb[0] - rad_a;
        for (int a = 0; a < 3; ++a) pa[a] = -rad_a * dir[0][a];
      }
      for (int k = 0; k < 3; ++k) {
        double cr[3];
        cross3(pa, dir[k], cr);
        rowa[k][0] = dir[k][0]; rowa[k][1] = dir[k][1]; rowa[k][2] = dir[k][2];
        mat_t_vec(Ra, cr, rowa[k] + 3);
        if (bb >= 0) {
          cross3(pb, dir[k], cr);
          rowb[k][0] = dir[k][0]; rowb[k][1] = dir[k][1]; rowb[k][2] = dir[k][2];
          mat_t_vec(rot + 9 * bb, cr, rowb[k] + 3);
        }
        e[L.e_off[j] + k] = k == 0 ? phi[0] / dt : 0.0;
      }
    } else if (bb >= 0) {
      const double* Rb = rot + 9 * bb;
      mat_vec(Ra, ra, xa);
      mat_vec(Rb, rb, xb);
      for (int a = 0; a < 3; ++a) { xa[a] += pos[3 * ba + a]; xb[a] += pos[3 * bb + a]; }
      if (ty == 1) {
        double Q[9];
        for (int r = 0; r < 3; ++r)
          for (int c = 0; c < 3; ++c) Q[3 * r + c] = Ra[r] * Rb[c] + Ra[3 + r] * Rb[3 + c] + Ra[6 + r] * Rb[6 + c];
        so3_log(Q, th);
      }
    }
    for (int k = 0; k < dim && ty != 2; ++k) {
      const double* f = link_frame + 9 * q + 3 * k;
      double d[3];
      mat_vec(Ra, f, d);
      if (ty == 0) point_row(Ra, ra, d, rowa[k]);
      else ang_row(Ra, d, rowa[k]);
      if (bb >= 0) {
        const double* Rb = rot + 9 * bb;
        if (ty == 0) {
          point_row(Rb, rb, d, rowb[k]);
          phi[k] = (xa[0] - xb[0]) * d[0] + (xa[1] - xb[1]) * d[1] + (xa[2] - xb[2]) * d[2];
        } else {
          ang_row(Rb, d, rowb[k]);
          phi[k] = -(f[0] * th[0] + f[1] * th[1] + f[2] * th[2]);
        }
      }
      double ek;
      if (kind == 3) ek = phi[k];
      else if (kind == 1) ek = k == 0 ? phi[0] / dt : 0.0;
      else ek = baumgarte * phi[k] / dt;
      e[L.e_off[j] + k] = ek;
    }
    const int32_t sa = body_sub[ba];
    const int ca = 6 * body_local[ba];
    if (if_nsub[j] == 1) {
      const int32_t i = if_sub[2 * j];
      if (sa != i || (bb >= 0 && body_sub[bb] != i)) { layout_free(&L); return -1; }
      const int n = sub_ndof[i];
      double* Ji = J + L.J_off[i];
      const int64_t r0 = L.if_slot[MEMB * j] - L.slot_off[i];
      for (int k = 0; k < dim; ++k)
        for (int c = 0; c < 6; ++c) {
          Ji[(r0 + k) * n + ca + c] += rowa[k][c];
          if (bb >= 0) Ji[(r0 + k) * n + 6 * body_local[bb] + c] -= rowb[k][c];
        }
    } else {
      if (bb < 0 || if_sub[2 * j] != sa || if_sub[2 * j + 1] != body_sub[bb]) { layout_free(&L); return -1; }
      const int32_t sb = body_sub[bb];
      const int na = sub_ndof[sa], nbb = sub_ndof[sb], cb = 6 * body_local[bb];
      double* Ja = J + L.J_off[sa];
      double* Jb = J + L.J_off[sb];
      const int64_t ra0 = L.if_slot[MEMB * j] - L.slot_off[sa];
      const int64_t rb0 = L.if_slot[MEMB * j + 1] - L.slot_off[sb];
      for (int k = 0; k < dim; ++k)
        for (int c = 0; c < 6; ++c) {
          Ja[(ra0 + k) * na + ca + c] = rowa[k][c];
          Jb[(rb0 + k) * nbb + cb + c] = -rowb[k][c];
        }
    }
  }
  layout_free(&L);
  return 0;
}

/* Soft links folded into a subsystem's own dynamics (Sec. III-B, the remark after Eq. 6):
 * a soft coupling (Eq. 3) between two bodies of subsystem i, lambda = -k (phi + alpha J v_hat)
 * with J the link's rows over subsystem i (body a's row minus body b's) and phi its
 * separation, is linear in v_hat, so the subsystem equation A_i v_hat = b_i + J^T lambda
 * becomes (A_i + k alpha J^T J) v_hat = b_i - k J^T phi.  Adds these terms to A and b (the
 * assembled layout) for every link with link_if < 0; rows and phi are those of the link
 * interfaces (oracle_rigid_links). */
int oracle_rigid_fold_soft(int32_t n_sub, const int32_t* sub_ndof, const int32_t* body_sub,
                           const int32_t* body_local, const double* pos, const double* rot, int32_t nl,
                           const int32_t* link_type, const int32_t* link_body, const double* link_anchor,
                           const double* link_frame, const int32_t* link_if, const int32_t* link_dim,
                           const double* link_k, const double* link_alpha, double* A, double* b) {
  int64_t* a_off = (int64_t*)calloc((size_t)n_sub + 1, sizeof(int64_t));
  int64_t* b_off = (int64_t*)calloc((size_t)n_sub + 1, sizeof(int64_t));
  if (!a_off || !b_off) { free(a_off); free(b_off); return -2; }
  for (int32_t i = 0; i < n_sub; ++i) {
    a_off[i + 1] = a_off[i] + (int64_t)sub_ndof[i] * sub_ndof[i];
    b_off[i + 1] = b_off[i] + sub_ndof[i];
  }
  int rc = 0;
  for (int32_t q = 0; q < nl && rc == 0; ++q) {
    if (link_if[q] >= 0) continue;
    const int32_t ba = link_body[2 * q], bb = link_body[2 * q + 1], ty = link_type[q], dim = link_dim[q];
    if (ba < 0 || bb < 0 || ba == bb || body_sub[ba] != body_sub[bb] || (ty != 0 && ty != 1) || dim < 1 ||
        dim > 3 || !(link_k[q] >= 0.0) || !(link_alpha[q] > 0.0)) {
      rc = -1;
      break;
    }
    const int32_t i = body_sub[ba];
    const int n = sub_ndof[i];
    const int col[2] = {6 * body_local[ba], 6 * body_local[bb]};
    const double* Ra = rot + 9 * ba;
    const double* Rb = rot + 9 * bb;
    const double* ra = link_anchor + 6 * q;
    const double* rb = ra + 3;
    double xa[3], xb[3], th[3] = {0.0, 0.0, 0.0};
    mat_vec(Ra, ra, xa);
    mat_vec(Rb, rb, xb);
    for (int a = 0; a < 3; ++a) { xa[a] += pos[3 * ba + a]; xb[a] += pos[3 * bb + a]; }
    if (ty == 1) {
      double Q[9];
      for (int r = 0; r < 3; ++r)
        for (int c = 0; c < 3; ++c) Q[3 * r + c] = Ra[r] * Rb[c] + Ra[3 + r] * Rb[3 + c] + Ra[6 + r] * Rb[6 + c];
      so3_log(Q, th);
    }
    double* Ai = A + a_off[i];
    double* bi = b + b_off[i];
    const double kk = link_k[q], ka = link_k[q] * link_alpha[q];
    for (int k = 0; k < dim; ++k) {
      const double* f = link_frame + 9 * q + 3 * k;
      double d[3], row[12], phi;
      mat_vec(Ra, f, d);
      if (ty == 0) {
        point_row(Ra, ra, d, row);
        point_row(Rb, rb, d, row + 6);
        phi = (xa[0] - xb[0]) * d[0] + (xa[1] - xb[1]) * d[1] + (xa[2] - xb[2]) * d[2];
      } else {
        ang_row(Ra, d, row);
        ang_row(Rb, d, row + 6);
        phi = -(f[0] * th[0] + f[1] * th[1] + f[2] * th[2]);
      }
      for (int c = 6; c < 12; ++c) row[c] = -row[c];
      for (int r = 0; r < 12; ++r) {
        const int gr = col[r / 6] + r % 6;
        bi[gr] -= kk * phi * row[r];
        for (int c = 0; c < 12; ++c) Ai[(int64_t)gr * n + col[c / 6] + c % 6] += ka * row[r] * row[c];
      }
    }
  }
  free(a_off);
  free(b_off);
  return rc;
}

/* exp([phi]x) by Rodrigues' formula, with Taylor coefficients for small angles. */
static void so3_exp(const double* phi, double* E) {
  double th2 = phi[0] * phi[0] + phi[1] * phi[1] + phi[2] * phi[2];
  double th = sqrt(th2);
  double a, c;
  if (th < 1e-6) {
    a = 1.0 - th2 / 6.0;
    c = 0.5 - th2 / 24.0;
  } else {
    a = sin(th) / th;
    c = (1.0 - cos(th)) / th2;
  }
  double X[9] = {0.0, -phi[2], phi[1], phi[2], 0.0, -phi[0], -phi[1], phi[0], 0.0};
  for (int r = 0; r < 3; ++r)
    for (int s = 0; s < 3; ++s) {
      double x2 = 0.0;
      for (int k = 0; k < 3; ++k) x2 += X[r * 3 + k] * X[k * 3 + s];
      E[r * 3 + s] = (r == s ? 1.0 : 0.0) + a * X[r * 3 + s] + c * x2;
    }
}

int oracle_rigid_advance(int32_t nb, const int32_t* body_sub, const int32_t* body_local,
                         int32_t n_sub, const int32_t* sub_ndof, const double* v_hat, double dt,
                         const double* pos, const double* rot, const double* vel,
                         const double* omega, double* pos_out, double* rot_out,
                         double* vel_out, double* omega_out) {
  int64_t* dof_off = calloc((size_t)n_sub + 1, sizeof(int64_t));
  if (!dof_off) return -1;
  for (int32_t i = 0; i < n_sub; ++i) dof_off[i + 1] = dof_off[i] + sub_ndof[i];
  for (int32_t k = 0; k < nb; ++k) {
    const double* vh = v_hat + dof_off[body_sub[k]] + 6 * body_local[k];
    double phi[3], E[9];
    for (int a = 0; a < 3; ++a) {
      vel_out[3 * k + a] = 2.0 * vh[a] - vel[3 * k + a];
      omega_out[3 * k + a] = 2.0 * vh[3 + a] - omega[3 * k + a];
      pos_out[3 * k + a] = pos[3 * k + a] + dt * vh[a];
      phi[a] = dt * vh[3 + a];
    }
    so3_exp(phi, E);
    double Rn[9];
    for (int r = 0; r < 3; ++r)
      for (int s = 0; s < 3; ++s) {
        double acc = 0.0;
        for (int t = 0; t < 3; ++t) acc += rot[9 * k + r * 3 + t] * E[t * 3 + s];
        Rn[r * 3 + s] = acc;
      }
    memcpy(rot_out + 9 * k, Rn, sizeof(Rn));
  }
  free(dof_off);
  return 0;
}
