/*
 * FP64 reference of the warm-start network (TEST INFRASTRUCTURE ONLY; see oracle/__init__.py).
 * A plain multilayer perceptron: hidden layers a_{k+1} = relu(W_k a_k + b_k), output
 * layer out = W_L a_L + b_L, evaluated row by row with no blocking; the gradient is the
 * textbook backward pass of the squared-error loss.
 */
#include <stdlib.h>
#include <string.h>

#include "subadmm_oracle.h"

static int64_t layer_offset(const int32_t* widths, int32_t k) {
  int64_t off = 0;
  for (int32_t q = 0; q < k; ++q) off += (int64_t)widths[q + 1] * widths[q] + widths[q + 1];
  return off;
}

/* Forward pass of one sample; acts[k] receives the input of layer k (acts[0] = x) and
 * acts[n_layers] the output. */
static void forward_one(int32_t n_layers, const int32_t* widths, const double* params,
                        const double* x, double** acts) {
  memcpy(acts[0], x, sizeof(double) * (size_t)widths[0]);
  for (int32_t k = 0; k < n_layers; ++k) {
    const double* W = params + layer_offset(widths, k);
    const double* b = W + (int64_t)widths[k + 1] * widths[k];
    for (int32_t o = 0; o < widths[k + 1]; ++o) {
      double s = b[o];
      for (int32_t i = 0; i < widths[k]; ++i) s += W[(int64_t)o * widths[k] + i] * acts[k][i];
      acts[k + 1][o] = (k + 1 < n_layers && s < 0.0) ? 0.0 : s;
    }
  }
}

static double** alloc_acts(int32_t n_layers, const int32_t* widths) {
  double** a = calloc((size_t)n_layers + 1, sizeof(double*));
  if (!a) return NULL;
  for (int32_t k = 0; k <= n_layers; ++k) a[k] = calloc((size_t)widths[k], sizeof(double));
  return a;
}

static void free_acts(double** a, int32_t n_layers) {
  if (!a) return;
  for (int32_t k = 0; k <= n_layers; ++k) free(a[k]);
  free(a);
}

int oracle_mlp_forward(int32_t n_layers, const int32_t* widths, const double* params,
                       int32_t batch, const double* in, double* out) {
  if (n_layers < 1 || batch < 0) return -1;
  double** a = alloc_acts(n_layers, widths);
  if (!a) return -1;
  for (int32_t s = 0; s < batch; ++s) {
    forward_one(n_layers, widths, params, in + (int64_t)s * widths[0], a);
    memcpy(out + (int64_t)s * widths[n_layers], a[n_layers], sizeof(double) * (size_t)widths[n_layers]);
  }
  free_acts(a, n_layers);
  return 0;
}

int oracle_mlp_backward(int32_t n_layers, const int32_t* widths, const double* params,
                        int32_t batch, const double* in, const double* target,
                        const double* wt, double* grad, double* loss) {
  if (n_layers < 1 || batch < 0) return -1;
  const int64_t np = layer_offset(widths, n_layers);
  memset(grad, 0, sizeof(double) * (size_t)np);
  double** a = alloc_acts(n_layers, widths);
  double** d = alloc_acts(n_layers, widths); /* d[k]: dL/d(pre-activation of layer k's output) */
  if (!a || !d) { free_acts(a, n_layers); free_acts(d, n_layers); return -1; }
  double L = 0.0;
  const int32_t no = widths[n_layers];
  for (int32_t s = 0; s < batch; ++s) {
    forward_one(n_layers, widths, params, in + (int64_t)s * widths[0], a);
    for (int32_t o = 0; o < no; ++o) {
      const double r = a[n_layers][o] - target[(int64_t)s * no + o];
      const double w = wt[(int64_t)s * no + o];
      L += 0.5 * w * r * r;
      d[n_layers][o] = w * r;
    }
    for (int32_t k = n_layers - 1; k >= 0; --k) {
      const double* W = params + layer_offset(widths, k);
      double* gW = grad + layer_offset(widths, k);
      double* gb = gW + (int64_t)widths[k + 1] * widths[k];
      for (int32_t o = 0; o < widths[k + 1]; ++o) {
        gb[o] += d[k + 1][o];
        for (int32_t i = 0; i < widths[k]; ++i) gW[(int64_t)o * widths[k] + i] += d[k + 1][o] * a[k][i];
      }
      if (k > 0) {
        /* through W_k, then through the ReLU that produced a[k] (a[k] > 0 <=> active) */
        for (int32_t i = 0; i < widths[k]; ++i) {
          double s2 = 0.0;
          for (int32_t o = 0; o < widths[k + 1]; ++o) s2 += W[(int64_t)o * widths[k] + i] * d[k + 1][o];
          d[k][i] = a[k][i] > 0.0 ? s2 : 0.0;
        }
      }
    }
  }
  *loss = L;
  free_acts(a, n_layers);
  free_acts(d, n_layers);
  return 0;
}
