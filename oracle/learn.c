/*
 * Oracle, learned-guess part: the multilayer perceptron used for the Poisson
 * initial guess, in FP64, with optional emulation of the BF16 rounding the GPU
 * applies where values enter a matrix product.  TEST INFRASTRUCTURE ONLY.
 *
 * Network m -> h -> h -> m:  Z1 = X W1^T + b1, H1 = GELU(Z1), Z2 = H1 W2^T + b2,
 * H2 = GELU(Z2), Y = H2 W3^T + b3, GELU(z) = z/2 (1 + erf(z / sqrt 2)).
 * Loss: mean over all B*m entries of (Y - T)^2.  Back-propagation by the
 * chain rule: dY = 2 (Y - T) / (B m); dW3 = dY^T H2; db3 = column sums of dY;
 * dH2 = dY W3; dZ2 = dH2 * GELU'(Z2); dW2 = dZ2^T H1; db2 = sums of dZ2;
 * dH1 = dZ2 W2; dZ1 = dH1 * GELU'(Z1); dW1 = dZ1^T X; db1 = sums of dZ1,
 * GELU'(z) = Phi(z) + z phi(z) (standard normal cdf and density).
 * With emulation on, X, the weights, H1, H2, dY, dZ2 and dZ1 are rounded to
 * BF16 (round to nearest even) before they are multiplied.
 * Parameter layout: [W1 h*m | b1 h | W2 h*h | b2 h | W3 m*h | b3 m], W[out][in].
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#include "oracle.h"

/* round to the nearest BF16 value (ties to even), through single precision */
double orc_bf16(double x) {
  float f = (float)x;
  uint32_t u;
  memcpy(&u, &f, 4);
  if ((u & 0x7f800000u) == 0x7f800000u && (u & 0x007fffffu)) return x; /* NaN */
  u += 0x7fffu + ((u >> 16) & 1u);
  u &= 0xffff0000u;
  memcpy(&f, &u, 4);
  return (double)f;
}

static double gelu(double z) { return 0.5 * z * (1.0 + erf(z / sqrt(2.0))); }
static double gelu_grad(double z) {
  const double cdf = 0.5 * (1.0 + erf(z / sqrt(2.0)));
  const double pdf = exp(-0.5 * z * z) / sqrt(2.0 * 3.14159265358979323846);
  return cdf + z * pdf;
}

double orc_gelu(double z) { return gelu(z); }
double orc_gelu_grad(double z) { return gelu_grad(z); }

static double *dvec(size_t n) { return (double *)calloc(n ? n : 1, sizeof(double)); }

/* C[r][o] = sum_i A[r][i] W[o][i] + bias[o] */
static void linear(int rows, int in, int out, const double *A, const double *W, const double *bias, double *C) {
  for (int r = 0; r < rows; r++)
    for (int o = 0; o < out; o++) {
      double s = 0.0;
      for (int i = 0; i < in; i++) s += A[(size_t)r * in + i] * W[(size_t)o * in + i];
      C[(size_t)r * out + o] = s + bias[o];
    }
}

static void round_all(double *v, size_t n, int emulate) {
  if (!emulate) return;
  for (size_t i = 0; i < n; i++) v[i] = orc_bf16(v[i]);
}

void orc_mlp_forward_backward(int m, int h, int B, const float *params, const float *X, const float *T, int emulate,
                              double *loss, double *Yout, double *grad) {
  const size_t w1 = 0, b1 = w1 + (size_t)h * m, w2 = b1 + h, b2 = w2 + (size_t)h * h, w3 = b2 + h,
               b3 = w3 + (size_t)m * h, total = b3 + m;
  double *P = dvec(total), *Pb = dvec(total);
  for (size_t i = 0; i < total; i++) P[i] = Pb[i] = params[i];
  round_all(Pb + w1, (size_t)h * m, emulate);
  round_all(Pb + w2, (size_t)h * h, emulate);
  round_all(Pb + w3, (size_t)m * h, emulate);
  double *Xb = dvec((size_t)B * m), *Z1 = dvec((size_t)B * h), *H1 = dvec((size_t)B * h), *Z2 = dvec((size_t)B * h);
  double *H2 = dvec((size_t)B * h), *Y = dvec((size_t)B * m), *dY = dvec((size_t)B * m);
  double *dH2 = dvec((size_t)B * h), *dZ2 = dvec((size_t)B * h), *dH1 = dvec((size_t)B * h), *dZ1 = dvec((size_t)B * h);
  for (size_t i = 0; i < (size_t)B * m; i++) Xb[i] = X[i];
  round_all(Xb, (size_t)B * m, emulate);
  /* forward */
  linear(B, m, h, Xb, Pb + w1, P + b1, Z1);
  for (size_t i = 0; i < (size_t)B * h; i++) H1[i] = gelu(Z1[i]);
  round_all(H1, (size_t)B * h, emulate);
  linear(B, h, h, H1, Pb + w2, P + b2, Z2);
  for (size_t i = 0; i < (size_t)B * h; i++) H2[i] = gelu(Z2[i]);
  round_all(H2, (size_t)B * h, emulate);
  linear(B, h, m, H2, Pb + w3, P + b3, Y);
  /* loss and output delta */
  double sse = 0.0;
  const double scale = 2.0 / ((double)B * m);
  for (size_t i = 0; i < (size_t)B * m; i++) {
    const double e = Y[i] - T[i];
    sse += e * e;
    dY[i] = scale * e;
  }
  if (loss) *loss = sse / ((double)B * m);
  if (Yout) memcpy(Yout, Y, sizeof(double) * (size_t)B * m);
  if (grad) {
    memset(grad, 0, sizeof(double) * total);
    double *dYb = dvec((size_t)B * m);
    memcpy(dYb, dY, sizeof(double) * (size_t)B * m);
    round_all(dYb, (size_t)B * m, emulate);
    /* layer 3 */
    for (int o = 0; o < m; o++)
      for (int i = 0; i < h; i++) {
        double s = 0.0;
        for (int r = 0; r < B; r++) s += dYb[(size_t)r * m + o] * H2[(size_t)r * h + i];
        grad[w3 + (size_t)o * h + i] = s;
      }
    for (int o = 0; o < m; o++) {
      double s = 0.0;
      for (int r = 0; r < B; r++) s += dY[(size_t)r * m + o];
      grad[b3 + o] = s;
    }
    for (int r = 0; r < B; r++)
      for (int i = 0; i < h; i++) {
        double s = 0.0;
        for (int o = 0; o < m; o++) s += dYb[(size_t)r * m + o] * Pb[w3 + (size_t)o * h + i];
        dH2[(size_t)r * h + i] = s;
      }
    for (size_t i = 0; i < (size_t)B * h; i++) dZ2[i] = dH2[i] * gelu_grad(Z2[i]);
    double *dZ2b = dvec((size_t)B * h);
    memcpy(dZ2b, dZ2, sizeof(double) * (size_t)B * h);
    round_all(dZ2b, (size_t)B * h, emulate);
    /* layer 2 */
    for (int o = 0; o < h; o++)
      for (int i = 0; i < h; i++) {
        double s = 0.0;
        for (int r = 0; r < B; r++) s += dZ2b[(size_t)r * h + o] * H1[(size_t)r * h + i];
        grad[w2 + (size_t)o * h + i] = s;
      }
    for (int o = 0; o < h; o++) {
      double s = 0.0;
      for (int r = 0; r < B; r++) s += dZ2[(size_t)r * h + o];
      grad[b2 + o] = s;
    }
    for (int r = 0; r < B; r++)
      for (int i = 0; i < h; i++) {
        double s = 0.0;
        for (int o = 0; o < h; o++) s += dZ2b[(size_t)r * h + o] * Pb[w2 + (size_t)o * h + i];
        dH1[(size_t)r * h + i] = s;
      }
    for (size_t i = 0; i < (size_t)B * h; i++) dZ1[i] = dH1[i] * gelu_grad(Z1[i]);
    double *dZ1b = dvec((size_t)B * h);
    memcpy(dZ1b, dZ1, sizeof(double) * (size_t)B * h);
    round_all(dZ1b, (size_t)B * h, emulate);
    /* layer 1 */
    for (int o = 0; o < h; o++)
      for (int i = 0; i < m; i++) {
        double s = 0.0;
        for (int r = 0; r < B; r++) s += dZ1b[(size_t)r * h + o] * Xb[(size_t)r * m + i];
        grad[w1 + (size_t)o * m + i] = s;
      }
    for (int o = 0; o < h; o++) {
      double s = 0.0;
      for (int r = 0; r < B; r++) s += dZ1[(size_t)r * h + o];
      grad[b1 + o] = s;
    }
    free(dYb); free(dZ2b); free(dZ1b);
  }
  free(P); free(Pb); free(Xb); free(Z1); free(H1); free(Z2); free(H2); free(Y); free(dY);
  free(dH2); free(dZ2); free(dH1); free(dZ1);
}

/* One Adam step (Kingma & Ba 2015) in FP64 on w with gradient g; t >= 1 is the step number. */
void orc_adam(int n, double *w, const double *g, double *m1, double *m2, int t, double lr, double b1, double b2,
              double eps) {
  for (int i = 0; i < n; i++) {
    m1[i] = b1 * m1[i] + (1.0 - b1) * g[i];
    m2[i] = b2 * m2[i] + (1.0 - b2) * g[i] * g[i];
    const double mh = m1[i] / (1.0 - pow(b1, t)), vh = m2[i] / (1.0 - pow(b2, t));
    w[i] -= lr * mh / (sqrt(vh) + eps);
  }
}
