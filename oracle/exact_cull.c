/*
 * FP64 radiance of a Gaussian photon field at many query points, exact test
 * over candidates from a uniform grid of primitive bounding spheres.
 *
 * TEST INFRASTRUCTURE ONLY (oracle mode for large fields); never linked into
 * the product library.  Shares no code with the HIP kernels.
 *
 * Definition (Sec. 4.1 Eq. gaussian_contribution; Sec. 4.2 aggregation;
 * local frame of the supplementary hybrid query): primitive i has centre mu,
 * quaternion q = (w,x,y,z) normalised, Hamilton rotation R(q) whose columns are
 * the local axes, scales s = exp(log_scale) and flux rgb.  For a query x,
 * u = diag(1/s) R^T (x - mu), m2 = u.u; the primitive contributes
 * exp(-m2/2) rgb when m2 <= cutoff^2.  Every primitive with m2 <= cutoff^2
 * lies within cutoff * max(s) of x, so listing each primitive in every grid
 * cell that its sphere of that radius touches, and testing exactly the
 * primitives listed in x's cell, gives the brute-force result.  Sums run in
 * primitive-index order with Neumaier compensation.
 *
 * Outputs per query and channel as in the Python brute-force oracle: L, L_abs,
 * L_lo/L_hi (ambiguity envelope: |m2 - cutoff^2| <= amb_rel * max s / min s),
 * L_cond (sum of w |rgb| sum_k |u_k| eta_k, eta_k = sum_j |W_kj d_j|), count,
 * n_amb.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

typedef struct {
  double W[3][3];
  double mu[3];
  double rgb[3];
  double rho;
  double rad;
} prim_t;

typedef struct {
  double s, c;
} nsum_t; /* Neumaier compensated sum */

static void nadd(nsum_t *a, double v) {
  double t = a->s + v;
  if (fabs(a->s) >= fabs(v))
    a->c += (a->s - t) + v;
  else
    a->c += (v - t) + a->s;
  a->s = t;
}

static int prep(const float *mu, const float *quat, const float *ls, const float *rgb, int64_t i,
                double cutoff, prim_t *p) {
  double w = quat[4 * i], x = quat[4 * i + 1], y = quat[4 * i + 2], z = quat[4 * i + 3];
  double n = sqrt(w * w + x * x + y * y + z * z);
  if (!(n > 0.0)) return -1;
  w /= n; x /= n; y /= n; z /= n;
  double R[3][3] = {{1 - 2 * (y * y + z * z), 2 * (x * y - w * z), 2 * (x * z + w * y)},
                    {2 * (x * y + w * z), 1 - 2 * (x * x + z * z), 2 * (y * z - w * x)},
                    {2 * (x * z - w * y), 2 * (y * z + w * x), 1 - 2 * (x * x + y * y)}};
  double s[3], smax = 0, smin = INFINITY;
  for (int k = 0; k < 3; ++k) {
    s[k] = exp((double)ls[3 * i + k]);
    if (s[k] > smax) smax = s[k];
    if (s[k] < smin) smin = s[k];
  }
  for (int k = 0; k < 3; ++k)
    for (int j = 0; j < 3; ++j) p->W[k][j] = R[j][k] / s[k];
  for (int k = 0; k < 3; ++k) {
    p->mu[k] = mu[3 * i + k];
    p->rgb[k] = rgb[3 * i + k];
  }
  p->rho = smax / smin;
  p->rad = cutoff * smax * 1.001;
  return 0;
}

int gpf_oracle_radiance(const float *mu, const float *quat, const float *ls, const float *rgb,
                        int64_t n, const float *x, int64_t q, double cutoff, double amb_rel,
                        double *L, double *L_abs, double *L_lo, double *L_hi, double *L_cond,
                        int64_t *count, int64_t *n_amb) {
  prim_t *P = (prim_t *)malloc(sizeof(prim_t) * (size_t)n);
  if (!P) return -2;
  double lo[3] = {INFINITY, INFINITY, INFINITY}, hi[3] = {-INFINITY, -INFINITY, -INFINITY};
  double radsum = 0;
  for (int64_t i = 0; i < n; ++i) {
    if (prep(mu, quat, ls, rgb, i, cutoff, &P[i]) != 0) {
      free(P);
      return -1;
    }
    for (int a = 0; a < 3; ++a) {
      if (P[i].mu[a] - P[i].rad < lo[a]) lo[a] = P[i].mu[a] - P[i].rad;
      if (P[i].mu[a] + P[i].rad > hi[a]) hi[a] = P[i].mu[a] + P[i].rad;
    }
    radsum += P[i].rad;
  }
  /* cell edge: about the mean sphere radius, at most 256 cells per axis */
  double h = radsum / (double)n;
  int dim[3];
  for (int a = 0; a < 3; ++a) {
    double e = hi[a] - lo[a];
    if (e / h > 256) h = e / 256;
  }
  for (int a = 0; a < 3; ++a) dim[a] = (int)floor((hi[a] - lo[a]) / h) + 1;
  int64_t ncell = (int64_t)dim[0] * dim[1] * dim[2];
  int64_t *start = (int64_t *)calloc((size_t)ncell + 1, sizeof(int64_t));
  if (!start) {
    free(P);
    return -2;
  }
  /* count, prefix, fill (prims appended in index order) */
  for (int pass = 0; pass < 2; ++pass) {
    int64_t *fill = NULL;
    int32_t *list = NULL;
    if (pass == 1) {
      for (int64_t c = 0; c < ncell; ++c) start[c + 1] += start[c];
      fill = (int64_t *)calloc((size_t)ncell, sizeof(int64_t));
      list = (int32_t *)malloc(sizeof(int32_t) * (size_t)(start[ncell] + 1));
      if (!fill || !list) {
        free(fill);
        free(list);
        free(start);
        free(P);
        return -2;
      }
    }
    for (int64_t i = 0; i < n; ++i) {
      int c0[3], c1[3];
      for (int a = 0; a < 3; ++a) {
        c0[a] = (int)floor((P[i].mu[a] - P[i].rad - lo[a]) / h);
        c1[a] = (int)floor((P[i].mu[a] + P[i].rad - lo[a]) / h);
        if (c0[a] < 0) c0[a] = 0;
        if (c1[a] > dim[a] - 1) c1[a] = dim[a] - 1;
      }
      for (int cz = c0[2]; cz <= c1[2]; ++cz)
        for (int cy = c0[1]; cy <= c1[1]; ++cy)
          for (int cx = c0[0]; cx <= c1[0]; ++cx) {
            int64_t c = ((int64_t)cz * dim[1] + cy) * dim[0] + cx;
            if (pass == 0)
              start[c + 1] += 1;
            else
              list[start[c] + fill[c]++] = (int32_t)i;
          }
    }
    if (pass == 1) {
      free(fill);
      const double c2 = cutoff * cutoff;
#pragma omp parallel for schedule(dynamic, 256)
      for (int64_t j = 0; j < q; ++j) {
        double xq[3] = {x[3 * j], x[3 * j + 1], x[3 * j + 2]};
        nsum_t sL[3], sA[3], sLo[3], sHi[3];
        double cond[3] = {0, 0, 0};
        memset(sL, 0, sizeof sL);
        memset(sA, 0, sizeof sA);
        memset(sLo, 0, sizeof sLo);
        memset(sHi, 0, sizeof sHi);
        int64_t cnt = 0, amb = 0;
        int inside = 1;
        int ci[3];
        for (int a = 0; a < 3; ++a) {
          double t = floor((xq[a] - lo[a]) / h);
          if (t < 0 || t > dim[a] - 1) inside = 0;
          ci[a] = (int)t;
        }
        if (inside) {
          int64_t c = ((int64_t)ci[2] * dim[1] + ci[1]) * dim[0] + ci[0];
          for (int64_t e = start[c]; e < start[c + 1]; ++e) {
            const prim_t *p = &P[list[e]];
            double d[3] = {xq[0] - p->mu[0], xq[1] - p->mu[1], xq[2] - p->mu[2]};
            double u[3], eta[3], m2 = 0;
            for (int k = 0; k < 3; ++k) {
              u[k] = p->W[k][0] * d[0] + p->W[k][1] * d[1] + p->W[k][2] * d[2];
              eta[k] = fabs(p->W[k][0] * d[0]) + fabs(p->W[k][1] * d[1]) + fabs(p->W[k][2] * d[2]);
              m2 += u[k] * u[k];
            }
            int inc = m2 <= c2;
            int isamb = fabs(m2 - c2) <= amb_rel * p->rho;
            if (!inc && !isamb) continue;
            double w = exp(-0.5 * m2);
            double sens = fabs(u[0]) * eta[0] + fabs(u[1]) * eta[1] + fabs(u[2]) * eta[2];
            for (int ch = 0; ch < 3; ++ch) {
              double v = w * p->rgb[ch];
              if (inc) {
                nadd(&sL[ch], v);
                nadd(&sA[ch], fabs(v));
                cond[ch] += fabs(v) * sens;
              }
              if (isamb) {
                nadd(&sLo[ch], v < 0 ? v : 0.0);
                nadd(&sHi[ch], v > 0 ? v : 0.0);
              } else if (inc) {
                nadd(&sLo[ch], v);
                nadd(&sHi[ch], v);
              }
            }
            cnt += inc;
            amb += isamb;
          }
        }
        for (int ch = 0; ch < 3; ++ch) {
          L[3 * j + ch] = sL[ch].s + sL[ch].c;
          L_abs[3 * j + ch] = sA[ch].s + sA[ch].c;
          L_lo[3 * j + ch] = sLo[ch].s + sLo[ch].c;
          L_hi[3 * j + ch] = sHi[ch].s + sHi[ch].c;
          L_cond[3 * j + ch] = cond[ch];
        }
        count[j] = cnt;
        n_amb[j] = amb;
      }
      free(list);
    }
  }
  free(start);
  free(P);
  return 0;
}
