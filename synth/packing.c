/*
 * packing.c -- seeded synthetic packings for the DEM workloads.
 *
 * Input generator only: it places spheres by pure geometry (a downward shift
 * followed by pairwise overlap projection, repeated), with none of the contact,
 * drag or integration arithmetic of the method.  Shared by the oracle side and
 * the GPU side; neither computes anything from it but positions.
 *
 * Region kinds
 *   0 box      : p = {x0, y0, z0, x1, y1, z1}
 *   1 annulus  : p = {cx, cy, r_in, r_out, z0, z1}   (z-axis hollow cylinder)
 * The particles settle towards z0; z1 bounds the start volume only.
 *
 * Neighbour search: the larger sphere of every pair finds it (ties by index),
 * searching 2 r_i around itself in a grid of side 2 r_median.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

typedef struct {
  double lo[3];
  double h;
  int64_t nc[3];
  int64_t* start;
  int64_t* idx;
} grid_t;

static int cmpd(const void* a, const void* b) {
  double p = *(const double*)a, q = *(const double*)b;
  return p < q ? -1 : (p > q ? 1 : 0);
}

static int64_t clampi(int64_t v, int64_t lo, int64_t hi) { return v < lo ? lo : (v > hi ? hi : v); }

static void grid_build(grid_t* g, int64_t n, const double* x, double h) {
  double lo[3] = {1e300, 1e300, 1e300}, hi[3] = {-1e300, -1e300, -1e300};
  for (int64_t i = 0; i < n; ++i)
    for (int c = 0; c < 3; ++c) {
      if (x[3 * i + c] < lo[c]) lo[c] = x[3 * i + c];
      if (x[3 * i + c] > hi[c]) hi[c] = x[3 * i + c];
    }
  g->h = h;
  int64_t tot = 1;
  for (int c = 0; c < 3; ++c) {
    g->lo[c] = lo[c];
    g->nc[c] = (int64_t)floor((hi[c] - lo[c]) / h) + 1;
    if (g->nc[c] > 4096) g->nc[c] = 4096;
    tot *= g->nc[c];
  }
  int64_t* cnt = (int64_t*)calloc((size_t)tot + 1, sizeof(int64_t));
  int64_t* cell = (int64_t*)malloc(sizeof(int64_t) * (size_t)n);
  for (int64_t i = 0; i < n; ++i) {
    int64_t k[3];
    for (int c = 0; c < 3; ++c) k[c] = clampi((int64_t)floor((x[3 * i + c] - g->lo[c]) / h), 0, g->nc[c] - 1);
    cell[i] = (k[2] * g->nc[1] + k[1]) * g->nc[0] + k[0];
    cnt[cell[i] + 1]++;
  }
  for (int64_t c = 0; c < tot; ++c) cnt[c + 1] += cnt[c];
  g->start = (int64_t*)malloc(sizeof(int64_t) * ((size_t)tot + 1));
  memcpy(g->start, cnt, sizeof(int64_t) * ((size_t)tot + 1));
  g->idx = (int64_t*)malloc(sizeof(int64_t) * (size_t)n);
  for (int64_t i = 0; i < n; ++i) g->idx[cnt[cell[i]]++] = i;
  free(cnt);
  free(cell);
}

static void grid_free(grid_t* g) {
  free(g->start);
  free(g->idx);
}

static void confine(int kind, const double* p, double r, double* x) {
  if (kind == 0) {
    for (int c = 0; c < 3; ++c) {
      double lo = p[c] + r, hi = p[3 + c] - r;
      if (c == 2) hi = 1e300;
      if (x[c] < lo) x[c] = lo;
      if (x[c] > hi) x[c] = hi;
    }
  } else {
    double ex = x[0] - p[0], ey = x[1] - p[1];
    double rho = sqrt(ex * ex + ey * ey);
    double rin = p[2] + r, rout = p[3] - r;
    if (rho > 0.0) {
      double t = rho;
      if (t < rin) t = rin;
      if (t > rout) t = rout;
      x[0] = p[0] + ex * (t / rho);
      x[1] = p[1] + ey * (t / rho);
    }
    if (x[2] < p[4] + r) x[2] = p[4] + r;
  }
}

/* pair list: every pair whose gap is below `skin` (the larger sphere finds it) */
static int64_t build_pairs(int64_t n, const double* x, const double* rr, double h, double skin,
                           int64_t** pi, int64_t** pj, int64_t* cap) {
  grid_t g;
  grid_build(&g, n, x, h);
  int64_t cnt = 0;
  for (int64_t i = 0; i < n; ++i) {
    double R = 2.0 * rr[i] + skin;
    int64_t k0[3], k1[3];
    for (int c = 0; c < 3; ++c) {
      k0[c] = clampi((int64_t)floor((x[3 * i + c] - R - g.lo[c]) / h), 0, g.nc[c] - 1);
      k1[c] = clampi((int64_t)floor((x[3 * i + c] + R - g.lo[c]) / h), 0, g.nc[c] - 1);
    }
    for (int64_t kz = k0[2]; kz <= k1[2]; ++kz)
      for (int64_t ky = k0[1]; ky <= k1[1]; ++ky)
        for (int64_t kx = k0[0]; kx <= k1[0]; ++kx) {
          int64_t cid = (kz * g.nc[1] + ky) * g.nc[0] + kx;
          for (int64_t q = g.start[cid]; q < g.start[cid + 1]; ++q) {
            int64_t j = g.idx[q];
            if (j == i) continue;
            if (rr[j] > rr[i] || (rr[j] == rr[i] && j < i)) continue;
            double d2 = 0.0;
            for (int c = 0; c < 3; ++c) { double d = x[3 * j + c] - x[3 * i + c]; d2 += d * d; }
            double cc = rr[i] + rr[j] + skin;
            if (d2 >= cc * cc) continue;
            if (cnt == *cap) {
              *cap = *cap * 2 + 1024;
              *pi = (int64_t*)realloc(*pi, sizeof(int64_t) * (size_t)*cap);
              *pj = (int64_t*)realloc(*pj, sizeof(int64_t) * (size_t)*cap);
            }
            (*pi)[cnt] = i; (*pj)[cnt] = j; ++cnt;
          }
        }
  }
  grid_free(&g);
  return cnt;
}

/*
 * Settle n spheres of radii r (scaled by `shrink` during placement) from the
 * start positions x (in/out).  Each iteration shifts every sphere down by
 * `drop` (decaying linearly to zero over the first `settle_iters` iterations),
 * confines it to the region, then removes every pairwise overlap in one
 * Gauss-Seidel sweep over a Verlet pair list (each partner moves by its
 * share, split by volume, under-relaxed by `relax`).
 * Returns the largest remaining overlap relative to the smaller radius.
 */
double settle_packing(int64_t n, double* x, const double* r, int kind, const double* prm,
                      double shrink, int iters, int settle_iters, double drop, double relax) {
  double* rr = (double*)malloc(sizeof(double) * (size_t)n);
  double* tmp = (double*)malloc(sizeof(double) * (size_t)n);
  double* xref = (double*)malloc(sizeof(double) * 3 * (size_t)n);
  for (int64_t i = 0; i < n; ++i) { rr[i] = r[i] * shrink; tmp[i] = rr[i]; }
  qsort(tmp, (size_t)n, sizeof(double), cmpd);
  double rmed = tmp[n / 2];
  double h = 2.0 * rmed;
  double skin = 0.5 * rmed;
  int64_t *pi = NULL, *pj = NULL, cap = 0, np = 0;
  double cum = 0.0;
  int need = 1;
  double worst = 0.0;
  for (int it = 0; it < iters; ++it) {
    double dz = 0.0;
    if (it < settle_iters) dz = drop * (1.0 - (double)it / (double)settle_iters);
    cum += dz;
    for (int64_t i = 0; i < n; ++i) {
      x[3 * i + 2] -= dz;
      confine(kind, prm, rr[i], &x[3 * i]);
    }
    if (!need) {
      double m2 = 0.0;
      for (int64_t i = 0; i < n; ++i) {
        double d0 = x[3 * i] - xref[3 * i], d1 = x[3 * i + 1] - xref[3 * i + 1];
        double d2 = x[3 * i + 2] - (xref[3 * i + 2] - cum);
        double q = d0 * d0 + d1 * d1 + d2 * d2;
        if (q > m2) m2 = q;
      }
      if (m2 > 0.25 * skin * skin) need = 1;
    }
    if (need) {
      np = build_pairs(n, x, rr, h, skin, &pi, &pj, &cap);
      memcpy(xref, x, sizeof(double) * 3 * (size_t)n);
      cum = 0.0;
      need = 0;
    }
    worst = 0.0;
    for (int64_t k = 0; k < np; ++k) {
      int64_t i = pi[k], j = pj[k];
      double d[3], d2 = 0.0;
      for (int c = 0; c < 3; ++c) { d[c] = x[3 * j + c] - x[3 * i + c]; d2 += d[c] * d[c]; }
      double cc = rr[i] + rr[j];
      if (d2 >= cc * cc) continue;
      double dist = sqrt(d2);
      double ov = cc - dist;
      double rel = ov / (rr[j] < rr[i] ? rr[j] : rr[i]);
      if (rel > worst) worst = rel;
      double nn[3];
      if (dist > 0.0) { for (int c = 0; c < 3; ++c) nn[c] = d[c] / dist; }
      else { nn[0] = 0.0; nn[1] = 0.0; nn[2] = 1.0; }
      double vi = rr[i] * rr[i] * rr[i], vj = rr[j] * rr[j] * rr[j];
      double si = relax * ov * vj / (vi + vj), sj = relax * ov * vi / (vi + vj);
      for (int c = 0; c < 3; ++c) {
        x[3 * i + c] -= si * nn[c];
        x[3 * j + c] += sj * nn[c];
      }
    }
    for (int64_t i = 0; i < n; ++i) confine(kind, prm, rr[i], &x[3 * i]);
  }
  free(rr); free(tmp); free(xref); free(pi); free(pj);
  return worst;
}

/*
 * settle_packing_jacobi: the same settling as settle_packing for large n,
 * parallel (OpenMP) and deterministic for any thread count.  Each iteration
 * shifts every sphere down (as above), then removes overlaps by a Jacobi sweep:
 * every sphere gathers, over its own neighbour row (all spheres within
 * r_i + r_j + skin, found by a search of the grid cells around it, in a fixed
 * cell order), the displacement its share of each overlap asks for, and all
 * spheres then move at once by `relax` times their sum; then confinement.  Rows
 * are rebuilt when a sphere has moved more than half the skin.
 */
static void rows_build(int64_t n, const double* x, const double* rr, double rmax, double h, double skin,
                       int64_t** rowp, int64_t** cols, int64_t* cap) {
  grid_t g;
  grid_build(&g, n, x, h);
  int64_t* cnt = (int64_t*)calloc((size_t)n + 1, sizeof(int64_t));
  for (int pass = 0; pass < 2; ++pass) {
    if (pass == 1) {
      for (int64_t i = 0; i < n; ++i) cnt[i + 1] += cnt[i];
      if (cnt[n] > *cap) {
        *cap = cnt[n] + cnt[n] / 4 + 1024;
        *cols = (int64_t*)realloc(*cols, sizeof(int64_t) * (size_t)*cap);
      }
    }
#pragma omp parallel for schedule(dynamic, 1024)
    for (int64_t i = 0; i < n; ++i) {
      double R = rr[i] + rmax + skin;
      int64_t k0[3], k1[3];
      for (int c = 0; c < 3; ++c) {
        k0[c] = clampi((int64_t)floor((x[3 * i + c] - R - g.lo[c]) / h), 0, g.nc[c] - 1);
        k1[c] = clampi((int64_t)floor((x[3 * i + c] + R - g.lo[c]) / h), 0, g.nc[c] - 1);
      }
      int64_t at = pass == 1 ? cnt[i] : 0, m = 0;
      for (int64_t kz = k0[2]; kz <= k1[2]; ++kz)
        for (int64_t ky = k0[1]; ky <= k1[1]; ++ky)
          for (int64_t kx = k0[0]; kx <= k1[0]; ++kx) {
            int64_t cid = (kz * g.nc[1] + ky) * g.nc[0] + kx;
            for (int64_t q = g.start[cid]; q < g.start[cid + 1]; ++q) {
              int64_t j = g.idx[q];
              if (j == i) continue;
              double d2 = 0.0;
              for (int c = 0; c < 3; ++c) { double d = x[3 * j + c] - x[3 * i + c]; d2 += d * d; }
              double cc = rr[i] + rr[j] + skin;
              if (d2 >= cc * cc) continue;
              if (pass == 1) (*cols)[at + m] = j;
              ++m;
            }
          }
      if (pass == 0) cnt[i + 1] = m;
    }
  }
  free(*rowp);
  *rowp = cnt;
  grid_free(&g);
}

double settle_packing_jacobi(int64_t n, double* x, const double* r, int kind, const double* prm, double shrink,
                             int iters, int settle_iters, double drop, double relax) {
  double* rr = (double*)malloc(sizeof(double) * (size_t)n);
  double* tmp = (double*)malloc(sizeof(double) * (size_t)n);
  double* xref = (double*)malloc(sizeof(double) * 3 * (size_t)n);
  double* disp = (double*)malloc(sizeof(double) * 3 * (size_t)n);
  double rmax = 0.0;
  for (int64_t i = 0; i < n; ++i) {
    rr[i] = r[i] * shrink;
    tmp[i] = rr[i];
    if (rr[i] > rmax) rmax = rr[i];
  }
  qsort(tmp, (size_t)n, sizeof(double), cmpd);
  double rmed = tmp[n / 2];
  double h = 2.0 * rmed;
  double skin = 0.5 * rmed;
  int64_t *rowp = NULL, *cols = NULL, cap = 0;
  double cum = 0.0;
  int need = 1;
  double worst = 0.0;
  for (int it = 0; it < iters; ++it) {
    double dz = 0.0;
    if (it < settle_iters) dz = drop * (1.0 - (double)it / (double)settle_iters);
    cum += dz;
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n; ++i) {
      x[3 * i + 2] -= dz;
      confine(kind, prm, rr[i], &x[3 * i]);
    }
    if (!need) {
      double m2 = 0.0;
#pragma omp parallel for schedule(static) reduction(max : m2)
      for (int64_t i = 0; i < n; ++i) {
        double d0 = x[3 * i] - xref[3 * i], d1 = x[3 * i + 1] - xref[3 * i + 1];
        double d2 = x[3 * i + 2] - (xref[3 * i + 2] - cum);
        double q = d0 * d0 + d1 * d1 + d2 * d2;
        if (q > m2) m2 = q;
      }
      if (m2 > 0.25 * skin * skin) need = 1;
    }
    if (need) {
      rows_build(n, x, rr, rmax, h, skin, &rowp, &cols, &cap);
      memcpy(xref, x, sizeof(double) * 3 * (size_t)n);
      cum = 0.0;
      need = 0;
    }
    double w = 0.0;
#pragma omp parallel for schedule(dynamic, 1024) reduction(max : w)
    for (int64_t i = 0; i < n; ++i) {
      double s[3] = {0.0, 0.0, 0.0};
      double vi = rr[i] * rr[i] * rr[i];
      for (int64_t e = rowp[i]; e < rowp[i + 1]; ++e) {
        int64_t j = cols[e];
        double d[3], d2 = 0.0;
        for (int c = 0; c < 3; ++c) { d[c] = x[3 * j + c] - x[3 * i + c]; d2 += d[c] * d[c]; }
        double cc = rr[i] + rr[j];
        if (d2 >= cc * cc) continue;
        double dist = sqrt(d2);
        double ov = cc - dist;
        double rel = ov / (rr[j] < rr[i] ? rr[j] : rr[i]);
        if (rel > w) w = rel;
        double nn[3];
        if (dist > 0.0) { for (int c = 0; c < 3; ++c) nn[c] = d[c] / dist; }
        else { nn[0] = 0.0; nn[1] = 0.0; nn[2] = (i < j) ? 1.0 : -1.0; }
        double vj = rr[j] * rr[j] * rr[j];
        double si = ov * vj / (vi + vj);
        for (int c = 0; c < 3; ++c) s[c] -= si * nn[c];
      }
      for (int c = 0; c < 3; ++c) disp[3 * i + c] = s[c];
    }
    worst = w;
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n; ++i) {
      for (int c = 0; c < 3; ++c) x[3 * i + c] += relax * disp[3 * i + c];
      confine(kind, prm, rr[i], &x[3 * i]);
    }
  }
  free(rr); free(tmp); free(xref); free(disp); free(rowp); free(cols);
  return worst;
}

/* build_pairs in two parallel passes (counts per larger sphere, then the
 * pairs at their offsets): the same list in the same order */
static int64_t build_pairs_par(int64_t n, const double* x, const double* rr, double h, double skin,
                               int64_t** pi, int64_t** pj, int64_t* cap) {
  grid_t g;
  grid_build(&g, n, x, h);
  int64_t* cnt = (int64_t*)calloc((size_t)n + 1, sizeof(int64_t));
  for (int pass = 0; pass < 2; ++pass) {
    if (pass == 1) {
      for (int64_t i = 0; i < n; ++i) cnt[i + 1] += cnt[i];
      if (cnt[n] > *cap) {
        *cap = cnt[n] + cnt[n] / 4 + 1024;
        *pi = (int64_t*)realloc(*pi, sizeof(int64_t) * (size_t)*cap);
        *pj = (int64_t*)realloc(*pj, sizeof(int64_t) * (size_t)*cap);
      }
    }
#pragma omp parallel for schedule(dynamic, 1024)
    for (int64_t i = 0; i < n; ++i) {
      double R = 2.0 * rr[i] + skin;
      int64_t k0[3], k1[3];
      for (int c = 0; c < 3; ++c) {
        k0[c] = clampi((int64_t)floor((x[3 * i + c] - R - g.lo[c]) / h), 0, g.nc[c] - 1);
        k1[c] = clampi((int64_t)floor((x[3 * i + c] + R - g.lo[c]) / h), 0, g.nc[c] - 1);
      }
      int64_t at = pass == 1 ? cnt[i] : 0, m = 0;
      for (int64_t kz = k0[2]; kz <= k1[2]; ++kz)
        for (int64_t ky = k0[1]; ky <= k1[1]; ++ky)
          for (int64_t kx = k0[0]; kx <= k1[0]; ++kx) {
            int64_t cid = (kz * g.nc[1] + ky) * g.nc[0] + kx;
            for (int64_t q = g.start[cid]; q < g.start[cid + 1]; ++q) {
              int64_t j = g.idx[q];
              if (j == i) continue;
              if (rr[j] > rr[i] || (rr[j] == rr[i] && j < i)) continue;
              double d2 = 0.0;
              for (int c = 0; c < 3; ++c) { double d = x[3 * j + c] - x[3 * i + c]; d2 += d * d; }
              double cc = rr[i] + rr[j] + skin;
              if (d2 >= cc * cc) continue;
              if (pass == 1) { (*pi)[at + m] = i; (*pj)[at + m] = j; }
              ++m;
            }
          }
      if (pass == 0) cnt[i + 1] = m;
    }
  }
  int64_t np = cnt[n];
  free(cnt);
  grid_free(&g);
  return np;
}

/*
 * settle_packing_colored: settle_packing with the overlap sweep spread over
 * threads (OpenMP), still Gauss-Seidel (every correction sees the positions the
 * corrections before it left) and deterministic for any thread count.  At
 * every pair-list rebuild each pair goes to the block (a cube of side B, more
 * than the longest pair reach 2 r_max + skin) that holds its larger sphere, in
 * list order; a block's colour is its coordinates mod 3, and a sweep takes the
 * 27 colours in turn.  Two blocks of one colour are at least 2 B apart, so no
 * sphere is within reach of both: the spheres their pairs move are distinct
 * (the pairs are fixed between rebuilds), and the blocks of a colour run in
 * parallel, each through its pairs in list order.
 */
double settle_packing_colored(int64_t n, double* x, const double* r, int kind, const double* prm,
                              double shrink, int iters, int settle_iters, double drop, double relax) {
  double* rr = (double*)malloc(sizeof(double) * (size_t)n);
  double* tmp = (double*)malloc(sizeof(double) * (size_t)n);
  double* xref = (double*)malloc(sizeof(double) * 3 * (size_t)n);
  double rmax = 0.0;
  for (int64_t i = 0; i < n; ++i) {
    rr[i] = r[i] * shrink;
    tmp[i] = rr[i];
    if (rr[i] > rmax) rmax = rr[i];
  }
  qsort(tmp, (size_t)n, sizeof(double), cmpd);
  double rmed = tmp[n / 2];
  double h = 2.0 * rmed;
  double skin = 0.5 * rmed;
  double B = 1.05 * (2.0 * rmax + skin);
  int64_t *pi = NULL, *pj = NULL, cap = 0, np = 0;
  int64_t *si = NULL, *sj = NULL, *bstart = NULL, *cblk = NULL, ccnt[28];
  double cum = 0.0;
  int need = 1;
  double worst = 0.0;
  for (int it = 0; it < iters; ++it) {
    double dz = 0.0;
    if (it < settle_iters) dz = drop * (1.0 - (double)it / (double)settle_iters);
    cum += dz;
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n; ++i) {
      x[3 * i + 2] -= dz;
      confine(kind, prm, rr[i], &x[3 * i]);
    }
    if (!need) {
      double m2 = 0.0;
#pragma omp parallel for schedule(static) reduction(max : m2)
      for (int64_t i = 0; i < n; ++i) {
        double d0 = x[3 * i] - xref[3 * i], d1 = x[3 * i + 1] - xref[3 * i + 1];
        double d2 = x[3 * i + 2] - (xref[3 * i + 2] - cum);
        double q = d0 * d0 + d1 * d1 + d2 * d2;
        if (q > m2) m2 = q;
      }
      if (m2 > 0.25 * skin * skin) need = 1;
    }
    if (need) {
      np = build_pairs_par(n, x, rr, h, skin, &pi, &pj, &cap);
      memcpy(xref, x, sizeof(double) * 3 * (size_t)n);
      cum = 0.0;
      need = 0;
      // blocks of the larger spheres, a stable counting sort of the pairs by
      // block, and the non-empty blocks listed by colour
      double lo[3] = {1e300, 1e300, 1e300}, hi[3] = {-1e300, -1e300, -1e300};
      for (int64_t i = 0; i < n; ++i)
        for (int c = 0; c < 3; ++c) {
          if (x[3 * i + c] < lo[c]) lo[c] = x[3 * i + c];
          if (x[3 * i + c] > hi[c]) hi[c] = x[3 * i + c];
        }
      int64_t nb[3], tot = 1;
      for (int c = 0; c < 3; ++c) {
        nb[c] = (int64_t)floor((hi[c] - lo[c]) / B) + 1;
        tot *= nb[c];
      }
      int64_t* blk = (int64_t*)malloc(sizeof(int64_t) * (size_t)(np > 0 ? np : 1));
      free(bstart);
      bstart = (int64_t*)calloc((size_t)tot + 1, sizeof(int64_t));
      for (int64_t k = 0; k < np; ++k) {
        const double* p = &x[3 * pi[k]];
        int64_t b[3];
        for (int c = 0; c < 3; ++c) b[c] = clampi((int64_t)floor((p[c] - lo[c]) / B), 0, nb[c] - 1);
        blk[k] = (b[2] * nb[1] + b[1]) * nb[0] + b[0];
        bstart[blk[k] + 1]++;
      }
      for (int64_t b = 0; b < tot; ++b) bstart[b + 1] += bstart[b];
      free(si); free(sj);
      si = (int64_t*)malloc(sizeof(int64_t) * (size_t)(np > 0 ? np : 1));
      sj = (int64_t*)malloc(sizeof(int64_t) * (size_t)(np > 0 ? np : 1));
      {
        int64_t* at = (int64_t*)malloc(sizeof(int64_t) * (size_t)tot);
        memcpy(at, bstart, sizeof(int64_t) * (size_t)tot);
        for (int64_t k = 0; k < np; ++k) {
          int64_t q = at[blk[k]]++;
          si[q] = pi[k];
          sj[q] = pj[k];
        }
        free(at);
      }
      free(blk);
      free(cblk);
      cblk = (int64_t*)malloc(sizeof(int64_t) * (size_t)tot);
      int64_t m = 0;
      for (int col = 0; col < 27; ++col) {
        ccnt[col] = m;
        for (int64_t bz = col / 9; bz < nb[2]; bz += 3)
          for (int64_t by = (col / 3) % 3; by < nb[1]; by += 3)
            for (int64_t bx = col % 3; bx < nb[0]; bx += 3) {
              int64_t b = (bz * nb[1] + by) * nb[0] + bx;
              if (bstart[b + 1] > bstart[b]) cblk[m++] = b;
            }
      }
      ccnt[27] = m;
    }
    worst = 0.0;
    for (int col = 0; col < 27; ++col) {
      double w = 0.0;
#pragma omp parallel for schedule(dynamic, 4) reduction(max : w)
      for (int64_t q = ccnt[col]; q < ccnt[col + 1]; ++q) {
        const int64_t b = cblk[q];
        for (int64_t k = bstart[b]; k < bstart[b + 1]; ++k) {
          int64_t i = si[k], j = sj[k];
          double d[3], d2 = 0.0;
          for (int c = 0; c < 3; ++c) { d[c] = x[3 * j + c] - x[3 * i + c]; d2 += d[c] * d[c]; }
          double cc = rr[i] + rr[j];
          if (d2 >= cc * cc) continue;
          double dist = sqrt(d2);
          double ov = cc - dist;
          double rel = ov / (rr[j] < rr[i] ? rr[j] : rr[i]);
          if (rel > w) w = rel;
          double nn[3];
          if (dist > 0.0) { for (int c = 0; c < 3; ++c) nn[c] = d[c] / dist; }
          else { nn[0] = 0.0; nn[1] = 0.0; nn[2] = 1.0; }
          double vi = rr[i] * rr[i] * rr[i], vj = rr[j] * rr[j] * rr[j];
          double s_i = relax * ov * vj / (vi + vj), s_j = relax * ov * vi / (vi + vj);
          for (int c = 0; c < 3; ++c) {
            x[3 * i + c] -= s_i * nn[c];
            x[3 * j + c] += s_j * nn[c];
          }
        }
      }
      if (w > worst) worst = w;
    }
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n; ++i) confine(kind, prm, rr[i], &x[3 * i]);
  }
  free(rr); free(tmp); free(xref); free(pi); free(pj);
  free(si); free(sj); free(bstart); free(cblk);
  return worst;
}

/*
 * deep_overlaps: flags[k] = 1 for the smaller sphere (ties: the higher index)
 * of every pair whose overlap exceeds `thresh` times the smaller radius;
 * returns the number of flagged spheres.
 */
int64_t deep_overlaps(int64_t n, const double* x, const double* r, double thresh, uint8_t* flags) {
  double rmax = 0.0;
  for (int64_t i = 0; i < n; ++i) {
    flags[i] = 0;
    if (r[i] > rmax) rmax = r[i];
  }
  const double h = 2.0 * rmax;
  grid_t g;
  grid_build(&g, n, x, h);
#pragma omp parallel for schedule(dynamic, 1024)
  for (int64_t i = 0; i < n; ++i) {
    int64_t k0[3], k1[3];
    for (int c = 0; c < 3; ++c) {
      k0[c] = clampi((int64_t)floor((x[3 * i + c] - h - g.lo[c]) / h), 0, g.nc[c] - 1);
      k1[c] = clampi((int64_t)floor((x[3 * i + c] + h - g.lo[c]) / h), 0, g.nc[c] - 1);
    }
    for (int64_t kz = k0[2]; kz <= k1[2]; ++kz)
      for (int64_t ky = k0[1]; ky <= k1[1]; ++ky)
        for (int64_t kx = k0[0]; kx <= k1[0]; ++kx) {
          int64_t cid = (kz * g.nc[1] + ky) * g.nc[0] + kx;
          for (int64_t q = g.start[cid]; q < g.start[cid + 1]; ++q) {
            int64_t j = g.idx[q];
            // i is the smaller sphere of the pair (ties: the higher index)
            if (j == i || r[j] < r[i] || (r[j] == r[i] && j > i)) continue;
            double d2 = 0.0;
            for (int c = 0; c < 3; ++c) { double d = x[3 * j + c] - x[3 * i + c]; d2 += d * d; }
            double ov = r[i] + r[j] - sqrt(d2);
            if (ov > thresh * r[i]) flags[i] = 1;
          }
        }
  }
  grid_free(&g);
  int64_t m = 0;
  for (int64_t i = 0; i < n; ++i) m += flags[i];
  return m;
}
