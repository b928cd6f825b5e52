/*
 * dem_oracle.c -- plain FP64 CPU oracle of the coarse-grained CFD-DEM step.
 *
 * TEST INFRASTRUCTURE ONLY: used by tests/, by the smoke check and by the
 * cpu_baseline leg of the benchmark.  The product path never calls it.
 *
 * Sources (arXiv:2211.06142):
 *   Newton-Euler motion ............... section 2.1, eq 1-2
 *   tangential spring-dashpot-slider .. section 2.1, eq 4 (Coulomb cap, eq 35)
 *   contact torque .................... section 2.1, eq 5
 *   linear normal law (test mode) ..... section 2.1, eq 3
 *   particle drag, cell drag source ... section 2.2, eq 7-11
 *   modified JKR normal law ........... section 2.3, eq 12-13, Table 1, Fig. 2
 *   damping / restitution ............. section 2.4, eq 31-34
 *   coarse-grained drag ............... section 2.4, eq 21 (forces scale k^3 for
 *                                       body forces acting over the same time)
 * Everything the paper leaves open (integrator, tangential stiffness, void
 * fraction method, outlet) follows the readings listed in the design notes;
 * each appears below where it is used.
 *
 * Build: gcc -O2 -ffp-contract=off (no fused multiply-add, no fast-math).
 * parity unpinned: none of the functions here is unpinned; see tests/.
 */
#include "dem_oracle.h"
#include <math.h>
#include <stdlib.h>
#include <string.h>

#ifndef M_PI
#define M_PI 3.14159265358979323846
#endif

/* ------------------------------------------------------------------ */
/* small vector helpers                                                */
/* ------------------------------------------------------------------ */
static double dot3(const double* a, const double* b) { return (a[0] * b[0] + a[1] * b[1]) + a[2] * b[2]; }
static double norm3(const double* a) { return sqrt(dot3(a, a)); }
static void cross3(const double* a, const double* b, double* o) {
  o[0] = a[1] * b[2] - a[2] * b[1];
  o[1] = a[2] * b[0] - a[0] * b[2];
  o[2] = a[0] * b[1] - a[1] * b[0];
}

/* ------------------------------------------------------------------ */
/* modified JKR single-contact law (section 2.3)                       */
/* ------------------------------------------------------------------ */

/* eq 13: overlap as a function of the contact radius a */
double or_jkr_delta_of_a(double a, double Rs, double Es, double gamma) {
  return a * a / Rs - sqrt(4.0 * M_PI * gamma * a / Es);
}

/* eq 12: normal force (positive = repulsive) as a function of a */
double or_jkr_force_of_a(double a, double Rs, double Es, double gamma) {
  return 4.0 * Es * a * a * a / (3.0 * Rs) - sqrt(16.0 * M_PI * gamma * Es * a * a * a);
}

/* eq 13 inverted on its stable (increasing) branch.  delta(a) has its
 * minimum at a_S^3 = pi gamma R*^2 / (4 E*); every bonded state (delta at
 * or above the pull-off overlap of Table 1, point C) has a unique root
 * a >= a_S.  Plain bisection down to adjacent doubles. */
double or_jkr_a_of_delta(double delta, double Rs, double Es, double gamma) {
  if (gamma == 0.0) return delta > 0.0 ? sqrt(Rs * delta) : 0.0;
  double lo = cbrt(M_PI * gamma * Rs * Rs / (4.0 * Es));
  double hi = 2.0 * lo;
  while (or_jkr_delta_of_a(hi, Rs, Es, gamma) < delta) hi *= 2.0;
  for (;;) {
    double mid = 0.5 * (lo + hi);
    if (mid <= lo || mid >= hi) break;
    if (or_jkr_delta_of_a(mid, Rs, Es, gamma) < delta) lo = mid; else hi = mid;
  }
  double rl = fabs(or_jkr_delta_of_a(lo, Rs, Es, gamma) - delta);
  double rh = fabs(or_jkr_delta_of_a(hi, Rs, Es, gamma) - delta);
  return rl < rh ? lo : hi;
}

/* Bond persistence (Fig. 2: the bond breaks at point C, the pull-off point).
 * Table 1 gives delta_C = -(3/16)^(1/3) (pi^2 gamma^2 R* / E*^2)^(1/3); the
 * test is written with cubes so that no cube root enters a decision:
 * bonded iff delta > 0, or (-delta)^3 <= (3/16) pi^2 gamma^2 R* / E*^2.
 * delta equal to delta_C stays bonded. */
int or_bond_holds(double d2, double c, double Rs, double Es, double gamma) {
  if (d2 < c * c) return 1;
  double sep = sqrt(d2) - c;
  double lhs = (sep * sep) * sep;
  double rhs = (((3.0 / 16.0) * (M_PI * M_PI)) * (gamma * gamma)) * Rs / (Es * Es);
  return lhs <= rhs;
}

/* Original JKR (section 2.3, Fig. 1): the contact lasts down to point S, the
 * smallest overlap of eq 13, where d(delta)/da = 0: a_S^3 = pi gamma R*^2 /
 * (4 E*), which gives delta_S = -3 (1/16)^(1/3) (pi^2 gamma^2 R* / E*^2)^(1/3),
 * i.e. (-delta_S)^3 = (27/16) pi^2 gamma^2 R* / E*^2.  Written with cubes, as
 * the bond test above; delta equal to delta_S holds. */
int or_contact_holds_to_S(double d2, double c, double Rs, double Es, double gamma) {
  if (d2 < c * c) return 1;
  double sep = sqrt(d2) - c;
  double lhs = (sep * sep) * sep;
  double rhs = (((27.0 / 16.0) * (M_PI * M_PI)) * (gamma * gamma)) * Rs / (Es * Es);
  return lhs <= rhs;
}

/* Critical damping ratio from the restitution coefficient (eq 33, with the
 * square on ln e that the printed equation drops). */
double or_beta_of_e(double e) {
  double l = log(e);
  return -l / sqrt(l * l + M_PI * M_PI);
}

/* ------------------------------------------------------------------ */
/* Di Felice drag (section 2.2, eq 8-11) with the coarse-grained rule    */
/* ------------------------------------------------------------------ */
/* s = u - v (slip), d = particle (grain) diameter, k_cg = coarse-grain factor:
 * the grain feels k^3 times the drag of a fine particle of diameter d/k under
 * the same slip and porosity (eq 21: the body force on a grain acts over the
 * same time as on the k^3 particles it stands for). */
void or_drag(const double s[3], double d, double k_cg, double n, double rho_f, double mu_f,
             double c_drag, double out_f[3]) {
  double sm = norm3(s);
  if (sm == 0.0) { out_f[0] = out_f[1] = out_f[2] = 0.0; return; }
  double de = d / k_cg;
  double Re = rho_f * de * sm / mu_f;                              /* eq 11 */
  double cd = 0.63 + 4.8 / sqrt(Re);
  double Cd = cd * cd;                                             /* eq 9 */
  double lg = 1.5 - log10(Re);
  double chi = 3.7 - 0.65 * exp(-(lg * lg) / 2.0);                 /* eq 10 */
  double coef = 0.125 * Cd * rho_f * M_PI * de * de * sm * pow(n, -chi); /* eq 8 */
  double k3 = k_cg * k_cg * k_cg;
  for (int c = 0; c < 3; ++c) out_f[c] = k3 * coef * s[c] * c_drag;
}

/* ------------------------------------------------------------------ */
/* contact sets                                                         */
/* ------------------------------------------------------------------ */
static int pair_pred(const double* x, const double* r, int64_t i, int64_t j, double extra) {
  double dx = x[3 * j + 0] - x[3 * i + 0];
  double dy = x[3 * j + 1] - x[3 * i + 1];
  double dz = x[3 * j + 2] - x[3 * i + 2];
  double d2 = (dx * dx + dy * dy) + dz * dz;
  double c = (r[i] + r[j]) + extra;
  return d2 < c * c;
}

int64_t or_pairs_brute(int64_t n, const double* x, const double* r, const uint8_t* alive,
                       double extra, int64_t cap, int64_t* pi, int64_t* pj) {
  int64_t cnt = 0;
  for (int64_t i = 0; i < n; ++i) {
    if (alive && !alive[i]) continue;
    for (int64_t j = i + 1; j < n; ++j) {
      if (alive && !alive[j]) continue;
      if (pair_pred(x, r, i, j, extra)) {
        if (cnt < cap) { pi[cnt] = i; pj[cnt] = j; }
        ++cnt;
      }
    }
  }
  return cnt;
}

typedef struct { int64_t i, j; } ipair;
static int cmp_ipair(const void* a, const void* b) {
  const ipair* p = (const ipair*)a; const ipair* q = (const ipair*)b;
  if (p->i != q->i) return p->i < q->i ? -1 : 1;
  if (p->j != q->j) return p->j < q->j ? -1 : 1;
  return 0;
}

/* Plain uniform grid: cell side >= the largest cutoff, 27 neighbouring
 * cells, result sorted by (i, j).  Must equal or_pairs_brute. */
static int64_t pairs_grid_alloc(int64_t n, const double* x, const double* r, const uint8_t* alive,
                                double extra, ipair** out) {
  *out = NULL;
  double lo[3] = {1e300, 1e300, 1e300}, hi[3] = {-1e300, -1e300, -1e300}, rmax = 0.0;
  int64_t nal = 0;
  for (int64_t i = 0; i < n; ++i) {
    if (alive && !alive[i]) continue;
    ++nal;
    for (int c = 0; c < 3; ++c) {
      if (x[3 * i + c] < lo[c]) lo[c] = x[3 * i + c];
      if (x[3 * i + c] > hi[c]) hi[c] = x[3 * i + c];
    }
    if (r[i] > rmax) rmax = r[i];
  }
  if (nal < 2) return 0;
  double h = 2.0 * rmax + extra;
  h *= 1.0001;
  int64_t nc[3], ncell;
  /* coarsen the grid if the particles are spread far apart */
  for (;;) {
    for (int c = 0; c < 3; ++c) {
      double q = floor((hi[c] - lo[c]) / h) + 1.0;
      nc[c] = q > 4096.0 ? 4096 : (int64_t)q;
    }
    ncell = nc[0] * nc[1] * nc[2];
    if (ncell <= 8 * nal + 64) break;
    h *= 2.0;
  }
  int64_t* head = (int64_t*)malloc(sizeof(int64_t) * ncell);
  int64_t* next = (int64_t*)malloc(sizeof(int64_t) * n);
  int64_t* cell = (int64_t*)malloc(sizeof(int64_t) * n);
  for (int64_t c = 0; c < ncell; ++c) head[c] = -1;
  /* insert in decreasing index order so that every list runs in increasing index order */
  for (int64_t i = n - 1; i >= 0; --i) {
    if (alive && !alive[i]) { cell[i] = -1; continue; }
    int64_t ci[3];
    for (int c = 0; c < 3; ++c) {
      int64_t k = (int64_t)floor((x[3 * i + c] - lo[c]) / h);
      if (k < 0) k = 0;
      if (k >= nc[c]) k = nc[c] - 1;
      ci[c] = k;
    }
    int64_t id = (ci[2] * nc[1] + ci[1]) * nc[0] + ci[0];
    cell[i] = id;
    next[i] = head[id];
    head[id] = i;
  }
  int64_t cap = 1024, cnt = 0;
  ipair* buf = (ipair*)malloc(sizeof(ipair) * cap);
  for (int64_t i = 0; i < n; ++i) {
    if (cell[i] < 0) continue;
    int64_t cz = cell[i] / (nc[0] * nc[1]);
    int64_t cy = (cell[i] / nc[0]) % nc[1];
    int64_t cx = cell[i] % nc[0];
    for (int64_t dz = -1; dz <= 1; ++dz)
      for (int64_t dy = -1; dy <= 1; ++dy)
        for (int64_t dx = -1; dx <= 1; ++dx) {
          int64_t qx = cx + dx, qy = cy + dy, qz = cz + dz;
          if (qx < 0 || qy < 0 || qz < 0 || qx >= nc[0] || qy >= nc[1] || qz >= nc[2]) continue;
          for (int64_t j = head[(qz * nc[1] + qy) * nc[0] + qx]; j >= 0; j = next[j]) {
            if (j <= i) continue;
            if (pair_pred(x, r, i, j, extra)) {
              if (cnt == cap) { cap *= 2; buf = (ipair*)realloc(buf, sizeof(ipair) * cap); }
              buf[cnt].i = i; buf[cnt].j = j; ++cnt;
            }
          }
        }
  }
  free(head); free(next); free(cell);
  qsort(buf, (size_t)cnt, sizeof(ipair), cmp_ipair);
  *out = buf;
  return cnt;
}

int64_t or_pairs_grid(int64_t n, const double* x, const double* r, const uint8_t* alive,
                      double extra, int64_t cap, int64_t* pi, int64_t* pj) {
  ipair* buf;
  int64_t cnt = pairs_grid_alloc(n, x, r, alive, extra, &buf);
  for (int64_t k = 0; k < cnt && k < cap; ++k) { pi[k] = buf[k].i; pj[k] = buf[k].j; }
  free(buf);
  return cnt;
}

/* ------------------------------------------------------------------ */
/* simulation state                                                     */
/* ------------------------------------------------------------------ */
typedef struct {
  int64_t i, j;
  double dt[3];     /* tangential spring elongation, orientation i -> j */
  uint8_t bonded;
  uint8_t touch;    /* took part in the last force evaluation */
} hrec;

struct or_sim {
  or_params p;
  int64_t n;
  double *x, *v, *w, *F, *T, *r, *m, *I;
  double *fscale, *tscale;
  uint8_t* alive;
  hrec* h; int64_t nh;
  double* wall_dt;
  double wall_force[3 * OR_MAX_WALLS];   /* the particles' force on each wall, last evaluation */
  double *fdrag, *fbuoy;          /* particle coupling forces held between coupling steps */
  double *u_cell, *gp_cell; int have_fluid;
  double *eps_cell, *fd_cell;
  double *c_drag, *c_coh;
  double* mlp;                    /* closure network parameters (NULL: off) */
  double* cfeat;                  /* n x 6 features of the latest closure evaluation */
  double mlp_norm[12];            /* feature mean[6], standard deviation[6] */
  double Es, Gs, beta;
  double produced;
  int64_t broken, step;
};

static int cmp_hrec(const void* a, const void* b) {
  const hrec* p = (const hrec*)a; const hrec* q = (const hrec*)b;
  if (p->i != q->i) return p->i < q->i ? -1 : 1;
  if (p->j != q->j) return p->j < q->j ? -1 : 1;
  return 0;
}

static hrec* find_h(hrec* h, int64_t nh, int64_t i, int64_t j) {
  int64_t lo = 0, hi = nh;
  while (lo < hi) {
    int64_t mid = (lo + hi) / 2;
    if (h[mid].i < i || (h[mid].i == i && h[mid].j < j)) lo = mid + 1; else hi = mid;
  }
  if (lo < nh && h[lo].i == i && h[lo].j == j) return &h[lo];
  return NULL;
}

static double* dup(const double* a, int64_t n) {
  double* o = (double*)calloc((size_t)(n > 0 ? n : 1), sizeof(double));
  if (a) memcpy(o, a, sizeof(double) * n);
  return o;
}

static int64_t ncells(const or_sim* s) { return (int64_t)s->p.grid.n[0] * s->p.grid.n[1] * s->p.grid.n[2]; }

or_sim* or_create(const or_params* p, int64_t n, const double* x, const double* v,
                  const double* w, const double* F, const double* T, const double* r,
                  const uint8_t* alive,
                  int64_t npairs, const int64_t* pi, const int64_t* pj,
                  const double* pdt, const uint8_t* pbond, int bond_at_init,
                  const double* wall_dt) {
  or_sim* s = (or_sim*)calloc(1, sizeof(or_sim));
  s->p = *p;
  s->n = n;
  s->x = dup(x, 3 * n); s->v = dup(v, 3 * n); s->w = dup(w, 3 * n);
  s->F = dup(F, 3 * n); s->T = dup(T, 3 * n); s->r = dup(r, n);
  s->fscale = dup(NULL, n); s->tscale = dup(NULL, n);
  s->m = dup(NULL, n); s->I = dup(NULL, n);
  s->alive = (uint8_t*)calloc((size_t)(n > 0 ? n : 1), 1);
  for (int64_t i = 0; i < n; ++i) {
    s->alive[i] = alive ? alive[i] : 1;
    /* eq 20: m = rho V with the grain's own radius; solid sphere inertia */
    s->m[i] = p->rho * (4.0 / 3.0) * M_PI * r[i] * r[i] * r[i];
    s->I[i] = 0.4 * s->m[i] * r[i] * r[i];
  }
  s->Es = p->E / (2.0 * (1.0 - p->nu * p->nu));
  s->Gs = p->E / (4.0 * (2.0 - p->nu) * (1.0 + p->nu));
  s->beta = or_beta_of_e(p->e);
  s->wall_dt = dup(wall_dt, 3 * n * (p->n_walls > 0 ? p->n_walls : 1));
  s->fdrag = dup(NULL, 3 * n); s->fbuoy = dup(NULL, 3 * n);
  int64_t nc = ncells(s);
  s->u_cell = dup(NULL, 3 * nc); s->gp_cell = dup(NULL, 3 * nc);
  s->eps_cell = dup(NULL, nc); s->fd_cell = dup(NULL, 3 * nc);
  s->c_drag = NULL; s->c_coh = NULL;
  if (npairs > 0) {
    s->h = (hrec*)calloc((size_t)npairs, sizeof(hrec));
    for (int64_t k = 0; k < npairs; ++k) {
      int64_t a = pi[k], b = pj[k];
      double sg = 1.0;
      if (a > b) { int64_t t = a; a = b; b = t; sg = -1.0; }
      s->h[k].i = a; s->h[k].j = b;
      for (int c = 0; c < 3; ++c) s->h[k].dt[c] = pdt ? sg * pdt[3 * k + c] : 0.0;
      s->h[k].bonded = pbond ? pbond[k] : 0;
      if (p->normal_model != OR_NORMAL_JKR_MOD && p->normal_model != OR_NORMAL_JKR_ORIG) s->h[k].bonded = 0;
    }
    s->nh = npairs;
    qsort(s->h, (size_t)s->nh, sizeof(hrec), cmp_hrec);
  } else if (bond_at_init && (p->normal_model == OR_NORMAL_JKR_MOD || p->normal_model == OR_NORMAL_JKR_ORIG)) {
    /* every touching pair (delta > 0) starts bonded */
    ipair* buf;
    int64_t cnt = pairs_grid_alloc(n, s->x, s->r, s->alive, 0.0, &buf);
    s->h = (hrec*)calloc((size_t)(cnt > 0 ? cnt : 1), sizeof(hrec));
    for (int64_t k = 0; k < cnt; ++k) { s->h[k].i = buf[k].i; s->h[k].j = buf[k].j; s->h[k].bonded = 1; }
    s->nh = cnt;
    free(buf);
  }
  return s;
}

void or_destroy(or_sim* s) {
  if (!s) return;
  free(s->x); free(s->v); free(s->w); free(s->F); free(s->T); free(s->r);
  free(s->fscale); free(s->tscale); free(s->m); free(s->I); free(s->alive);
  free(s->h); free(s->wall_dt); free(s->fdrag); free(s->fbuoy);
  free(s->u_cell); free(s->gp_cell); free(s->eps_cell); free(s->fd_cell);
  free(s->c_drag); free(s->c_coh); free(s->mlp); free(s->cfeat);
  free(s);
}

int or_set_fluid(or_sim* s, const double* u_cell, const double* gradp_cell) {
  int64_t nc = ncells(s);
  memcpy(s->u_cell, u_cell, sizeof(double) * 3 * nc);
  memcpy(s->gp_cell, gradp_cell, sizeof(double) * 3 * nc);
  s->have_fluid = 1;
  return 0;
}

int or_set_held(or_sim* s, int64_t step, const double* fluid_force) {
  s->step = step;
  for (int64_t k = 0; k < 3 * s->n; ++k) {
    s->fdrag[k] = fluid_force ? fluid_force[k] : 0.0;
    s->fbuoy[k] = 0.0;
  }
  return 0;
}

int or_set_closure(or_sim* s, const double* c_drag, const double* c_coh) {
  free(s->c_drag); free(s->c_coh);
  s->c_drag = c_drag ? dup(c_drag, s->n) : NULL;
  s->c_coh = c_coh ? dup(c_coh, s->n) : NULL;
  return 0;
}

/* ------------------------------------------------------------------ */
/* the contact law for one contact                                      */
/* ------------------------------------------------------------------ */
/* Inputs: normal model, bonded flag, overlap delta, effective radius and
 * mass, surface energy of the contact, unit normal n (from i towards the
 * other body), relative contact-point velocity vrel of i w.r.t. the other
 * body, relative angular velocity wrel, and the tangential history dt.
 * Outputs: force on i, c = n x F_t (torque on body b is r_b * c), rolling
 * torque on i, scale = sum of the magnitudes of every force term. */
typedef struct { double F[3], c[3], Tr[3], scale, tscale_t, tscale_roll; } law_out;

static void contact_law(const or_sim* s, int bonded, double delta, double Rs, double ms, double gam,
                        const double* n, const double* vrel, const double* wrel, double* dt,
                        law_out* o) {
  const or_params* p = &s->p;
  double Es = s->Es, Gs = s->Gs, beta = s->beta;
  double a, Fel, kn, kt, etan, etat, L, scale;
  if (p->normal_model == OR_NORMAL_LINEAR) {
    /* eq 3 with a constant spring; critical-damping form gives COR = e */
    a = 0.0;
    kn = p->k_lin;
    Fel = kn * delta;
    kt = (2.0 / 7.0) * kn;
    etan = 2.0 * beta * sqrt(kn * ms);
    etat = 2.0 * beta * sqrt(kt * ms);
    L = p->mu * Fel;
    scale = fabs(Fel);
  } else {
    if (bonded) {
      a = or_jkr_a_of_delta(delta, Rs, Es, gam);                   /* eq 13 */
      Fel = or_jkr_force_of_a(a, Rs, Es, gam);                     /* eq 12 */
      scale = fabs(4.0 * Es * a * a * a / (3.0 * Rs)) + fabs(sqrt(16.0 * M_PI * gam * Es * a * a * a));
      L = p->mu * (Fel + 2.0 * (3.0 * M_PI * gam * Rs));           /* eq 35, shifted by the pull-off force */
    } else {
      a = sqrt(Rs * delta);                                        /* Hertz: eq 12-13 with gamma = 0 */
      Fel = 4.0 * Es * a * a * a / (3.0 * Rs);
      scale = fabs(Fel);
      L = p->mu * Fel;
    }
    kn = 2.0 * Es * a;
    kt = 8.0 * Gs * a;
    /* eq 32: -beta sqrt(20/3 E* a m*) u_n = -2 sqrt(5/6) beta sqrt(k_n m*) u_n */
    etan = 2.0 * sqrt(5.0 / 6.0) * beta * sqrt(kn * ms);
    etat = 2.0 * sqrt(5.0 / 6.0) * beta * sqrt(kt * ms);
  }
  double vn = dot3(vrel, n);
  double vt[3];
  for (int c = 0; c < 3; ++c) vt[c] = vrel[c] - vn * n[c];
  double Fn = Fel + etan * vn;
  for (int c = 0; c < 3; ++c) o->F[c] = -Fn * n[c];
  scale += fabs(etan * vn);

  /* tangential spring (eq 4): rotate the stored elongation into the current
   * tangent plane keeping its length, then add the tangential slip of this step */
  double old = norm3(dt);
  double dn = dot3(dt, n);
  double tp[3];
  for (int c = 0; c < 3; ++c) tp[c] = dt[c] - dn * n[c];
  double tpl = norm3(tp);
  if (tpl > 0.0) { for (int c = 0; c < 3; ++c) dt[c] = tp[c] * (old / tpl); }
  else { dt[0] = dt[1] = dt[2] = 0.0; }
  /* magnitudes of the terms entering F_t: spring on the carried elongation,
   * spring and dashpot on this step's slip (which itself is v_rel minus its
   * normal part) */
  double tsc = kt * norm3(dt) + (kt * p->dt + etat) * norm3(vrel);
  for (int c = 0; c < 3; ++c) dt[c] += vt[c] * p->dt;
  double Ft[3];
  for (int c = 0; c < 3; ++c) Ft[c] = -kt * dt[c] - etat * vt[c];
  double ftm = norm3(Ft);
  if (ftm > L) {
    /* Coulomb slider: cap the force, reset the spring to the capped value */
    double sc = L / ftm;
    for (int c = 0; c < 3; ++c) Ft[c] = Ft[c] * sc;
    if (kt > 0.0) { for (int c = 0; c < 3; ++c) dt[c] = -(Ft[c] + etat * vt[c]) / kt; }
    else { dt[0] = dt[1] = dt[2] = 0.0; }
  }
  for (int c = 0; c < 3; ++c) o->F[c] += Ft[c];
  scale += tsc;
  o->tscale_t = tsc;
  cross3(n, Ft, o->c);                                              /* eq 5 */

  /* optional rolling resistance (constant directional torque) */
  o->Tr[0] = o->Tr[1] = o->Tr[2] = 0.0;
  o->tscale_roll = 0.0;
  if (p->mu_roll > 0.0) {
    double wn = dot3(wrel, n);
    double wr[3];
    for (int c = 0; c < 3; ++c) wr[c] = wrel[c] - wn * n[c];
    double wm = norm3(wr);
    if (wm > 0.0) {
      double tm = p->mu_roll * Rs * fabs(Fel);
      for (int c = 0; c < 3; ++c) o->Tr[c] = -tm * wr[c] / wm;
      o->tscale_roll = tm;
    }
  }
  o->scale = scale;
}

/* ------------------------------------------------------------------ */
/* fluid coupling (section 2.2)                                         */
/* ------------------------------------------------------------------ */
/* Trilinear (cloud-in-cell) weights of a point w.r.t. the cell centres.
 * Positions outside the hull of the cell centres are projected onto it, so
 * that weight beyond the grid folds into the boundary cells. */
static void cic(const or_grid* g, const double* x, int64_t base[3], double f[3]) {
  for (int c = 0; c < 3; ++c) {
    double h = (g->hi[c] - g->lo[c]) / g->n[c];
    double t = (x[c] - g->lo[c]) / h - 0.5;
    double tmax = (double)(g->n[c] - 1);
    if (t < 0.0) t = 0.0;
    if (t > tmax) t = tmax;
    int64_t b = (int64_t)floor(t);
    if (g->n[c] >= 2 && b > g->n[c] - 2) b = g->n[c] - 2;
    if (g->n[c] == 1) b = 0;
    base[c] = b;
    f[c] = t - (double)b;
  }
}

/* visit the (up to 8) cells a particle touches with their weights */
typedef struct { int64_t cell[8]; double w[8]; int cnt; } cellw;
static void particle_cells(const or_sim* s, const double* x, cellw* o) {
  const or_grid* g = &s->p.grid;
  o->cnt = 0;
  if (s->p.voidfrac == OR_VOID_CENTROID) {
    int64_t k[3];
    for (int c = 0; c < 3; ++c) {
      double h = (g->hi[c] - g->lo[c]) / g->n[c];
      int64_t b = (int64_t)floor((x[c] - g->lo[c]) / h);
      if (b < 0) b = 0;
      if (b > g->n[c] - 1) b = g->n[c] - 1;
      k[c] = b;
    }
    o->cell[0] = (k[2] * g->n[1] + k[1]) * g->n[0] + k[0];
    o->w[0] = 1.0;
    o->cnt = 1;
    return;
  }
  int64_t b[3]; double f[3];
  cic(g, x, b, f);
  for (int dz = 0; dz < 2; ++dz)
    for (int dy = 0; dy < 2; ++dy)
      for (int dx = 0; dx < 2; ++dx) {
        int64_t kx = b[0] + dx, ky = b[1] + dy, kz = b[2] + dz;
        if (kx >= g->n[0] || ky >= g->n[1] || kz >= g->n[2]) continue;
        double wx = dx ? f[0] : 1.0 - f[0];
        double wy = dy ? f[1] : 1.0 - f[1];
        double wz = dz ? f[2] : 1.0 - f[2];
        o->cell[o->cnt] = (kz * g->n[1] + ky) * g->n[0] + kx;
        o->w[o->cnt] = (wx * wy) * wz;
        o->cnt++;
      }
}

static double cell_volume(const or_sim* s) {
  const or_grid* g = &s->p.grid;
  return ((g->hi[0] - g->lo[0]) / g->n[0]) * ((g->hi[1] - g->lo[1]) / g->n[1]) *
         ((g->hi[2] - g->lo[2]) / g->n[2]);
}

/* solid volume fraction per cell (porosity n of eq 6 is 1 - eps), clamped
 * porosity and interstitial fluid velocity per cell */
static void porosity_fields(or_sim* s, double* ncell, double* ucell) {
  const or_params* p = &s->p;
  int64_t nc = ncells(s);
  double vcell = cell_volume(s);
  for (int64_t c = 0; c < nc; ++c) s->eps_cell[c] = 0.0;
  for (int64_t i = 0; i < s->n; ++i) {
    if (!s->alive[i]) continue;
    double V = (4.0 / 3.0) * M_PI * s->r[i] * s->r[i] * s->r[i];
    cellw cw; particle_cells(s, &s->x[3 * i], &cw);
    for (int k = 0; k < cw.cnt; ++k) s->eps_cell[cw.cell[k]] += cw.w[k] * V;
  }
  for (int64_t c = 0; c < nc; ++c) s->eps_cell[c] /= vcell;
  for (int64_t c = 0; c < nc; ++c) {
    double nn = 1.0 - s->eps_cell[c];
    if (nn < p->n_min) nn = p->n_min;
    if (nn > 1.0) nn = 1.0;
    ncell[c] = nn;
    for (int k = 0; k < 3; ++k) ucell[3 * c + k] = p->u_superficial ? s->u_cell[3 * c + k] / nn : s->u_cell[3 * c + k];
  }
}

/* porosity, fluid velocity and dynamic pressure gradient at particle i (the
 * same cell weights as the deposition) */
static void particle_fluid(const or_sim* s, int64_t i, const double* ncell, const double* ucell, double* np,
                           double u[3], double gp[3]) {
  cellw cw; particle_cells(s, &s->x[3 * i], &cw);
  *np = 0.0;
  for (int c = 0; c < 3; ++c) { u[c] = 0.0; gp[c] = 0.0; }
  for (int k = 0; k < cw.cnt; ++k) {
    *np += cw.w[k] * ncell[cw.cell[k]];
    for (int c = 0; c < 3; ++c) {
      u[c] += cw.w[k] * ucell[3 * cw.cell[k] + c];
      gp[c] += cw.w[k] * s->gp_cell[3 * cw.cell[k] + c];
    }
  }
}

/* ------------------------------------------------------------------ */
/* learned closure (an extension; not in the paper)                     */
/* ------------------------------------------------------------------ */
/* Features of particle i: porosity at the particle, slip speed |u - v|, the
 * particle Reynolds number of the drag law (eq 11, fine diameter d/k), the
 * coarse-graining factor k, the mean of delta/R* over the pairs that took part
 * in the last force evaluation (delta = r_i + r_j - |x_j - x_i| at the current
 * positions) and the number of those pairs.  Dead particles: all zero. */
static void closure_features(const or_sim* s, const double* ncell, const double* ucell, double* feat) {
  const or_params* p = &s->p;
  int64_t n = s->n;
  double* sum = (double*)calloc((size_t)(n > 0 ? n : 1), sizeof(double));
  double* cnt = (double*)calloc((size_t)(n > 0 ? n : 1), sizeof(double));
  for (int64_t k = 0; k < s->nh; ++k) {
    int64_t i = s->h[k].i, j = s->h[k].j;
    if (!s->alive[i] || !s->alive[j]) continue;
    double dx[3];
    for (int c = 0; c < 3; ++c) dx[c] = s->x[3 * j + c] - s->x[3 * i + c];
    double delta = (s->r[i] + s->r[j]) - norm3(dx);
    double Rs = s->r[i] * s->r[j] / (s->r[i] + s->r[j]);
    sum[i] += delta / Rs; sum[j] += delta / Rs;
    cnt[i] += 1.0; cnt[j] += 1.0;
  }
  for (int64_t i = 0; i < n; ++i) {
    double* f = &feat[6 * i];
    for (int c = 0; c < 6; ++c) f[c] = 0.0;
    if (!s->alive[i]) continue;
    double np, u[3], gp[3];
    particle_fluid(s, i, ncell, ucell, &np, u, gp);
    double sl[3];
    for (int c = 0; c < 3; ++c) sl[c] = u[c] - s->v[3 * i + c];
    double sm = norm3(sl);
    f[0] = np;
    f[1] = sm;
    f[2] = p->rho_f * (2.0 * s->r[i] / p->k_cg) * sm / p->mu_f;
    f[3] = p->k_cg;
    f[4] = cnt[i] > 0.0 ? sum[i] / cnt[i] : 0.0;
    f[5] = cnt[i];
  }
  free(sum); free(cnt);
}

static double gelu(double x) { return 0.5 * x * (1.0 + erf(x / sqrt(2.0))); }

/* network 6 -> 64 -> 64 -> 64 -> 2, GELU on the hidden layers; flat parameters
 * W1 6x64 | b1 | W2 64x64 | b2 | W3 64x64 | b3 | W4 64x2 | b4, W[k][m] row-major */
void or_mlp_forward(const double* prm, const double* xh, double* y) {
  static const int sz[5] = {6, 64, 64, 64, 2};
  double h[64], z[64];
  for (int k = 0; k < 6; ++k) h[k] = xh[k];
  const double* q = prm;
  for (int l = 0; l < 4; ++l) {
    int K = sz[l], M = sz[l + 1];
    const double* W = q;
    const double* b = q + K * M;
    for (int m = 0; m < M; ++m) {
      double acc = 0.0;
      for (int k = 0; k < K; ++k) acc += h[k] * W[k * M + m];
      z[m] = acc + b[m];
    }
    for (int m = 0; m < M; ++m) h[m] = l < 3 ? gelu(z[m]) : z[m];
    q += K * M + M;
  }
  y[0] = h[0];
  y[1] = h[1];
}

/* closure factors c = exp(clip(y, -ln 2, ln 2)) of every particle */
static void closure_apply(or_sim* s, const double* ncell, const double* ucell) {
  int64_t n = s->n;
  if (!s->cfeat) s->cfeat = dup(NULL, 6 * n);
  double* feat = s->cfeat;
  closure_features(s, ncell, ucell, feat);
  if (!s->c_drag) s->c_drag = dup(NULL, n);
  if (!s->c_coh) s->c_coh = dup(NULL, n);
  const double L2 = log(2.0);
  for (int64_t i = 0; i < n; ++i) {
    double xh[6], y[2];
    for (int c = 0; c < 6; ++c) xh[c] = (feat[6 * i + c] - s->mlp_norm[c]) / s->mlp_norm[6 + c];
    or_mlp_forward(s->mlp, xh, y);
    for (int c = 0; c < 2; ++c) {
      if (y[c] < -L2) y[c] = -L2;
      if (y[c] > L2) y[c] = L2;
    }
    s->c_drag[i] = exp(y[0]);
    s->c_coh[i] = exp(y[1]);
  }
}

int or_set_closure_mlp(or_sim* s, const double* params, const double* norm) {
  free(s->mlp);
  s->mlp = NULL;
  if (!params) return 0;
  s->mlp = dup(params, OR_MLP_NPARAMS);
  for (int c = 0; c < 12; ++c) s->mlp_norm[c] = norm[c];
  return 0;
}

void or_get_closure_features(const or_sim* s, double* feat) {
  for (int64_t k = 0; k < 6 * s->n; ++k) feat[k] = s->cfeat ? s->cfeat[k] : 0.0;
}

void or_get_closure(const or_sim* s, double* c_drag, double* c_coh) {
  for (int64_t i = 0; i < s->n; ++i) {
    c_drag[i] = s->c_drag ? s->c_drag[i] : 1.0;
    c_coh[i] = s->c_coh ? s->c_coh[i] : 1.0;
  }
}

int or_closure_features(or_sim* s, double* feat) {
  int64_t nc = ncells(s);
  double* ncell = (double*)malloc(sizeof(double) * (nc > 0 ? nc : 1));
  double* ucell = (double*)malloc(sizeof(double) * 3 * (nc > 0 ? nc : 1));
  porosity_fields(s, ncell, ucell);
  closure_features(s, ncell, ucell, feat);
  free(ncell); free(ucell);
  return 0;
}

static void coupling(or_sim* s) {
  const or_params* p = &s->p;
  int64_t nc = ncells(s);
  double vcell = cell_volume(s);
  double* ncell = (double*)malloc(sizeof(double) * nc);
  double* ucell = (double*)malloc(sizeof(double) * 3 * nc);
  porosity_fields(s, ncell, ucell);
  if (s->mlp) closure_apply(s, ncell, ucell);
  for (int64_t c = 0; c < 3 * nc; ++c) s->fd_cell[c] = 0.0;
  for (int64_t i = 0; i < s->n; ++i) {
    for (int k = 0; k < 3; ++k) { s->fdrag[3 * i + k] = 0.0; s->fbuoy[3 * i + k] = 0.0; }
    if (!s->alive[i]) continue;
    double np, u[3], gp[3];
    particle_fluid(s, i, ncell, ucell, &np, u, gp);
    double sl[3];
    for (int c = 0; c < 3; ++c) sl[c] = u[c] - s->v[3 * i + c];
    double cd = s->c_drag ? s->c_drag[i] : 1.0;
    or_drag(sl, 2.0 * s->r[i], p->k_cg, np, p->rho_f, p->mu_f, cd, &s->fdrag[3 * i]);
    /* buoyancy and the dynamic pressure gradient (eq 1, F_b) */
    double V = (4.0 / 3.0) * M_PI * s->r[i] * s->r[i] * s->r[i];
    for (int c = 0; c < 3; ++c) s->fbuoy[3 * i + c] = -V * (gp[c] + p->rho_f * p->g[c]);
    /* eq 7: drag source of each cell */
    cellw cw; particle_cells(s, &s->x[3 * i], &cw);
    for (int k = 0; k < cw.cnt; ++k)
      for (int c = 0; c < 3; ++c) s->fd_cell[3 * cw.cell[k] + c] += cw.w[k] * s->fdrag[3 * i + c];
  }
  for (int64_t c = 0; c < 3 * nc; ++c) s->fd_cell[c] /= vcell;
  free(ncell); free(ucell);
}

/* ------------------------------------------------------------------ */
/* walls                                                                */
/* ------------------------------------------------------------------ */
/* signed distance of the centre from the wall surface (positive on the
 * particle side) and the wall's unit normal pointing into the particle side */
static int wall_geom(const or_wall* wl, const double* x, double* sd, double* nw) {
  if (wl->kind == OR_WALL_PLANE) {
    nw[0] = wl->p[0]; nw[1] = wl->p[1]; nw[2] = wl->p[2];
    *sd = dot3(nw, x) - wl->p[3];
    return 1;
  }
  if (wl->kind == OR_WALL_PLANE_HOLE) {
    double hx = x[0] - wl->p[0], hy = x[1] - wl->p[1];
    if (hx * hx + hy * hy < wl->p[4] * wl->p[4]) return 0;   /* over the hole: no plane */
    nw[0] = 0.0; nw[1] = 0.0; nw[2] = wl->p[3];
    *sd = wl->p[3] * (x[2] - wl->p[2]);
    return 1;
  }
  double ex = x[0] - wl->p[0], ey = x[1] - wl->p[1];
  double rho = sqrt(ex * ex + ey * ey);
  if (rho == 0.0) return 0;
  if (wl->kind == OR_WALL_CYL_IN) {
    *sd = wl->p[2] - rho;
    nw[0] = -ex / rho; nw[1] = -ey / rho; nw[2] = 0.0;
  } else {
    *sd = rho - wl->p[2];
    nw[0] = ex / rho; nw[1] = ey / rho; nw[2] = 0.0;
  }
  return 1;
}

/* ------------------------------------------------------------------ */
/* one step                                                             */
/* ------------------------------------------------------------------ */
static void one_step(or_sim* s) {
  const or_params* p = &s->p;
  const int64_t n = s->n;
  const double dt = p->dt;
  int nw = p->n_walls;

  /* 1. first half kick and drift (velocity Verlet, eq 1-2) */
  for (int64_t i = 0; i < n; ++i) {
    if (!s->alive[i]) continue;
    for (int c = 0; c < 3; ++c) {
      s->v[3 * i + c] += 0.5 * dt * s->F[3 * i + c] / s->m[i];
      s->w[3 * i + c] += 0.5 * dt * s->T[3 * i + c] / s->I[i];
    }
    for (int c = 0; c < 3; ++c) s->x[3 * i + c] += dt * s->v[3 * i + c];
  }

  /* 2. outlet: a centre inside the cavity (or above the outlet level) leaves
   *    the sample as produced sand */
  int removed = 0;
  if (p->outlet_kind == OR_OUTLET_CAVITY || p->outlet_kind == OR_OUTLET_ABOVE) {
    double rc = p->outlet[2];
    for (int64_t i = 0; i < n; ++i) {
      if (!s->alive[i]) continue;
      double ex = s->x[3 * i + 0] - p->outlet[0], ey = s->x[3 * i + 1] - p->outlet[1];
      int leaves = p->outlet_kind == OR_OUTLET_CAVITY ? ex * ex + ey * ey < rc * rc : s->x[3 * i + 2] > p->outlet[3];
      if (leaves) {
        s->alive[i] = 0;
        s->produced += s->m[i];
        for (int c = 0; c < 3; ++c) { s->F[3 * i + c] = 0.0; s->T[3 * i + c] = 0.0; }
        for (int k = 0; k < 3 * nw; ++k) s->wall_dt[3 * nw * i + k] = 0.0;
        removed = 1;
      }
    }
  }
  if (removed) {
    int64_t k2 = 0;
    for (int64_t k = 0; k < s->nh; ++k)
      if (s->alive[s->h[k].i] && s->alive[s->h[k].j]) s->h[k2++] = s->h[k];
    s->nh = k2;
  }

  /* 3. fluid coupling every couple_every steps (fields held in between) */
  if (p->fluid_on && s->have_fluid && (s->step % p->couple_every) == 0) coupling(s);

  /* 4. contact set: bonded pairs still holding, plus touching unbonded pairs */
  for (int64_t k = 0; k < 3 * n; ++k) { s->F[k] = 0.0; s->T[k] = 0.0; }
  for (int64_t i = 0; i < n; ++i) { s->fscale[i] = 0.0; s->tscale[i] = 0.0; }
  ipair* touch;
  int64_t nt;
  if (p->use_grid_search) {
    nt = pairs_grid_alloc(n, s->x, s->r, s->alive, 0.0, &touch);
  } else {
    int64_t cnt = or_pairs_brute(n, s->x, s->r, s->alive, 0.0, 0, NULL, NULL);
    touch = (ipair*)malloc(sizeof(ipair) * (cnt > 0 ? cnt : 1));
    int64_t* a = (int64_t*)malloc(sizeof(int64_t) * (cnt > 0 ? cnt : 1));
    int64_t* b = (int64_t*)malloc(sizeof(int64_t) * (cnt > 0 ? cnt : 1));
    or_pairs_brute(n, s->x, s->r, s->alive, 0.0, cnt, a, b);
    for (int64_t k = 0; k < cnt; ++k) { touch[k].i = a[k]; touch[k].j = b[k]; }
    free(a); free(b);
    nt = cnt;
  }
  /* union of the touching set and the bonded history, both sorted */
  int64_t cap = nt + s->nh + 1, nu = 0;
  ipair* uni = (ipair*)malloc(sizeof(ipair) * cap);
  {
    int64_t a = 0, b = 0;
    while (a < nt || b < s->nh) {
      ipair next;
      int take_a;
      if (b >= s->nh) take_a = 1;
      else if (a >= nt) take_a = 0;
      else {
        ipair hb = {s->h[b].i, s->h[b].j};
        take_a = cmp_ipair(&touch[a], &hb) <= 0;
      }
      if (take_a) {
        next = touch[a++];
        if (b < s->nh && s->h[b].i == next.i && s->h[b].j == next.j) ++b;
      } else {
        if (!s->h[b].bonded) { ++b; continue; }   /* unbonded and not touching: gone */
        next.i = s->h[b].i; next.j = s->h[b].j; ++b;
      }
      uni[nu++] = next;
    }
  }
  free(touch);
  hrec* nh = (hrec*)calloc((size_t)(nu > 0 ? nu : 1), sizeof(hrec));
  int64_t nnh = 0;
  for (int64_t k = 0; k < nu; ++k) {
    int64_t i = uni[k].i, j = uni[k].j;
    hrec* old = find_h(s->h, s->nh, i, j);
    double dx[3];
    for (int c = 0; c < 3; ++c) dx[c] = s->x[3 * j + c] - s->x[3 * i + c];
    double d2 = (dx[0] * dx[0] + dx[1] * dx[1]) + dx[2] * dx[2];
    double ri = s->r[i], rj = s->r[j];
    double cc = ri + rj;
    double Rs = ri * rj / (ri + rj);
    double ms = s->m[i] * s->m[j] / (s->m[i] + s->m[j]);
    double gam = p->gamma;
    if (s->c_coh) gam = p->gamma * sqrt(s->c_coh[i] * s->c_coh[j]);
    int bonded = old ? old->bonded : 0;
    if (p->normal_model == OR_NORMAL_JKR_ORIG) {
      /* original JKR: a touching pair is in contact (snap-in at point A); the
       * contact separates below delta_S (point S), counted like a broken bond,
       * and forms again on the next touch */
      if (d2 < cc * cc) bonded = 1;
      if (bonded && !or_contact_holds_to_S(d2, cc, Rs, s->Es, gam)) {
        s->broken += 1;
        continue;
      }
    } else if (bonded && !or_bond_holds(d2, cc, Rs, s->Es, gam)) {
      s->broken += 1;                       /* broke at point C; never re-forms */
      continue;
    }
    if (!bonded && !(d2 < cc * cc)) continue;
    double dist = sqrt(d2);
    double delta = cc - dist;
    double nrm[3];
    for (int c = 0; c < 3; ++c) nrm[c] = dx[c] / dist;
    double vrel[3], wsum[3], wxn[3], wrel[3];
    for (int c = 0; c < 3; ++c) wsum[c] = ri * s->w[3 * i + c] + rj * s->w[3 * j + c];
    cross3(wsum, nrm, wxn);
    for (int c = 0; c < 3; ++c) {
      vrel[c] = (s->v[3 * i + c] - s->v[3 * j + c]) + wxn[c];
      wrel[c] = s->w[3 * i + c] - s->w[3 * j + c];
    }
    hrec rec;
    rec.i = i; rec.j = j; rec.bonded = (uint8_t)bonded; rec.touch = 1;
    for (int c = 0; c < 3; ++c) rec.dt[c] = old ? old->dt[c] : 0.0;
    law_out o;
    contact_law(s, bonded, delta, Rs, ms, gam, nrm, vrel, wrel, rec.dt, &o);
    for (int c = 0; c < 3; ++c) {
      s->F[3 * i + c] += o.F[c];
      s->F[3 * j + c] -= o.F[c];
      s->T[3 * i + c] += ri * o.c[c] + o.Tr[c];
      s->T[3 * j + c] += rj * o.c[c] - o.Tr[c];
    }
    s->fscale[i] += o.scale; s->fscale[j] += o.scale;
    s->tscale[i] += ri * o.tscale_t + o.tscale_roll; s->tscale[j] += rj * o.tscale_t + o.tscale_roll;
    nh[nnh++] = rec;
  }
  free(uni);
  free(s->h);
  s->h = nh; s->nh = nnh;

  /* 5. walls: Hertz law with the wall as a body of infinite radius and mass */
  for (int k = 0; k < 3 * OR_MAX_WALLS; ++k) s->wall_force[k] = 0.0;
  for (int64_t i = 0; i < n; ++i) {
    if (!s->alive[i]) continue;
    for (int wi = 0; wi < nw; ++wi) {
      double* hdt = &s->wall_dt[3 * (nw * i + wi)];
      double sd, nwv[3];
      if (!wall_geom(&p->walls[wi], &s->x[3 * i], &sd, nwv) || !(sd < s->r[i])) {
        hdt[0] = hdt[1] = hdt[2] = 0.0;
        continue;
      }
      double ri = s->r[i];
      double delta = ri - sd;
      double nrm[3] = {-nwv[0], -nwv[1], -nwv[2]};
      double wr[3], wxn[3], vrel[3];
      for (int c = 0; c < 3; ++c) wr[c] = ri * s->w[3 * i + c];
      cross3(wr, nrm, wxn);
      for (int c = 0; c < 3; ++c) vrel[c] = s->v[3 * i + c] + wxn[c];
      law_out o;
      contact_law(s, 0, delta, ri, s->m[i], 0.0, nrm, vrel, &s->w[3 * i], hdt, &o);
      for (int c = 0; c < 3; ++c) {
        s->F[3 * i + c] += o.F[c];
        s->T[3 * i + c] += ri * o.c[c] + o.Tr[c];
        s->wall_force[3 * wi + c] -= o.F[c];   /* the particle pushes the wall back */
      }
      s->fscale[i] += o.scale;
      s->tscale[i] += ri * o.tscale_t + o.tscale_roll;
    }
  }

  /* 6. body forces: gravity, drag and buoyancy (eq 1) */
  for (int64_t i = 0; i < n; ++i) {
    if (!s->alive[i]) continue;
    double gmag = 0.0;
    for (int c = 0; c < 3; ++c) { s->F[3 * i + c] += s->m[i] * p->g[c]; }
    gmag = s->m[i] * norm3(p->g);
    s->fscale[i] += gmag;
    if (p->fluid_on && s->have_fluid) {
      for (int c = 0; c < 3; ++c) s->F[3 * i + c] += s->fdrag[3 * i + c] + s->fbuoy[3 * i + c];
      s->fscale[i] += norm3(&s->fdrag[3 * i]) + norm3(&s->fbuoy[3 * i]);
    }
  }

  /* 7. second half kick */
  for (int64_t i = 0; i < n; ++i) {
    if (!s->alive[i]) continue;
    for (int c = 0; c < 3; ++c) {
      s->v[3 * i + c] += 0.5 * dt * s->F[3 * i + c] / s->m[i];
      s->w[3 * i + c] += 0.5 * dt * s->T[3 * i + c] / s->I[i];
    }
  }
  s->step += 1;
}

int or_step(or_sim* s, int64_t nsteps) {
  if (s->p.fluid_on && !s->have_fluid) return -1;
  for (int64_t k = 0; k < nsteps; ++k) one_step(s);
  return 0;
}

/* ------------------------------------------------------------------ */
/* accessors                                                            */
/* ------------------------------------------------------------------ */
void or_get_state(const or_sim* s, double* x, double* v, double* w, double* F, double* T,
                  uint8_t* alive, double* fscale, double* tscale) {
  int64_t n = s->n;
  if (x) memcpy(x, s->x, sizeof(double) * 3 * n);
  if (v) memcpy(v, s->v, sizeof(double) * 3 * n);
  if (w) memcpy(w, s->w, sizeof(double) * 3 * n);
  if (F) memcpy(F, s->F, sizeof(double) * 3 * n);
  if (T) memcpy(T, s->T, sizeof(double) * 3 * n);
  if (alive) memcpy(alive, s->alive, (size_t)n);
  if (fscale) memcpy(fscale, s->fscale, sizeof(double) * n);
  if (tscale) memcpy(tscale, s->tscale, sizeof(double) * n);
}

void or_get_scalars(const or_sim* s, double* produced_mass, int64_t* broken_bonds,
                    int64_t* step, int64_t* n_contacts, double* kinetic) {
  if (produced_mass) *produced_mass = s->produced;
  if (broken_bonds) *broken_bonds = s->broken;
  if (step) *step = s->step;
  if (n_contacts) {
    int64_t c = 0;
    for (int64_t k = 0; k < s->nh; ++k) c += s->h[k].touch ? 1 : 0;
    *n_contacts = c;
  }
  if (kinetic) {
    double ke = 0.0;
    for (int64_t i = 0; i < s->n; ++i) {
      if (!s->alive[i]) continue;
      ke += 0.5 * s->m[i] * dot3(&s->v[3 * i], &s->v[3 * i]) + 0.5 * s->I[i] * dot3(&s->w[3 * i], &s->w[3 * i]);
    }
    *kinetic = ke;
  }
}

int64_t or_get_pairs(const or_sim* s, int64_t cap, int64_t* pi, int64_t* pj, double* pdt,
                     uint8_t* pbond, uint8_t* ptouch) {
  for (int64_t k = 0; k < s->nh && k < cap; ++k) {
    if (pi) pi[k] = s->h[k].i;
    if (pj) pj[k] = s->h[k].j;
    if (pdt) for (int c = 0; c < 3; ++c) pdt[3 * k + c] = s->h[k].dt[c];
    if (pbond) pbond[k] = s->h[k].bonded;
    if (ptouch) ptouch[k] = s->h[k].touch;
  }
  return s->nh;
}

void or_get_wall_forces(const or_sim* s, double* force) {
  memcpy(force, s->wall_force, sizeof(double) * 3 * OR_MAX_WALLS);
}

/* replace the walls (same count): a wall moved between calls */
int or_set_walls(or_sim* s, int n_walls, const or_wall* walls) {
  if (n_walls != s->p.n_walls) return -1;
  for (int w = 0; w < n_walls; ++w) s->p.walls[w] = walls[w];
  return 0;
}

void or_get_wall_dt(const or_sim* s, double* wall_dt) {
  int nw = s->p.n_walls > 0 ? s->p.n_walls : 0;
  memcpy(wall_dt, s->wall_dt, sizeof(double) * 3 * s->n * nw);
}

void or_get_fluid(const or_sim* s, double* eps_s, double* fdrag_cell, double* f_part,
                  double* fb_part) {
  int64_t nc = ncells(s);
  if (eps_s) memcpy(eps_s, s->eps_cell, sizeof(double) * nc);
  if (fdrag_cell) memcpy(fdrag_cell, s->fd_cell, sizeof(double) * 3 * nc);
  if (f_part) memcpy(f_part, s->fdrag, sizeof(double) * 3 * s->n);
  if (fb_part) memcpy(fb_part, s->fbuoy, sizeof(double) * 3 * s->n);
}
