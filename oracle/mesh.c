/*
 * Oracle, mesh part: validation, nested 1:4 subdivision (Section 2.2), CSR
 * pattern and element colouring.  TEST INFRASTRUCTURE ONLY.
 *
 * Subdivision: every triangle is split at its edge midpoints into four
 * (Section 2.2).  Numbering: the nodes of level k keep their numbers at level
 * k+1 and the midpoint of the r-th edge (edges as sorted (min,max) pairs)
 * gets number N_k + r.  Coarse nodes are therefore a prefix of every finer
 * level, which realises the injection index pairs of Eq. (30); the two
 * endpoints of each edge are the interpolation parents of Eq. (29).
 */
#include <math.h>
#include <stdlib.h>
#include <string.h>

#include "oracle.h"

/* ------------------------------------------------------------------ helpers */

typedef struct { int a, b; } pair_t;

static int cmp_pair(const void *x, const void *y) {
  const pair_t *p = (const pair_t *)x, *q = (const pair_t *)y;
  if (p->a != q->a) return p->a < q->a ? -1 : 1;
  if (p->b != q->b) return p->b < q->b ? -1 : 1;
  return 0;
}

/* sorted unique undirected edges of a triangle list */
static int build_edges(int t, const int *tri, int **out) {
  pair_t *e = (pair_t *)malloc(sizeof(pair_t) * (size_t)(3 * t + 1));
  for (int i = 0; i < t; i++)
    for (int k = 0; k < 3; k++) {
      int a = tri[3 * i + k], b = tri[3 * i + (k + 1) % 3];
      e[3 * i + k].a = a < b ? a : b;
      e[3 * i + k].b = a < b ? b : a;
    }
  qsort(e, (size_t)3 * t, sizeof(pair_t), cmp_pair);
  int ne = 0;
  for (int i = 0; i < 3 * t; i++)
    if (ne == 0 || cmp_pair(&e[i], &e[ne - 1]) != 0) e[ne++] = e[i];
  int *res = (int *)malloc(sizeof(int) * (size_t)(2 * ne + 2));
  for (int i = 0; i < ne; i++) { res[2 * i] = e[i].a; res[2 * i + 1] = e[i].b; }
  free(e);
  *out = res;
  return ne;
}

/* rank of edge {a,b} in the sorted edge list, -1 if absent */
static int edge_rank(int ne, const int *edge, int a, int b) {
  pair_t key = {a < b ? a : b, a < b ? b : a};
  int lo = 0, hi = ne - 1;
  while (lo <= hi) {
    int mid = (lo + hi) / 2;
    pair_t m = {edge[2 * mid], edge[2 * mid + 1]};
    int c = cmp_pair(&m, &key);
    if (c == 0) return mid;
    if (c < 0) lo = mid + 1; else hi = mid - 1;
  }
  return -1;
}

/* ------------------------------------------------------------ S1: validity */

int orc_check_mesh(int n, const double *xy, int t, const int *tri, int nb, const int *bedge,
                   const int *bkind) {
  if (n <= 0 || t <= 0 || nb < 0 || !xy || !tri || (nb > 0 && (!bedge || !bkind))) return ORC_E_ARG;
  for (int i = 0; i < t; i++) {
    const int *v = tri + 3 * i;
    for (int k = 0; k < 3; k++)
      if (v[k] < 0 || v[k] >= n) return ORC_E_MESH;
    double x1 = xy[2 * v[0]], y1 = xy[2 * v[0] + 1];
    double x2 = xy[2 * v[1]], y2 = xy[2 * v[1] + 1];
    double x3 = xy[2 * v[2]], y3 = xy[2 * v[2] + 1];
    double a2 = (x2 - x1) * (y3 - y1) - (x3 - x1) * (y2 - y1);
    if (!(a2 > 0.0)) return ORC_E_MESH; /* clockwise, degenerate or NaN */
  }
  /* count how many triangles use each edge */
  int *edge;
  int ne = build_edges(t, tri, &edge);
  int *use = (int *)calloc((size_t)ne, sizeof(int));
  for (int i = 0; i < t; i++)
    for (int k = 0; k < 3; k++) use[edge_rank(ne, edge, tri[3 * i + k], tri[3 * i + (k + 1) % 3])]++;
  int st = ORC_OK;
  int *tagged = (int *)calloc((size_t)ne, sizeof(int));
  for (int j = 0; j < nb && st == ORC_OK; j++) {
    int r = edge_rank(ne, edge, bedge[2 * j], bedge[2 * j + 1]);
    if (r < 0 || use[r] != 1 || (bkind[j] != ORC_EDGE_VEL && bkind[j] != ORC_EDGE_OUT) || tagged[r])
      st = ORC_E_MESH;
    else
      tagged[r] = 1;
  }
  for (int r = 0; r < ne && st == ORC_OK; r++) {
    if (use[r] > 2) st = ORC_E_MESH;
    if (use[r] == 1 && !tagged[r]) st = ORC_E_MESH;
  }
  free(use); free(tagged); free(edge);
  return st;
}

/* ------------------------------------------------------ S2: 1:4 subdivision */

static void refine(const orc_level *c, orc_level *f) {
  int nc = c->n, ne = c->ne;
  f->n = nc + ne;
  f->t = 4 * c->t;
  f->nb = 2 * c->nb;
  f->xy = (double *)malloc(sizeof(double) * 2 * (size_t)f->n);
  f->tri = (int *)malloc(sizeof(int) * 3 * (size_t)f->t);
  f->bedge = (int *)malloc(sizeof(int) * (2 * (size_t)f->nb + 1));
  f->bkind = (int *)malloc(sizeof(int) * ((size_t)f->nb + 1));
  f->parent = (int *)malloc(sizeof(int) * 2 * (size_t)ne);
  memcpy(f->xy, c->xy, sizeof(double) * 2 * (size_t)nc);
  for (int r = 0; r < ne; r++) {
    int a = c->edge[2 * r], b = c->edge[2 * r + 1];
    f->xy[2 * (nc + r)] = (c->xy[2 * a] + c->xy[2 * b]) * 0.5;
    f->xy[2 * (nc + r) + 1] = (c->xy[2 * a + 1] + c->xy[2 * b + 1]) * 0.5;
    f->parent[2 * r] = a;
    f->parent[2 * r + 1] = b;
  }
  for (int i = 0; i < c->t; i++) {
    int v0 = c->tri[3 * i], v1 = c->tri[3 * i + 1], v2 = c->tri[3 * i + 2];
    int m01 = nc + edge_rank(ne, c->edge, v0, v1);
    int m12 = nc + edge_rank(ne, c->edge, v1, v2);
    int m20 = nc + edge_rank(ne, c->edge, v2, v0);
    int ch[4][3] = {{v0, m01, m20}, {m01, v1, m12}, {m20, m12, v2}, {m01, m12, m20}};
    memcpy(f->tri + 12 * (size_t)i, ch, sizeof ch);
  }
  for (int j = 0; j < c->nb; j++) {
    int a = c->bedge[2 * j], b = c->bedge[2 * j + 1];
    int m = nc + edge_rank(ne, c->edge, a, b);
    f->bedge[4 * j] = a; f->bedge[4 * j + 1] = m;
    f->bedge[4 * j + 2] = m; f->bedge[4 * j + 3] = b;
    f->bkind[2 * j] = c->bkind[j];
    f->bkind[2 * j + 1] = c->bkind[j];
  }
  f->ne = build_edges(f->t, f->tri, &f->edge);
}

/* ------------------------------------------------------- S3: CSR pattern */

static void build_csr(int n, int t, const int *tri, orc_csr *A) {
  pair_t *e = (pair_t *)malloc(sizeof(pair_t) * (size_t)(9 * t + 1));
  for (int i = 0; i < t; i++)
    for (int a = 0; a < 3; a++)
      for (int b = 0; b < 3; b++) {
        e[9 * i + 3 * a + b].a = tri[3 * i + a];
        e[9 * i + 3 * a + b].b = tri[3 * i + b];
      }
  qsort(e, (size_t)9 * t, sizeof(pair_t), cmp_pair);
  int m = 0;
  for (int i = 0; i < 9 * t; i++)
    if (m == 0 || cmp_pair(&e[i], &e[m - 1]) != 0) e[m++] = e[i];
  A->n = n;
  A->nnz = m;
  A->rp = (int *)calloc((size_t)n + 1, sizeof(int));
  A->col = (int *)malloc(sizeof(int) * (size_t)(m + 1));
  for (int k = 0; k < m; k++) { A->rp[e[k].a + 1]++; A->col[k] = e[k].b; }
  for (int i = 0; i < n; i++) A->rp[i + 1] += A->rp[i];
  free(e);
}

/* position of column j in row i, -1 if absent */
static int csr_find(const orc_csr *A, int i, int j) {
  int lo = A->rp[i], hi = A->rp[i + 1] - 1;
  while (lo <= hi) {
    int mid = (lo + hi) / 2;
    if (A->col[mid] == j) return mid;
    if (A->col[mid] < j) lo = mid + 1; else hi = mid - 1;
  }
  return -1;
}

int orc_csr_find(const orc_csr *A, int i, int j) { return csr_find(A, i, j); }

/* ------------------------------------------------------- S4: colouring */

/* SplitMix64 output finaliser (Steele, Lea & Flood 2014): a bijection of 64-bit words */
uint64_t orc_priority(uint64_t z) {
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
  return z ^ (z >> 31);
}

typedef struct { uint64_t pri; int t; } pri_t;

static int cmp_pri_desc(const void *x, const void *y) {
  const pri_t *p = (const pri_t *)x, *q = (const pri_t *)y;
  if (p->pri != q->pri) return p->pri > q->pri ? -1 : 1;
  return 0;
}

/* Greedy first-fit in decreasing priority: an element takes the smallest colour
 * not already taken by a node-sharing element of higher priority. */
static int colour_mesh(int n, int t, const int *tri, int *colour) {
  int *cnt = (int *)calloc((size_t)n + 1, sizeof(int));
  for (int i = 0; i < 3 * t; i++) cnt[tri[i] + 1]++;
  for (int i = 0; i < n; i++) cnt[i + 1] += cnt[i];
  int *adj = (int *)malloc(sizeof(int) * (size_t)(3 * t));
  int *fill = (int *)calloc((size_t)n, sizeof(int));
  for (int i = 0; i < t; i++)
    for (int k = 0; k < 3; k++) {
      int v = tri[3 * i + k];
      adj[cnt[v] + fill[v]++] = i;
    }
  pri_t *order = (pri_t *)malloc(sizeof(pri_t) * (size_t)t);
  for (int i = 0; i < t; i++) { order[i].pri = orc_priority((uint64_t)i); order[i].t = i; colour[i] = -1; }
  qsort(order, (size_t)t, sizeof(pri_t), cmp_pri_desc);
  int ncol = 0;
  for (int s = 0; s < t; s++) {
    int e = order[s].t;
    unsigned char used[256];
    memset(used, 0, sizeof used);
    for (int k = 0; k < 3; k++) {
      int v = tri[3 * e + k];
      for (int q = cnt[v]; q < cnt[v + 1]; q++) {
        int o = adj[q];
        if (o != e && colour[o] >= 0) used[colour[o]] = 1;
      }
    }
    int c = 0;
    while (used[c]) c++;
    colour[e] = c;
    if (c + 1 > ncol) ncol = c + 1;
  }
  free(cnt); free(adj); free(fill); free(order);
  return ncol;
}

/* ------------------------------------------------------- problem object */

orc_problem *orc_create(int n, const double *xy, int t, const int *tri, int nb, const int *bedge,
                        const int *bkind, int levels, int *status) {
  int st = orc_check_mesh(n, xy, t, tri, nb, bedge, bkind);
  if (st == ORC_OK && (levels < 0 || levels > ORC_MAXLEV)) st = ORC_E_ARG;
  if (status) *status = st;
  if (st != ORC_OK) return NULL;
  orc_problem *p = (orc_problem *)calloc(1, sizeof(orc_problem));
  p->levels = levels;
  orc_level *c = &p->lev[0];
  c->n = n; c->t = t; c->nb = nb;
  c->xy = (double *)malloc(sizeof(double) * 2 * (size_t)n);
  c->tri = (int *)malloc(sizeof(int) * 3 * (size_t)t);
  c->bedge = (int *)malloc(sizeof(int) * (2 * (size_t)nb + 1));
  c->bkind = (int *)malloc(sizeof(int) * ((size_t)nb + 1));
  memcpy(c->xy, xy, sizeof(double) * 2 * (size_t)n);
  memcpy(c->tri, tri, sizeof(int) * 3 * (size_t)t);
  if (nb) {
    memcpy(c->bedge, bedge, sizeof(int) * 2 * (size_t)nb);
    memcpy(c->bkind, bkind, sizeof(int) * (size_t)nb);
  }
  c->ne = build_edges(t, tri, &c->edge);
  for (int k = 0; k < levels; k++) refine(&p->lev[k], &p->lev[k + 1]);
  const orc_level *F = &p->lev[levels];
  build_csr(F->n, F->t, F->tri, &p->pf);
  build_csr(c->n, c->t, c->tri, &p->pc);
  p->colour_f = (int *)malloc(sizeof(int) * (size_t)F->t);
  p->ncol_f = colour_mesh(F->n, F->t, F->tri, p->colour_f);
  p->colour_c = (int *)malloc(sizeof(int) * (size_t)c->t);
  p->ncol_c = colour_mesh(c->n, c->t, c->tri, p->colour_c);
  /* S5: boundary masks */
  p->vdir = (unsigned char *)calloc((size_t)F->n, 1);
  for (int j = 0; j < F->nb; j++)
    if (F->bkind[j] == ORC_EDGE_VEL) { p->vdir[F->bedge[2 * j]] = 1; p->vdir[F->bedge[2 * j + 1]] = 1; }
  p->pdir = (unsigned char *)calloc((size_t)c->n, 1);
  for (int j = 0; j < c->nb; j++)
    if (c->bkind[j] == ORC_EDGE_OUT) { p->pdir[c->bedge[2 * j]] = 1; p->pdir[c->bedge[2 * j + 1]] = 1; }
  p->n_pdir = 0;
  for (int i = 0; i < c->n; i++) p->n_pdir += p->pdir[i];
  return p;
}

void orc_free(orc_problem *p) {
  if (!p) return;
  for (int k = 0; k <= p->levels; k++) {
    orc_level *L = &p->lev[k];
    free(L->xy); free(L->tri); free(L->bedge); free(L->bkind); free(L->edge); free(L->parent);
  }
  free(p->pf.rp); free(p->pf.col); free(p->pc.rp); free(p->pc.col);
  free(p->colour_f); free(p->colour_c); free(p->vdir); free(p->pdir);
  free(p->Mf); free(p->Kf); free(p->Dxf); free(p->Dyf); free(p->mlf);
  free(p->Kc); free(p->Kc_bc); free(p->Dxc); free(p->Dyc); free(p->mc);
  free(p);
}

/* out: n_f, t_f, n_c, t_c, nnz_f, nnz_c, ncol_f, ncol_c, nb_f, nb_c, levels, n_pdir */
void orc_info(const orc_problem *p, int64_t *out) {
  const orc_level *F = &p->lev[p->levels], *C = &p->lev[0];
  out[0] = F->n; out[1] = F->t; out[2] = C->n; out[3] = C->t;
  out[4] = p->pf.nnz; out[5] = p->pc.nnz; out[6] = p->ncol_f; out[7] = p->ncol_c;
  out[8] = F->nb; out[9] = C->nb; out[10] = p->levels; out[11] = p->n_pdir;
}

/* Export topology.  what: 0 xy, 1 tri, 2 bedge, 3 bkind, 4 parent (level>=1), 5 edges,
 * 6 fine row_ptr, 7 fine col, 8 fine slot[t][9], 9 fine colour, 10 coarse row_ptr,
 * 11 coarse col, 12 coarse slot, 13 coarse colour, 14 velocity-Dirichlet mask (int),
 * 15 pressure-Dirichlet mask (int), 16 n_nodes of level (int) */
int orc_export(const orc_problem *p, int what, int level, void *dst) {
  if (level < 0 || level > p->levels) return ORC_E_ARG;
  const orc_level *L = &p->lev[level];
  const orc_level *F = &p->lev[p->levels], *C = &p->lev[0];
  int *I = (int *)dst;
  switch (what) {
    case 0: memcpy(dst, L->xy, sizeof(double) * 2 * (size_t)L->n); return 0;
    case 1: memcpy(dst, L->tri, sizeof(int) * 3 * (size_t)L->t); return 0;
    case 2: memcpy(dst, L->bedge, sizeof(int) * 2 * (size_t)L->nb); return 0;
    case 3: memcpy(dst, L->bkind, sizeof(int) * (size_t)L->nb); return 0;
    case 4:
      if (level == 0) return ORC_E_ARG;
      memcpy(dst, L->parent, sizeof(int) * 2 * (size_t)(L->n - p->lev[level - 1].n));
      return 0;
    case 5: memcpy(dst, L->edge, sizeof(int) * 2 * (size_t)L->ne); return 0;
    case 6: memcpy(dst, p->pf.rp, sizeof(int) * ((size_t)p->pf.n + 1)); return 0;
    case 7: memcpy(dst, p->pf.col, sizeof(int) * (size_t)p->pf.nnz); return 0;
    case 10: memcpy(dst, p->pc.rp, sizeof(int) * ((size_t)p->pc.n + 1)); return 0;
    case 11: memcpy(dst, p->pc.col, sizeof(int) * (size_t)p->pc.nnz); return 0;
    case 8:
    case 12: {
      const orc_level *M = what == 8 ? F : C;
      const orc_csr *A = what == 8 ? &p->pf : &p->pc;
      for (int e = 0; e < M->t; e++)
        for (int a = 0; a < 3; a++)
          for (int b = 0; b < 3; b++) I[9 * e + 3 * a + b] = csr_find(A, M->tri[3 * e + a], M->tri[3 * e + b]);
      return 0;
    }
    case 9: memcpy(dst, p->colour_f, sizeof(int) * (size_t)F->t); return 0;
    case 13: memcpy(dst, p->colour_c, sizeof(int) * (size_t)C->t); return 0;
    case 14: for (int i = 0; i < F->n; i++) I[i] = p->vdir[i]; return 0;
    case 15: for (int i = 0; i < C->n; i++) I[i] = p->pdir[i]; return 0;
    case 16: I[0] = L->n; I[1] = L->t; I[2] = L->nb; I[3] = L->ne; return 0;
    default: return ORC_E_ARG;
  }
}
