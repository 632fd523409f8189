/*
 * Oracle: icosahedral mesh of flat triangles on a sphere of radius R.
 * TEST INFRASTRUCTURE ONLY (see oracle.h).
 *
 * The paper's experiments use icosahedral grids (Sec. 3, mesh description:
 * 20480 cells at refinement level 5).  Level 0 is the regular icosahedron;
 * each refinement splits every triangle into four by its edge midpoints, and
 * each new midpoint is pushed out radially onto the sphere.
 */
#include <math.h>
#include <stdlib.h>
#include <string.h>
#include "oracle.h"
#include "om_internal.h"

static int cmp_i64(const void *a, const void *b) {
  int64_t x = *(const int64_t *)a, y = *(const int64_t *)b;
  return (x > y) - (x < y);
}

/* Position of key in the sorted unique array keys[0..n). */
static int find_key(const int64_t *keys, int n, int64_t key) {
  int lo = 0, hi = n - 1;
  while (lo <= hi) {
    int mid = (lo + hi) / 2;
    if (keys[mid] == key) return mid;
    if (keys[mid] < key) lo = mid + 1; else hi = mid - 1;
  }
  return -1;
}

static int64_t pair_key(int a, int b, int nv) {
  int lo = a < b ? a : b, hi = a < b ? b : a;
  return (int64_t)lo * nv + hi;
}

/* Sorted list of the distinct vertex pairs that are triangle sides. */
static int64_t *unique_sides(const int *tri, int nt, int nv, int *nout) {
  int64_t *k = malloc(sizeof(int64_t) * 3 * nt);
  for (int t = 0; t < nt; t++)
    for (int i = 0; i < 3; i++)
      k[3 * t + i] = pair_key(tri[3 * t + (i + 1) % 3], tri[3 * t + (i + 2) % 3], nv);
  qsort(k, 3 * (size_t)nt, sizeof(int64_t), cmp_i64);
  int n = 0;
  for (int i = 0; i < 3 * nt; i++)
    if (n == 0 || k[i] != k[n - 1]) k[n++] = k[i];
  *nout = n;
  return k;
}

static void to_sphere(double *p, double R) {
  double r = sqrt(p[0] * p[0] + p[1] * p[1] + p[2] * p[2]);
  for (int d = 0; d < 3; d++) p[d] *= R / r;
}

om_mesh *om_mesh_create(int level, double R) {
  if (level < 0 || level > 9) return NULL;
  const double phi = 0.5 * (1.0 + sqrt(5.0));
  int nv = 12, nt = 20;
  int nv_final = 10 * (1 << (2 * level)) + 2;
  int nt_final = 20 * (1 << (2 * level));
  double *x = malloc(sizeof(double) * 3 * nv_final);
  int *tri = malloc(sizeof(int) * 3 * nt_final);
  /* the 12 cyclic permutations of (0, +-1, +-phi) */
  int n = 0;
  for (int s1 = -1; s1 <= 1; s1 += 2)
    for (int s2 = -1; s2 <= 1; s2 += 2) {
      double a = s1, b = s2 * phi;
      double v[3][3] = {{0, a, b}, {a, b, 0}, {b, 0, a}};
      for (int c = 0; c < 3; c++) {
        memcpy(x + 3 * n, v[c], sizeof(v[c]));
        n++;
      }
    }
  /* faces: triples of mutually adjacent vertices (squared distance 4) */
  n = 0;
  for (int i = 0; i < 12; i++)
    for (int j = i + 1; j < 12; j++)
      for (int k = j + 1; k < 12; k++) {
        int ok = 1;
        int id[3] = {i, j, k};
        for (int p = 0; p < 3 && ok; p++) {
          const double *a = x + 3 * id[p], *b = x + 3 * id[(p + 1) % 3];
          double d2 = 0;
          for (int d = 0; d < 3; d++) d2 += (a[d] - b[d]) * (a[d] - b[d]);
          if (fabs(d2 - 4.0) > 1e-9) ok = 0;
        }
        if (ok) {
          tri[3 * n] = i; tri[3 * n + 1] = j; tri[3 * n + 2] = k;
          n++;
        }
      }
  for (int i = 0; i < 12; i++) to_sphere(x + 3 * i, R);

  /* refinement: (a,b,c) -> (a,ab,ca), (b,bc,ab), (c,ca,bc), (ab,bc,ca) */
  for (int l = 0; l < level; l++) {
    int ns;
    int64_t *sides = unique_sides(tri, nt, nv, &ns);
    for (int s = 0; s < ns; s++) {
      int a = (int)(sides[s] / nv), b = (int)(sides[s] % nv);
      double *p = x + 3 * (nv + s);
      for (int d = 0; d < 3; d++) p[d] = 0.5 * (x[3 * a + d] + x[3 * b + d]);
      to_sphere(p, R);
    }
    int *nt_tri = malloc(sizeof(int) * 12 * nt);
    for (int t = 0; t < nt; t++) {
      int a = tri[3 * t], b = tri[3 * t + 1], c = tri[3 * t + 2];
      int ab = nv + find_key(sides, ns, pair_key(a, b, nv));
      int bc = nv + find_key(sides, ns, pair_key(b, c, nv));
      int ca = nv + find_key(sides, ns, pair_key(c, a, nv));
      int ch[4][3] = {{a, ab, ca}, {b, bc, ab}, {c, ca, bc}, {ab, bc, ca}};
      memcpy(nt_tri + 12 * t, ch, sizeof(ch));
    }
    free(tri);
    tri = nt_tri;
    nv += ns;
    nt *= 4;
    free(sides);
  }

  om_mesh *m = calloc(1, sizeof(om_mesh));
  m->level = level;
  m->R = R;
  m->nv = nv;
  m->nc = nt;
  m->x = x;
  m->cv = tri;
  /* orient every cell counter-clockwise seen from outside */
  for (int t = 0; t < nt; t++) {
    const double *p0 = x + 3 * tri[3 * t], *p1 = x + 3 * tri[3 * t + 1],
                 *p2 = x + 3 * tri[3 * t + 2];
    double e1[3], e2[3], k[3];
    om_sub(p1, p0, e1);
    om_sub(p2, p0, e2);
    om_cross(e1, e2, k);
    double c[3] = {p0[0] + p1[0] + p2[0], p0[1] + p1[1] + p2[1], p0[2] + p1[2] + p2[2]};
    if (om_dot(k, c) < 0) {
      int tmp = tri[3 * t + 1];
      tri[3 * t + 1] = tri[3 * t + 2];
      tri[3 * t + 2] = tmp;
    }
  }
  /* edges: one per distinct side; c0 is the lower-numbered cell */
  int ne;
  int64_t *sides = unique_sides(tri, nt, nv, &ne);
  m->ne = ne;
  m->ce = malloc(sizeof(int) * 3 * nt);
  m->csign = malloc(sizeof(int) * 3 * nt);
  m->ec = malloc(sizeof(int) * 2 * ne);
  m->ev = malloc(sizeof(int) * 2 * ne);
  for (int e = 0; e < 2 * ne; e++) m->ec[e] = -1;
  for (int t = 0; t < nt; t++)
    for (int i = 0; i < 3; i++) {
      int a = tri[3 * t + (i + 1) % 3], b = tri[3 * t + (i + 2) % 3];
      int e = find_key(sides, ne, pair_key(a, b, nv));
      m->ce[3 * t + i] = e;
      if (m->ec[2 * e] < 0) {
        m->ec[2 * e] = t;
        m->ev[2 * e] = a;
        m->ev[2 * e + 1] = b;
        m->csign[3 * t + i] = 1;
      } else {
        m->ec[2 * e + 1] = t;
        m->csign[3 * t + i] = -1;
      }
    }
  free(sides);
  return m;
}

void om_mesh_destroy(om_mesh *m) {
  if (!m) return;
  free(m->x); free(m->cv); free(m->ce); free(m->csign); free(m->ec); free(m->ev);
  free(m);
}

void om_mesh_counts(const om_mesh *m, int *nv, int *ne, int *nc) {
  if (nv) *nv = m->nv;
  if (ne) *ne = m->ne;
  if (nc) *nc = m->nc;
}

void om_mesh_export(const om_mesh *m, double *verts, int32_t *cell_verts,
                    int32_t *cell_edges, int32_t *cell_sign,
                    int32_t *edge_cells, int32_t *edge_verts) {
  if (verts) memcpy(verts, m->x, sizeof(double) * 3 * m->nv);
  for (int i = 0; i < 3 * m->nc; i++) {
    if (cell_verts) cell_verts[i] = m->cv[i];
    if (cell_edges) cell_edges[i] = m->ce[i];
    if (cell_sign) cell_sign[i] = m->csign[i];
  }
  for (int i = 0; i < 2 * m->ne; i++) {
    if (edge_cells) edge_cells[i] = m->ec[i];
    if (edge_verts) edge_verts[i] = m->ev[i];
  }
}
