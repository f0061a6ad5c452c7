/*
 * sbr_oracle.c -- plain, slow, obviously-correct CPU FP64 reference of the
 * shooting-and-bouncing-ray (SBR) channel method.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path may link, load or
 * call this file: only the test-suite, the smoke check and the CPU-baseline
 * leg of the benchmark use it.  It shares no code, header, table or constant
 * generator with the GPU library; every step is written again here from the
 * paper and the readings recorded beside the tests.
 *
 * Steps (paper, Section II-A: launch -> trace -> receive -> calculate):
 *   geodesic ray launch ............ Sec. II-A-1 (icosahedron sampling, Fig. 1)
 *   brute-force closest hit ........ Sec. II-A-2 (every triangle is tested)
 *   specular reflection ............ Sec. II-A-2 (Snell's law)
 *   reception sphere ............... Sec. II-A-3 (radius grows with distance)
 *   image-method path geometry ..... Sec. I (image method) applied to the
 *                                    face sequence a captured ray records
 *   field of one path .............. eq. (1) with Fresnel TE/TM (eq. (8)),
 *                                    Kirchhoff roughness (eq. (6)-(7)),
 *                                    free-space factor (eq. (3) -> Friis),
 *                                    table attenuation/dispersion (eq. (9)-(10))
 *
 * Everything is IEEE double; no fast-math.  OpenMP parallelises only over
 * independent rays and results are merged in ray order, so output is
 * deterministic.
 */
#include <complex.h>
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define ORC_PI 3.14159265358979323846
static const double ORC_C0 = 299792458.0;        /* m/s */
static const double ORC_EPS0 = 8.8541878128e-12;  /* F/m */

/* ------------------------------------------------------------------ vectors */
typedef struct { double x, y, z; } v3;
static v3 mk(double x, double y, double z) { v3 r = {x, y, z}; return r; }
static v3 add(v3 a, v3 b) { return mk(a.x + b.x, a.y + b.y, a.z + b.z); }
static v3 sub(v3 a, v3 b) { return mk(a.x - b.x, a.y - b.y, a.z - b.z); }
static v3 scl(v3 a, double s) { return mk(a.x * s, a.y * s, a.z * s); }
static double dot(v3 a, v3 b) { return a.x * b.x + a.y * b.y + a.z * b.z; }
static v3 crs(v3 a, v3 b) { return mk(a.y * b.z - a.z * b.y, a.z * b.x - a.x * b.z, a.x * b.y - a.y * b.x); }
static double nrm(v3 a) { return sqrt(dot(a, a)); }
static v3 unit(v3 a) { return scl(a, 1.0 / nrm(a)); }
static v3 ld(const double* p) { return mk(p[0], p[1], p[2]); }

/* =====================================================================
 * 1. Icosahedral geodesic launch (Sec. II-A-1).
 * Class-I geodesic of frequency N on the regular icosahedron: every face is
 * cut by the flat barycentric grid with step 1/N and the grid points are
 * pushed out to the unit sphere.  Rays per source: 10 N^2 + 2.
 * Canonical ray order: 12 corners; then the 30 edges (ascending vertex
 * pairs) with their N-1 interior points counted from the lower vertex; then
 * the 20 faces (ascending vertex triples) with their (N-1)(N-2)/2 interior
 * points in (i, j) order.
 * ===================================================================== */
typedef struct { v3 v[12]; int e[30][2]; int f[20][3]; } ico_t;

static void ico_build(ico_t* G) {
  const double ph = (1.0 + sqrt(5.0)) / 2.0;
  const double sg[4][2] = {{-1, -1}, {-1, 1}, {1, -1}, {1, 1}};
  for (int s = 0; s < 4; ++s) {
    G->v[s] = mk(0.0, sg[s][0] * 1.0, sg[s][1] * ph);
    G->v[4 + s] = mk(sg[s][0] * 1.0, sg[s][1] * ph, 0.0);
    G->v[8 + s] = mk(sg[s][0] * ph, 0.0, sg[s][1] * 1.0);
  }
  /* edges = vertex pairs at the minimum mutual distance (found by search) */
  double dmin = 1e300;
  for (int a = 0; a < 12; ++a)
    for (int b = a + 1; b < 12; ++b) {
      double d = nrm(sub(G->v[a], G->v[b]));
      if (d < dmin) dmin = d;
    }
  int ne = 0;
  int adj[12][12];
  memset(adj, 0, sizeof adj);
  for (int a = 0; a < 12; ++a)
    for (int b = a + 1; b < 12; ++b)
      if (nrm(sub(G->v[a], G->v[b])) < dmin * (1.0 + 1e-9)) {
        G->e[ne][0] = a; G->e[ne][1] = b; ++ne;
        adj[a][b] = adj[b][a] = 1;
      }
  int nf = 0;
  for (int a = 0; a < 12; ++a)
    for (int b = a + 1; b < 12; ++b)
      for (int c = b + 1; c < 12; ++c)
        if (adj[a][b] && adj[a][c] && adj[b][c]) { G->f[nf][0] = a; G->f[nf][1] = b; G->f[nf][2] = c; ++nf; }
  for (int a = 0; a < 12; ++a) G->v[a] = unit(G->v[a]);
  (void)ne; (void)nf;
}

int64_t orc_geodesic_count(int N) { return 10LL * N * N + 2; }

/* direction of ray `id` (0 <= id < 10N^2+2) */
static v3 geo_dir(const ico_t* G, int N, int64_t id) {
  if (id < 12) return G->v[id];
  id -= 12;
  if (id < 30LL * (N - 1)) {
    int e = (int)(id / (N - 1));
    int i = (int)(id % (N - 1)) + 1;
    v3 a = G->v[G->e[e][0]], b = G->v[G->e[e][1]];
    double w = (double)i / N;
    return unit(add(scl(a, 1.0 - w), scl(b, w)));
  }
  id -= 30LL * (N - 1);
  int64_t per = (int64_t)(N - 1) * (N - 2) / 2;
  int f = (int)(id / per);
  int64_t l = id % per;
  /* walk rows i = 1.. ; row i holds j = 1 .. N-1-i */
  int i = 1;
  while (l >= N - 1 - i) { l -= N - 1 - i; ++i; }
  int j = (int)l + 1;
  v3 a = G->v[G->f[f][0]], b = G->v[G->f[f][1]], c = G->v[G->f[f][2]];
  double wi = (double)i / N, wj = (double)j / N;
  return unit(add(add(scl(a, 1.0 - wi - wj), scl(b, wi)), scl(c, wj)));
}

int orc_geodesic(int N, int64_t first, int64_t count, double* out) {
  if (N < 1) return -1;
  ico_t G; ico_build(&G);
  for (int64_t k = 0; k < count; ++k) {
    v3 d = geo_dir(&G, N, first + k);
    out[3 * k] = d.x; out[3 * k + 1] = d.y; out[3 * k + 2] = d.z;
  }
  return 0;
}

/* Edge statistics of the geodesic triangulation (all 30 N^2 undirected
 * edges).  mean -> the default ray angular spacing alpha of the reception
 * sphere; min/max used by the exhaustive-capture pins. */
static v3 face_pt(const ico_t* G, int f, int N, int i, int j) {
  v3 a = G->v[G->f[f][0]], b = G->v[G->f[f][1]], c = G->v[G->f[f][2]];
  double wi = (double)i / N, wj = (double)j / N;
  return unit(add(add(scl(a, 1.0 - wi - wj), scl(b, wi)), scl(c, wj)));
}
static double ang(v3 a, v3 b) { return atan2(nrm(crs(a, b)), dot(a, b)); }

void orc_edge_stats(int N, double* mean, double* mn, double* mx) {
  ico_t G; ico_build(&G);
  double sum = 0.0, lo = 1e300, hi = 0.0;
  for (int f = 0; f < 20; ++f)
    for (int i = 0; i <= N; ++i)
      for (int j = 0; i + j <= N; ++j) {
        v3 p = face_pt(&G, f, N, i, j);
        if (i + j + 1 <= N) {
          v3 q1 = face_pt(&G, f, N, i + 1, j), q2 = face_pt(&G, f, N, i, j + 1);
          double a1 = ang(p, q1), a2 = ang(p, q2), a3 = ang(q1, q2);
          /* (i,j)-(i+1,j) lies on face edge ab when j == 0; (i,j)-(i,j+1) on ac
           * when i == 0; (i+1,j)-(i,j+1) on bc when i+j+1 == N.  Shared edges
           * are seen from both faces and weighted 1/2. */
          sum += a1 * (j == 0 ? 0.5 : 1.0) + a2 * (i == 0 ? 0.5 : 1.0) + a3 * (i + j + 1 == N ? 0.5 : 1.0);
          if (a1 < lo) lo = a1; if (a1 > hi) hi = a1;
          if (a2 < lo) lo = a2; if (a2 > hi) hi = a2;
          if (a3 < lo) lo = a3; if (a3 > hi) hi = a3;
        }
      }
  *mean = sum / (30.0 * N * N);
  *mn = lo; *mx = hi;
}

/* =====================================================================
 * 2. Scene: planes and face groups.
 * A face group is a set of triangles in one plane with equal materials; it
 * is the unit a path key refers to (a flat wall split into two triangles is
 * one reflector).  Pairs are joined when |n_i . n_j| >= 1 - 1e-12 and plane
 * offsets agree within 1e-9 of the scene diagonal (transitive closure);
 * group ids are numbered by their lowest triangle index.
 * ===================================================================== */
typedef struct {
  int T;
  const double* tri;
  const float *eps, *sig, *rough;
  v3* n; double* c;     /* unit normal and offset n.x = c per triangle */
  int* plane; int* group; int ngroups;
  int* gfirst;          /* lowest triangle of each group */
  int* gstart; int* gtri; /* CSR: triangles of each group */
  double diag;
  v3 center;            /* centre of the scene's bounding box */
  double* hgt;          /* [T][3] height of each triangle over the edge opposite vertex 0, 1, 2 */
} scene_t;

static int uf_find(int* p, int x) { while (p[x] != x) { p[x] = p[p[x]]; x = p[x]; } return x; }
static void uf_join(int* p, int a, int b) { a = uf_find(p, a); b = uf_find(p, b); if (a < b) p[b] = a; else if (b < a) p[a] = b; }

static v3 tv(const scene_t* S, int t, int k) { return ld(S->tri + 9 * t + 3 * k); }

static int scene_init(scene_t* S, const double* tri, int T, const float* eps, const float* sig, const float* rough) {
  memset(S, 0, sizeof *S);
  S->T = T; S->tri = tri; S->eps = eps; S->sig = sig; S->rough = rough;
  if (T == 0) { S->gstart = calloc(1, sizeof(int)); return 0; }
  S->n = malloc(sizeof(v3) * T); S->c = malloc(sizeof(double) * T);
  S->hgt = malloc(sizeof(double) * 3 * T);
  S->plane = malloc(sizeof(int) * T); S->group = malloc(sizeof(int) * T);
  v3 lo = mk(1e300, 1e300, 1e300), hi = mk(-1e300, -1e300, -1e300);
  for (int t = 0; t < T; ++t) {
    for (int k = 0; k < 3; ++k) {
      v3 p = tv(S, t, k);
      lo = mk(fmin(lo.x, p.x), fmin(lo.y, p.y), fmin(lo.z, p.z));
      hi = mk(fmax(hi.x, p.x), fmax(hi.y, p.y), fmax(hi.z, p.z));
    }
    v3 nn = crs(sub(tv(S, t, 1), tv(S, t, 0)), sub(tv(S, t, 2), tv(S, t, 0)));
    S->n[t] = unit(nn);
    S->c[t] = dot(S->n[t], tv(S, t, 0));
    double twoA = nrm(nn);
    S->hgt[3 * t] = twoA / nrm(sub(tv(S, t, 2), tv(S, t, 1)));
    S->hgt[3 * t + 1] = twoA / nrm(sub(tv(S, t, 2), tv(S, t, 0)));
    S->hgt[3 * t + 2] = twoA / nrm(sub(tv(S, t, 1), tv(S, t, 0)));
  }
  S->diag = nrm(sub(hi, lo));
  S->center = scl(add(lo, hi), 0.5);
  int* pp = malloc(sizeof(int) * T);
  int* pg = malloc(sizeof(int) * T);
  for (int t = 0; t < T; ++t) pp[t] = pg[t] = t;
  for (int a = 0; a < T; ++a)
    for (int b = a + 1; b < T; ++b) {
      double nd = dot(S->n[a], S->n[b]);
      if (fabs(nd) < 1.0 - 1e-12) continue;
      double s = nd > 0 ? 1.0 : -1.0;
      if (fabs(S->c[a] - s * S->c[b]) > 1e-9 * S->diag) continue;
      uf_join(pp, a, b);
      if (eps[a] == eps[b] && sig[a] == sig[b] && rough[a] == rough[b]) uf_join(pg, a, b);
    }
  /* number roots in order of first (= lowest) triangle */
  int* gid = malloc(sizeof(int) * T);
  int* pid = malloc(sizeof(int) * T);
  for (int t = 0; t < T; ++t) gid[t] = pid[t] = -1;
  int ng = 0, np = 0;
  for (int t = 0; t < T; ++t) {
    int rg = uf_find(pg, t), rp = uf_find(pp, t);
    if (gid[rg] < 0) gid[rg] = ng++;
    if (pid[rp] < 0) pid[rp] = np++;
    S->group[t] = gid[rg];
    S->plane[t] = pid[rp];
  }
  S->ngroups = ng;
  S->gfirst = malloc(sizeof(int) * ng);
  S->gstart = calloc(ng + 1, sizeof(int));
  S->gtri = malloc(sizeof(int) * T);
  for (int g = 0; g < ng; ++g) S->gfirst[g] = -1;
  for (int t = 0; t < T; ++t) { if (S->gfirst[S->group[t]] < 0) S->gfirst[S->group[t]] = t; S->gstart[S->group[t] + 1]++; }
  for (int g = 0; g < ng; ++g) S->gstart[g + 1] += S->gstart[g];
  int* fill = calloc(ng, sizeof(int));
  for (int t = 0; t < T; ++t) { int g = S->group[t]; S->gtri[S->gstart[g] + fill[g]++] = t; }
  free(fill); free(gid); free(pid); free(pp); free(pg);
  return 0;
}

static void scene_free(scene_t* S) {
  free(S->n); free(S->c); free(S->hgt); free(S->plane); free(S->group); free(S->gfirst); free(S->gstart); free(S->gtri);
}

int orc_scene_groups(const double* tri, int T, const float* eps, const float* sig, const float* rough,
                     int32_t* group, int32_t* plane) {
  scene_t S; scene_init(&S, tri, T, eps, sig, rough);
  for (int t = 0; t < T; ++t) { group[t] = S.group[t]; plane[t] = S.plane[t]; }
  int ng = S.ngroups;
  scene_free(&S);
  return ng;
}

/* =====================================================================
 * 3. Closest hit by brute force (Sec. II-A-2: the intersection step).
 * Moller-Trumbore in FP64, double-sided, inclusive barycentrics, a ray
 * parallel to the plane misses.  The nearest t > 1e-12 * diag wins, ties go
 * to the lower triangle index; triangles in the plane of the previous hit
 * are skipped (the reflected ray leaves that plane).
 * Ambiguity flags (where an FP32 tracer may legitimately disagree):
 *   1 hit near an edge of its triangle
 *   2 another triangle (not the hit) crossed near its edges no farther than
 *     the hit
 *   4 a second hit within 1e-5 relative in t
 *   8 grazing incidence |d.n| < 1e-5
 * ===================================================================== */
typedef struct { int tri; double t; double u, v; uint8_t amb; } hit_t;

/* "Near an edge": within 1e-5 in barycentric terms, or within an absolute
 * distance of the triangle's boundary that FP32 positions cannot resolve:
 * 4e-6 (about 32 single-precision units in the last place) of the crossing
 * point's distance from the scene centre plus the distance travelled to it.
 * The second band matters on slivers (a 5 cm partition face is 5e-7 m wide
 * in barycentric terms at 1e-5, below FP32 resolution at 15 m). */
static double seg_dist(v3 p, v3 a, v3 b) {
  v3 e = sub(b, a);
  double s = dot(sub(p, a), e) / dot(e, e);
  s = s < 0.0 ? 0.0 : (s > 1.0 ? 1.0 : s);
  return nrm(sub(p, add(a, scl(e, s))));
}
static int near_edge(const scene_t* S, int t, v3 P, double tt, double u, double v) {
  double b[3] = {1.0 - u - v, u, v};
  double mb = fmin(fmin(b[0], b[1]), b[2]);
  if (fabs(mb) < 1e-5) return 1;
  double band = 4e-6 * (nrm(sub(P, S->center)) + tt);
  /* the distance to an edge's line (|b_i| times the height over that edge)
   * bounds the distance to the edge from below: skip the exact test when
   * every line is farther than the band */
  const double* h = S->hgt + 3 * t;
  if (fabs(b[0]) * h[0] > band && fabs(b[1]) * h[1] > band && fabs(b[2]) * h[2] > band) return 0;
  v3 a = tv(S, t, 0), bb = tv(S, t, 1), c = tv(S, t, 2);
  double dmin = fmin(fmin(seg_dist(P, bb, c), seg_dist(P, c, a)), seg_dist(P, a, bb));
  return dmin <= band;
}

static hit_t closest_hit(const scene_t* S, v3 o, v3 d, int skip_plane) {
  hit_t h = {-1, INFINITY, 0, 0, 0};
  double tmin = 1e-12 * S->diag;
  /* the two nearest near-edge crossings (distance and triangle): the flag
   * concerns triangles other than the hit, so the second one stands in when
   * the nearest is the hit triangle itself */
  double t_edge = INFINITY, t_edge2 = INFINITY;
  int edge_tri = -1;
  double t2 = INFINITY;       /* second-nearest hit */
  for (int t = 0; t < S->T; ++t) {
    if (skip_plane >= 0 && S->plane[t] == skip_plane) continue;
    v3 v0 = tv(S, t, 0);
    v3 e1 = sub(tv(S, t, 1), v0), e2 = sub(tv(S, t, 2), v0);
    v3 pv = crs(d, e2);
    double det = dot(e1, pv);
    if (det == 0.0) continue;
    double inv = 1.0 / det;
    v3 tvec = sub(o, v0);
    double u = dot(tvec, pv) * inv;
    v3 qv = crs(tvec, e1);
    double v = dot(d, qv) * inv;
    double tt = dot(e2, qv) * inv;
    if (!(tt > tmin)) continue;
    double mb = fmin(fmin(u, v), 1.0 - u - v);
    if (near_edge(S, t, add(o, scl(d, tt)), tt, u, v)) {
      if (tt < t_edge) { t_edge2 = t_edge; t_edge = tt; edge_tri = t; }
      else if (tt < t_edge2) t_edge2 = tt;
    }
    if (mb >= 0.0) {
      if (tt < h.t) { t2 = h.t; h.t = tt; h.tri = t; h.u = u; h.v = v; }
      else if (tt < t2) t2 = tt;
    }
  }
  if (h.tri >= 0) {
    if (near_edge(S, h.tri, add(o, scl(d, h.t)), h.t, h.u, h.v)) h.amb |= 1;
    double t_other = edge_tri == h.tri ? t_edge2 : t_edge;
    if (t_other <= h.t * (1.0 + 1e-5)) h.amb |= 2;
    if (t2 - h.t <= 1e-5 * h.t) h.amb |= 4;
    if (fabs(dot(d, S->n[h.tri])) < 1e-5) h.amb |= 8;
  } else if (t_edge < INFINITY) {
    h.amb |= 2;
  }
  return h;
}

/* =====================================================================
 * 4.-5. Trace + receive for a list of rays.
 * Each ray of source p starts at T_p along its geodesic direction, is
 * reflected specularly (d' = d - 2 (d.n) n) up to K times and every segment
 * (including the last one, which ends at the (K+1)-th hit or at infinity) is
 * tested against every receive point: with t* = (q - o).d inside the
 * segment, the ray is captured by q when |q - o - t* d| <= coeff * alpha *
 * (L + t*) / sqrt(3), L being the unfolded length before the segment
 * (Sec. II-A-3: sphere radius set by the travelled distance, i.e. by the ray
 * tube's cross-section).
 * A capture event is the key (p, q, k, g_1..g_k): source, receiver, number
 * of reflections and the face groups reflected from.
 * ===================================================================== */
typedef struct { int32_t p, q, k; int32_t g[16]; int64_t ray; uint8_t amb; double ratio; } event_t;
typedef struct { event_t* e; int64_t n, cap; } evbuf_t;
static void ev_push(evbuf_t* b, const event_t* e) {
  if (b->n == b->cap) { b->cap = b->cap ? 2 * b->cap : 256; b->e = realloc(b->e, sizeof(event_t) * b->cap); }
  b->e[b->n++] = *e;
}
static int ev_cmp(const void* A, const void* B) {
  const event_t *a = A, *b = B;
  if (a->ray != b->ray) return a->ray < b->ray ? -1 : 1;
  if (a->k != b->k) return a->k - b->k;
  return a->q - b->q;
}

/* returns the number of events (may exceed ev_cap; then only ev_cap are written).
 * ev_amb bits: 1 capture within 1e-5 of the sphere or segment ends, 2 the ray
 * had an ambiguous hit at a bounce <= k, 4 near miss (recorded, not captured). */
int64_t orc_sbr(const double* tri, int T, const float* eps, const float* sig, const float* rough,
                const double* tx, int Nt, const double* rx, int Nr, int N, int K,
                double alpha, double coeff, const int64_t* ray_ids, int64_t nrays,
                int32_t* seq, double* tval, uint8_t* amb,
                int64_t ev_cap, int32_t* ev_key /* [cap][3+K] */, int64_t* ev_ray, uint8_t* ev_amb,
                double* ev_ratio, int nthreads) {
  if (K < 0 || K > 16 || N < 1) return -1;
  scene_t S; scene_init(&S, tri, T, eps, sig, rough);
  ico_t G; ico_build(&G);
  const int64_t R = orc_geodesic_count(N);
  if (alpha <= 0.0) { double mn, mx; orc_edge_stats(N, &alpha, &mn, &mx); }
  const double rfac = coeff * alpha / sqrt(3.0);
  int nth = 1;
#ifdef _OPENMP
  nth = nthreads > 0 ? nthreads : omp_get_max_threads();
#endif
  evbuf_t* bufs = calloc(nth, sizeof(evbuf_t));
#ifdef _OPENMP
#pragma omp parallel for schedule(dynamic, 64) num_threads(nth)
#endif
  for (int64_t ir = 0; ir < nrays; ++ir) {
    int tid = 0;
#ifdef _OPENMP
    tid = omp_get_thread_num();
#endif
    int64_t gid = ray_ids ? ray_ids[ir] : ir;
    int p = (int)(gid / R);
    int64_t r = gid % R;
    v3 o = ld(tx + 3 * p);
    v3 d = geo_dir(&G, N, r);
    double L = 0.0;
    int skip = -1;
    int32_t grp[16];
    uint8_t amb_acc = 0;
    for (int k = 0; k <= K; ++k) {
      seq[ir * (K + 1) + k] = -2; tval[ir * (K + 1) + k] = NAN; amb[ir * (K + 1) + k] = 0;
    }
    for (int k = 0; k <= K; ++k) {
      hit_t h = closest_hit(&S, o, d, skip);
      seq[ir * (K + 1) + k] = h.tri;
      tval[ir * (K + 1) + k] = h.t;
      amb[ir * (K + 1) + k] = h.amb;
      amb_acc |= h.amb;
      double tend = h.t;  /* INFINITY on a miss */
      for (int q = 0; q < Nr; ++q) {
        v3 w = sub(ld(rx + 3 * q), o);
        double ts = dot(w, d);
        if (ts < 0.0 || ts > tend) continue;
        double dist = nrm(sub(w, scl(d, ts)));
        double rad = rfac * (L + ts);
        /* captures, plus near misses within the 1e-5 band (flag 4, not a capture) */
        if (dist <= rad * (1.0 + 1e-5)) {
          event_t e; memset(&e, 0, sizeof e);
          e.p = p; e.q = q; e.k = k; e.ray = gid;
          for (int i = 0; i < 16; ++i) e.g[i] = i < k ? grp[i] : -1;
          double scale = isfinite(tend) ? tend : ts;
          int camb = fabs(dist - rad) <= 1e-5 * rad || ts <= 1e-5 * (L + ts) ||
                     (isfinite(tend) && tend - ts <= 1e-5 * scale);
          e.amb = (uint8_t)((camb ? 1 : 0) | (amb_acc ? 2 : 0) | (dist > rad ? 4 : 0));
          e.ratio = dist / rad;
          ev_push(&bufs[tid], &e);
        }
      }
      if (h.tri < 0 || k == K) break;
      v3 nn = S.n[h.tri];
      o = add(o, scl(d, h.t));
      L += h.t;
      d = sub(d, scl(nn, 2.0 * dot(d, nn)));
      grp[k] = S.group[h.tri];
      skip = S.plane[h.tri];
    }
  }
  int64_t tot = 0;
  for (int i = 0; i < nth; ++i) tot += bufs[i].n;
  event_t* all = malloc(sizeof(event_t) * (tot ? tot : 1));
  int64_t w = 0;
  for (int i = 0; i < nth; ++i) { memcpy(all + w, bufs[i].e, sizeof(event_t) * bufs[i].n); w += bufs[i].n; free(bufs[i].e); }
  free(bufs);
  qsort(all, tot, sizeof(event_t), ev_cmp);
  for (int64_t i = 0; i < tot && i < ev_cap; ++i) {
    int32_t* kk = ev_key + i * (3 + K);
    kk[0] = all[i].p; kk[1] = all[i].q; kk[2] = all[i].k;
    for (int j = 0; j < K; ++j) kk[3 + j] = all[i].g[j];
    ev_ray[i] = all[i].ray; ev_amb[i] = all[i].amb; ev_ratio[i] = all[i].ratio;
  }
  free(all);
  scene_free(&S);
  return tot;
}

/* =====================================================================
 * 6. Exact path geometry from a key by the image method (Sec. I).
 * S_0 = T_p, S_i = mirror of S_{i-1} in plane(g_i); back from X_{k+1} = R_q:
 * X_i = plane(g_i) cut by the line S_i -> X_{i+1}.  Valid when every X_i is
 * inside (inclusive, barycentric margin 1e-9) some triangle of g_i, X_{i-1} and X_{i+1} are strictly
 * on the same side of plane(g_i), and no triangle crosses any leg
 * X_{i-1} -> X_i at parameter s in (1e-9, 1 - 1e-9) (triangles of the two
 * end groups are ignored).  plane(g) is that of the group's lowest triangle.
 * ===================================================================== */
static int in_tri(const scene_t* S, int t, v3 x) {
  v3 a = tv(S, t, 0), b = tv(S, t, 1), c = tv(S, t, 2);
  v3 v0 = sub(b, a), v1 = sub(c, a), v2 = sub(x, a);
  double d00 = dot(v0, v0), d01 = dot(v0, v1), d11 = dot(v1, v1), d20 = dot(v2, v0), d21 = dot(v2, v1);
  double den = d00 * d11 - d01 * d01;
  double v = (d11 * d20 - d01 * d21) / den;
  double w = (d00 * d21 - d01 * d20) / den;
  double u = 1.0 - v - w;
  /* inclusive, with a 1e-9 barycentric margin: a face group is the union of
   * its triangles and a point on a shared edge must not fall through a
   * rounding crack between them */
  return u >= -1e-9 && v >= -1e-9 && w >= -1e-9;
}

static int blocked(const scene_t* S, v3 a, v3 b, int ga, int gb) {
  v3 D = sub(b, a);
  for (int t = 0; t < S->T; ++t) {
    int g = S->group[t];
    if (g == ga || g == gb) continue;
    v3 v0 = tv(S, t, 0);
    v3 e1 = sub(tv(S, t, 1), v0), e2 = sub(tv(S, t, 2), v0);
    v3 pv = crs(D, e2);
    double det = dot(e1, pv);
    if (det == 0.0) continue;
    double inv = 1.0 / det;
    v3 tvec = sub(a, v0);
    double u = dot(tvec, pv) * inv;
    if (u < -1e-9 || u > 1.0 + 1e-9) continue;
    v3 qv = crs(tvec, e1);
    double v = dot(D, qv) * inv;
    if (v < -1e-9 || u + v > 1.0 + 1e-9) continue;  /* same crack-free margin as in_tri */
    double s = dot(e2, qv) * inv;
    if (s > 1e-9 && s < 1.0 - 1e-9) return 1;
  }
  return 0;
}

/* X[0..k+1] out; returns 1 when valid */
static int image_path(const scene_t* S, v3 src, v3 dst, int k, const int32_t* g, v3* X) {
  v3 Sv[17];
  Sv[0] = src;
  for (int i = 1; i <= k; ++i) {
    int t0 = S->gfirst[g[i - 1]];
    v3 n = S->n[t0]; double c = S->c[t0];
    Sv[i] = sub(Sv[i - 1], scl(n, 2.0 * (dot(n, Sv[i - 1]) - c)));
  }
  X[0] = src; X[k + 1] = dst;
  for (int i = k; i >= 1; --i) {
    int t0 = S->gfirst[g[i - 1]];
    v3 n = S->n[t0]; double c = S->c[t0];
    v3 D = sub(X[i + 1], Sv[i]);
    double den = dot(n, D);
    if (den == 0.0) return 0;
    double s = (c - dot(n, Sv[i])) / den;
    X[i] = add(Sv[i], scl(D, s));
  }
  for (int i = 1; i <= k; ++i) {
    int gi = g[i - 1];
    int inside = 0;
    for (int j = S->gstart[gi]; j < S->gstart[gi + 1] && !inside; ++j) inside = in_tri(S, S->gtri[j], X[i]);
    if (!inside) return 0;
    int t0 = S->gfirst[gi];
    double sa = dot(S->n[t0], X[i - 1]) - S->c[t0];
    double sb = dot(S->n[t0], X[i + 1]) - S->c[t0];
    if (!(sa * sb > 0.0)) return 0;
  }
  for (int i = 1; i <= k + 1; ++i) {
    int ga = i - 1 >= 1 ? g[i - 2] : -1;
    int gb = i <= k ? g[i - 1] : -1;
    if (blocked(S, X[i - 1], X[i], ga, gb)) return 0;
  }
  return 1;
}

static void az_el(v3 u, double* az, double* el) {
  *az = atan2(u.y, u.x) * 180.0 / ORC_PI;
  double z = u.z > 1.0 ? 1.0 : (u.z < -1.0 ? -1.0 : u.z);
  *el = asin(z) * 180.0 / ORC_PI;
}

/* rec per key (8 doubles): valid, length, delay, aod_az, aod_el, aoa_az, aoa_el, k */
int orc_paths(const double* tri, int T, const float* eps, const float* sig, const float* rough,
              const double* tx, const double* rx, int K, const int32_t* keys, int64_t n, double* rec) {
  scene_t S; scene_init(&S, tri, T, eps, sig, rough);
#ifdef _OPENMP
#pragma omp parallel for schedule(dynamic, 16)
#endif
  for (int64_t i = 0; i < n; ++i) {
    const int32_t* kk = keys + i * (3 + K);
    int p = kk[0], q = kk[1], k = kk[2];
    v3 X[18];
    double* r = rec + 8 * i;
    for (int j = 0; j < 8; ++j) r[j] = 0.0;
    int ok = image_path(&S, ld(tx + 3 * p), ld(rx + 3 * q), k, kk + 3, X);
    r[0] = ok; r[7] = k;
    if (!ok) continue;
    /* image-method length: distance from the last image to the receiver */
    v3 Sv = ld(tx + 3 * p);
    for (int j = 1; j <= k; ++j) {
      int t0 = S.gfirst[kk[3 + j - 1]];
      Sv = sub(Sv, scl(S.n[t0], 2.0 * (dot(S.n[t0], Sv) - S.c[t0])));
    }
    double len = nrm(sub(ld(rx + 3 * q), Sv));
    r[1] = len; r[2] = len / ORC_C0;
    az_el(unit(sub(X[1], X[0])), &r[3], &r[4]);
    az_el(unit(sub(X[k], X[k + 1])), &r[5], &r[6]);
  }
  scene_free(&S);
  return 0;
}

/* =====================================================================
 * 7. Field of one path at one frequency: eq. (1) restricted to reflections
 * and the free-space factor, with eq. (3) giving Friis for a unit-gain
 * isotropic source (beta = 1, P_t = 1 W), eq. (6)-(8) Kirchhoff-corrected
 * Fresnel coefficients and eq. (9)-(10) applied from per-frequency tables.
 * Full vector tracking: E starts as theta-hat of the departure direction;
 * at each bounce E <- rho [ r_TE (E.s) s + r_TM (E.p_in) p_out ] with
 * s = k x n / |k x n|, p_in = s x k, p_out = s x k'; the receiver projects
 * on theta-hat of the arrival direction.  Time convention e^{+j w t}.
 * ===================================================================== */
typedef struct { double complex x, y, z; } c3;

static v3 theta_hat(v3 u) {
  double st = sqrt(u.x * u.x + u.y * u.y);
  double ct = u.z;
  double cp = 1.0, sp = 0.0;
  if (st > 0.0) { cp = u.x / st; sp = u.y / st; }
  return mk(ct * cp, ct * sp, -st);
}
static v3 phi_hat(v3 u) {
  double phi = atan2(u.y, u.x);  /* atan2(0, 0) = 0 at the poles */
  return mk(-sin(phi), cos(phi), 0.0);
}
/* antenna polarisation: 0 = theta-hat (vertical), 1 = phi-hat (horizontal) */
static v3 pol_vec(v3 u, int pol) { return pol ? phi_hat(u) : theta_hat(u); }

void orc_fresnel(double eps_r, double sigma, double f, double cos_i,
                 double* rte_re, double* rte_im, double* rtm_re, double* rtm_im) {
  double complex ec = eps_r - I * sigma / (2.0 * ORC_PI * f * ORC_EPS0);
  double s2 = 1.0 - cos_i * cos_i;
  double complex root = csqrt(ec - s2);
  double complex te = (cos_i - root) / (cos_i + root);
  double complex tm = (ec * cos_i - root) / (ec * cos_i + root);
  *rte_re = creal(te); *rte_im = cimag(te); *rtm_re = creal(tm); *rtm_im = cimag(tm);
}

double orc_roughness(double rough_std, double f, double cos_i) {
  double lam = ORC_C0 / f;
  double g = pow(4.0 * ORC_PI * rough_std * cos_i / lam, 2.0);
  return exp(-g / 2.0);
}

/* a[n][Nf][2] (re, im); paths that fail validation get 0 */
int orc_field(const double* tri, int T, const float* eps, const float* sig, const float* rough,
              const double* tx, const double* rx, int K, const int32_t* keys, int64_t n,
              const double* freq, int Nf, const float* atm_db, const float* atm_deg, int pol_tx, int pol_rx,
              double* a) {
  scene_t S; scene_init(&S, tri, T, eps, sig, rough);
#ifdef _OPENMP
#pragma omp parallel for schedule(dynamic, 4)
#endif
  for (int64_t i = 0; i < n; ++i) {
    const int32_t* kk = keys + i * (3 + K);
    int p = kk[0], q = kk[1], k = kk[2];
    v3 X[18];
    int ok = image_path(&S, ld(tx + 3 * p), ld(rx + 3 * q), k, kk + 3, X);
    double len = 0.0;
    for (int j = 1; j <= k + 1; ++j) len += nrm(sub(X[j], X[j - 1]));
    for (int fi = 0; fi < Nf; ++fi) {
      double* out = a + 2 * (i * Nf + fi);
      out[0] = out[1] = 0.0;
      if (!ok) continue;
      double f = freq[fi];
      double lam = ORC_C0 / f;
      v3 kd = unit(sub(X[1], X[0]));
      v3 th = pol_vec(kd, pol_tx);
      c3 E = {th.x, th.y, th.z};
      for (int b = 1; b <= k; ++b) {
        int gi = kk[3 + b - 1];
        int t0 = S.gfirst[gi];
        v3 nn = S.n[t0];
        if (dot(kd, nn) > 0) nn = scl(nn, -1.0);
        double cs = -dot(kd, nn);
        double rte_re, rte_im, rtm_re, rtm_im;
        orc_fresnel(eps[t0], sig[t0], f, cs, &rte_re, &rte_im, &rtm_re, &rtm_im);
        double complex rte = rte_re + I * rte_im, rtm = rtm_re + I * rtm_im;
        double rho = orc_roughness(rough[t0], f, cs);
        v3 s = crs(kd, nn);
        double sn = nrm(s);
        if (sn < 1e-15) {
          /* normal incidence: any unit vector orthogonal to k */
          v3 tmp = fabs(kd.x) < 0.9 ? mk(1, 0, 0) : mk(0, 1, 0);
          s = unit(crs(kd, tmp));
        } else {
          s = scl(s, 1.0 / sn);
        }
        v3 pin = crs(s, kd);
        v3 kr = sub(kd, scl(nn, 2.0 * dot(kd, nn)));
        v3 pout = crs(s, kr);
        double complex es = E.x * s.x + E.y * s.y + E.z * s.z;
        double complex ep = E.x * pin.x + E.y * pin.y + E.z * pin.z;
        double complex cs_ = rho * rte * es, cp_ = rho * rtm * ep;
        E.x = cs_ * s.x + cp_ * pout.x;
        E.y = cs_ * s.y + cp_ * pout.y;
        E.z = cs_ * s.z + cp_ * pout.z;
        kd = kr;
      }
      v3 tr = pol_vec(kd, pol_rx);
      double complex pol = E.x * tr.x + E.y * tr.y + E.z * tr.z;
      double amp = lam / (4.0 * ORC_PI * len);
      if (atm_db) amp *= pow(10.0, -(double)atm_db[fi] * len / 20.0);
      double cyc = f * len / ORC_C0;
      double ph = 2.0 * ORC_PI * (cyc - floor(cyc));
      if (atm_deg) ph += ORC_PI * (double)atm_deg[fi] * len / 180.0;
      double complex v = amp * pol * cexp(-I * ph);
      out[0] = creal(v); out[1] = cimag(v);
    }
  }
  scene_free(&S);
  return 0;
}
