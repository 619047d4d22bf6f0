/*
 * CPU ORACLE for the FE-LLG island solver -- TEST INFRASTRUCTURE ONLY.
 *
 * Plain, slow, FP64 reference of what the GPU path computes.  Only the test-suite, the smoke
 * check and the CPU-baseline leg of the benchmark may load it.  It shares no code, header,
 * table or helper with the GPU library; both consume the same seeded inputs.
 *
 * What it follows (Kovacs et al., J. Appl. Phys. 120, 013902 (2016)):
 *   - Sec. II.A: the recording simulation solves the Landau-Lifshitz-Gilbert equation at 0 K for
 *     the media island in the precomputed head field, moved down-track and scaled by a 0.1 ns
 *     rise (the paper's solver is a hybrid FE/BE code; here a P1 tetrahedral FE discretisation
 *     with a dense per-island magnetostatic operator).
 *   - Sec. II.B / Fig. 3: exchange-coupled composite island, soft layer + hard layer coupled
 *     through a 1 nm interlayer with exchange constant A_ex,int; aligned easy axes.
 *   - Sec. II.C: an extra uniform field H_ext added to the head field; switching of the target
 *     bit decides writing success.  The stochastic LLG (thermal field) of the attempt-frequency
 *     calculation in Sec. II.C is the Heun integrator below.
 * Everything the paper leaves open (time integrator, error norm, demag operator, switching
 * criterion, thermal-field variance, random numbers) follows one stated reading, given in the
 * comment of the function that implements it.
 *
 * Precision: IEEE double throughout.  Parallelism: OpenMP across independent systems only.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define OR_PI 3.14159265358979323846
#define OR_MU0 (4.0e-7 * OR_PI)          /* T m / A, SI definition before 2019 */
#define OR_GAMMA 1.76085963023e11        /* rad / (s T), electron gyromagnetic ratio (CODATA) */
#define OR_KB 1.380649e-23               /* J / K */

enum { OR_OK = 0, OR_EINVAL = -1, OR_ENOMEM = -2, OR_ENONFINITE = -5, OR_ESTEPUNDERFLOW = -6,
       OR_EMAXSTEPS = -7 };
enum { OR_DP45 = 0, OR_DP5_FIXED = 1, OR_HEUN = 2 };
enum { OR_FIELD_UNIFORM = 0, OR_FIELD_POLE = 1, OR_FIELD_GRID = 2 };

/* ------------------------------------------------------------------------------------------ */
/* Public structs (mirrored by ctypes in oracle.py)                                            */
/* ------------------------------------------------------------------------------------------ */
typedef struct {
  double Ms[2], K[2], A[2], axis[2][3];   /* index 0 soft, 1 hard */
  double A_int, delta_int, alpha;
} or_material;

typedef struct {
  int32_t kind, pad_;
  double B_peak, dir[3], t_rise, v[3], x_off[3], L_grad, W_pole, B_ext[3];
  const float *grid;           /* OR_FIELD_GRID: [3][nz][ny][nx] tesla */
  int32_t nx, ny, nz, pad2_;
  double g_origin[3], g_h;
} or_field;

typedef struct {
  int32_t integrator, save_every;
  double t_end, dt0, dt_fixed, rtol, atol, dt_min, temperature;
  int64_t max_steps;
  int32_t relax, pad_;         /* relax != 0: no precession term (energy descent) */
} or_opts;

typedef struct {
  int32_t status, switched;
  double t_sw, B_sw, mz_soft, mz_hard, t_reached, energy;
  int64_t n_accept, n_reject;
  double dt_min_used, dt_max_used, max_norm_dev;
} or_result;

typedef struct {
  int n, ntet, nif, nnz;
  double *x, *y, *z;
  int *tet, *layer, *iface;
  double *tetV, *grad, *V;
  int *rowptr, *col;
  double *K, *D, *aif;
  int *ifpart;          /* [n]: partner node across the interface, or -1 */
  int *ifidx;           /* [n]: interface pair index, or -1 */
  int *n2t_ptr, *n2t;   /* node -> tets */
  double centroid[3];
  double vol_layer[2];
} or_mesh;

/* ------------------------------------------------------------------------------------------ */
/* Mesh quantities: P1 volumes, gradients, stiffness, charge operator, interface areas        */
/* ------------------------------------------------------------------------------------------ */
static int cmp_i64(const void *a, const void *b) {
  int64_t x = *(const int64_t *)a, y = *(const int64_t *)b;
  return (x > y) - (x < y);
}

static int csr_find(const or_mesh *M, int i, int j) {
  int lo = M->rowptr[i], hi = M->rowptr[i + 1] - 1;
  while (lo <= hi) {
    int mid = (lo + hi) / 2;
    if (M->col[mid] == j) return mid;
    if (M->col[mid] < j) lo = mid + 1; else hi = mid - 1;
  }
  return -1;
}

static void cross3(const double *a, const double *b, double *c) {
  c[0] = a[1] * b[2] - a[2] * b[1];
  c[1] = a[2] * b[0] - a[0] * b[2];
  c[2] = a[0] * b[1] - a[1] * b[0];
}

void or_mesh_free(or_mesh *M) {
  if (!M) return;
  free(M->x); free(M->y); free(M->z); free(M->tet); free(M->layer); free(M->iface);
  free(M->tetV); free(M->grad); free(M->V); free(M->rowptr); free(M->col); free(M->K);
  free(M->D); free(M->aif); free(M->ifpart); free(M->ifidx); free(M->n2t_ptr); free(M->n2t);
  free(M);
}

/* Builds every mesh quantity of the P1 discretisation:
 *   V_e, grad(phi_a)|_e, lumped V_i = sum_e V_e / 4,
 *   K_ij = sum_e V_e grad(phi_i).grad(phi_j)                      (exchange stiffness)
 *   D_{k,(j,alpha)} = sum_{e contains j,k} (V_e/4) d_alpha phi_k   (charge operator b = D (Ms m))
 *   a_p = sum over interface faces containing p of area/3          (lumped interface area)     */
or_mesh *or_mesh_create(int n, int ntet, const double *xyz, const int32_t *tet,
                        const int32_t *layer, int nif, const int32_t *iface) {
  if (n <= 0 || ntet <= 0 || nif < 0) return NULL;
  or_mesh *M = (or_mesh *)calloc(1, sizeof(or_mesh));
  M->n = n; M->ntet = ntet; M->nif = nif;
  M->x = malloc(sizeof(double) * n); M->y = malloc(sizeof(double) * n);
  M->z = malloc(sizeof(double) * n);
  memcpy(M->x, xyz, sizeof(double) * n);
  memcpy(M->y, xyz + n, sizeof(double) * n);
  memcpy(M->z, xyz + 2 * n, sizeof(double) * n);
  M->tet = malloc(sizeof(int) * 4 * ntet);
  for (int i = 0; i < 4 * ntet; i++) {
    M->tet[i] = tet[i];
    if (tet[i] < 0 || tet[i] >= n) { or_mesh_free(M); return NULL; }
  }
  M->layer = malloc(sizeof(int) * n);
  for (int i = 0; i < n; i++) M->layer[i] = layer[i];
  M->iface = malloc(sizeof(int) * 2 * (nif > 0 ? nif : 1));
  for (int i = 0; i < 2 * nif; i++) M->iface[i] = iface[i];

  /* volumes and gradients */
  M->tetV = malloc(sizeof(double) * ntet);
  M->grad = malloc(sizeof(double) * 12 * ntet);
  M->V = calloc(n, sizeof(double));
  for (int e = 0; e < ntet; e++) {
    const int *t = M->tet + 4 * e;
    double p[4][3];
    for (int a = 0; a < 4; a++) { p[a][0] = M->x[t[a]]; p[a][1] = M->y[t[a]]; p[a][2] = M->z[t[a]]; }
    double e1[3], e2[3], e3[3];
    for (int c = 0; c < 3; c++) { e1[c] = p[1][c] - p[0][c]; e2[c] = p[2][c] - p[0][c]; e3[c] = p[3][c] - p[0][c]; }
    double c23[3], c31[3], c12[3];
    cross3(e2, e3, c23); cross3(e3, e1, c31); cross3(e1, e2, c12);
    double det = e1[0] * c23[0] + e1[1] * c23[1] + e1[2] * c23[2];
    double *g = M->grad + 12 * e;
    for (int c = 0; c < 3; c++) {
      g[3 + c] = c23[c] / det;
      g[6 + c] = c31[c] / det;
      g[9 + c] = c12[c] / det;
      g[c] = -(g[3 + c] + g[6 + c] + g[9 + c]);
    }
    M->tetV[e] = fabs(det) / 6.0;
    for (int a = 0; a < 4; a++) M->V[t[a]] += M->tetV[e] / 4.0;
  }

  /* CSR pattern: pairs of nodes sharing a tet (diagonal included) */
  int64_t *keys = malloc(sizeof(int64_t) * 16 * (size_t)ntet);
  for (int e = 0; e < ntet; e++)
    for (int a = 0; a < 4; a++)
      for (int b = 0; b < 4; b++)
        keys[16 * (size_t)e + 4 * a + b] = (int64_t)M->tet[4 * e + a] * n + M->tet[4 * e + b];
  qsort(keys, 16 * (size_t)ntet, sizeof(int64_t), cmp_i64);
  size_t nu = 0;
  for (size_t i = 0; i < 16 * (size_t)ntet; i++)
    if (i == 0 || keys[i] != keys[i - 1]) keys[nu++] = keys[i];
  M->nnz = (int)nu;
  M->rowptr = calloc(n + 1, sizeof(int));
  M->col = malloc(sizeof(int) * nu);
  for (size_t i = 0; i < nu; i++) {
    int r = (int)(keys[i] / n);
    M->col[i] = (int)(keys[i] % n);
    M->rowptr[r + 1]++;
  }
  for (int i = 0; i < n; i++) M->rowptr[i + 1] += M->rowptr[i];
  free(keys);

  M->K = calloc(nu, sizeof(double));
  M->D = calloc(3 * nu, sizeof(double));
  for (int e = 0; e < ntet; e++) {
    const int *t = M->tet + 4 * e;
    const double *g = M->grad + 12 * e;
    double Ve = M->tetV[e];
    for (int a = 0; a < 4; a++)
      for (int b = 0; b < 4; b++) {
        int pos = csr_find(M, t[a], t[b]);
        M->K[pos] += Ve * (g[3 * a] * g[3 * b] + g[3 * a + 1] * g[3 * b + 1] + g[3 * a + 2] * g[3 * b + 2]);
        /* row k = t[a] (test function gradient), column j = t[b] (magnetisation node) */
        for (int c = 0; c < 3; c++) M->D[3 * pos + c] += 0.25 * Ve * g[3 * a + c];
      }
  }

  /* interface: partner map and lumped areas from the faces lying on the interface */
  M->ifpart = malloc(sizeof(int) * n);
  M->ifidx = malloc(sizeof(int) * n);
  for (int i = 0; i < n; i++) { M->ifpart[i] = -1; M->ifidx[i] = -1; }
  for (int p = 0; p < nif; p++) {
    int s = M->iface[2 * p], h = M->iface[2 * p + 1];
    M->ifpart[s] = h; M->ifpart[h] = s; M->ifidx[s] = p; M->ifidx[h] = p;
  }
  M->aif = calloc(nif > 0 ? nif : 1, sizeof(double));
  double *aside[2];
  aside[0] = calloc(nif > 0 ? nif : 1, sizeof(double));
  aside[1] = calloc(nif > 0 ? nif : 1, sizeof(double));
  for (int e = 0; e < ntet; e++) {
    const int *t = M->tet + 4 * e;
    for (int skip = 0; skip < 4; skip++) {
      int f[3], k = 0, ok = 1;
      for (int a = 0; a < 4; a++) if (a != skip) f[k++] = t[a];
      for (int a = 0; a < 3; a++) if (M->ifidx[f[a]] < 0) ok = 0;
      if (!ok) continue;
      int L = M->layer[f[0]];
      if (M->layer[f[1]] != L || M->layer[f[2]] != L) continue;
      double u[3] = {M->x[f[1]] - M->x[f[0]], M->y[f[1]] - M->y[f[0]], M->z[f[1]] - M->z[f[0]]};
      double w[3] = {M->x[f[2]] - M->x[f[0]], M->y[f[2]] - M->y[f[0]], M->z[f[2]] - M->z[f[0]]};
      double c[3];
      cross3(u, w, c);
      double area = 0.5 * sqrt(c[0] * c[0] + c[1] * c[1] + c[2] * c[2]);
      for (int a = 0; a < 3; a++) aside[L][M->ifidx[f[a]]] += area / 3.0;
    }
  }
  for (int p = 0; p < nif; p++) M->aif[p] = 0.5 * (aside[0][p] + aside[1][p]);
  free(aside[0]); free(aside[1]);

  /* node -> tet adjacency */
  M->n2t_ptr = calloc(n + 1, sizeof(int));
  for (int i = 0; i < 4 * ntet; i++) M->n2t_ptr[M->tet[i] + 1]++;
  for (int i = 0; i < n; i++) M->n2t_ptr[i + 1] += M->n2t_ptr[i];
  M->n2t = malloc(sizeof(int) * 4 * ntet);
  int *fill = calloc(n, sizeof(int));
  for (int e = 0; e < ntet; e++)
    for (int a = 0; a < 4; a++) {
      int i = M->tet[4 * e + a];
      M->n2t[M->n2t_ptr[i] + fill[i]++] = e;
    }
  free(fill);

  double vs = 0.0, c[3] = {0, 0, 0};
  M->vol_layer[0] = M->vol_layer[1] = 0.0;
  for (int i = 0; i < n; i++) {
    vs += M->V[i];
    c[0] += M->V[i] * M->x[i]; c[1] += M->V[i] * M->y[i]; c[2] += M->V[i] * M->z[i];
    M->vol_layer[M->layer[i] ? 1 : 0] += M->V[i];
  }
  for (int k = 0; k < 3; k++) M->centroid[k] = c[k] / vs;
  return M;
}

int or_mesh_nnz(const or_mesh *M) { return M->nnz; }

void or_mesh_export(const or_mesh *M, double *V, int32_t *rowptr, int32_t *col, double *K,
                    double *D, double *aif, double *tetV, double *centroid) {
  if (V) memcpy(V, M->V, sizeof(double) * M->n);
  if (rowptr) for (int i = 0; i <= M->n; i++) rowptr[i] = M->rowptr[i];
  if (col) for (int i = 0; i < M->nnz; i++) col[i] = M->col[i];
  if (K) memcpy(K, M->K, sizeof(double) * M->nnz);
  if (D) memcpy(D, M->D, sizeof(double) * 3 * M->nnz);
  if (aif) memcpy(aif, M->aif, sizeof(double) * (M->nif > 0 ? M->nif : 0));
  if (tetV) memcpy(tetV, M->tetV, sizeof(double) * M->ntet);
  if (centroid) memcpy(centroid, M->centroid, sizeof(double) * 3);
}

/* ------------------------------------------------------------------------------------------ */
/* Demag operator S:  E_d = (mu0/2) b^T S b,  S_kl = (1/(V_k V_l)) <phi_k | G | phi_l>         */
/* The charge density of node k, phi_k / V_k, is sampled at the centroids of the tets around   */
/* it (weight V_e/4 each) and every sample is smeared as an isotropic Gaussian of standard    */
/* deviation beta * V_e^(1/3); two such blobs interact through erf(r/sqrt(2 s^2)) / (4 pi r). */
/* ------------------------------------------------------------------------------------------ */
static double blob_kernel(const double *ca, double sa, const double *cb, double sb) {
  double dx = ca[0] - cb[0], dy = ca[1] - cb[1], dz = ca[2] - cb[2];
  double r = sqrt(dx * dx + dy * dy + dz * dz);
  double s2 = sa * sa + sb * sb;
  if (r == 0.0) return sqrt(2.0 / OR_PI) / sqrt(s2) / (4.0 * OR_PI);
  return erf(r / sqrt(2.0 * s2)) / (4.0 * OR_PI * r);
}

static void tet_centroids(const or_mesh *M, double beta, double *c, double *s) {
  for (int e = 0; e < M->ntet; e++) {
    const int *t = M->tet + 4 * e;
    c[3 * e] = c[3 * e + 1] = c[3 * e + 2] = 0.0;
    for (int a = 0; a < 4; a++) {
      c[3 * e] += 0.25 * M->x[t[a]]; c[3 * e + 1] += 0.25 * M->y[t[a]]; c[3 * e + 2] += 0.25 * M->z[t[a]];
    }
    s[e] = beta * cbrt(M->tetV[e]);
  }
}

int or_demag_S(const or_mesh *M, double beta, double *S) {
  int n = M->n, nt = M->ntet;
  double *c = malloc(sizeof(double) * 3 * nt), *s = malloc(sizeof(double) * nt);
  double *GT = calloc((size_t)nt * n, sizeof(double));
  if (!c || !s || !GT) { free(c); free(s); free(GT); return OR_ENOMEM; }
  tet_centroids(M, beta, c, s);
  /* GT[e][l] = sum_f G_ef T_fl with T_fl = (V_f/4)/V_l */
#pragma omp parallel for schedule(dynamic, 16)
  for (int e = 0; e < nt; e++) {
    double *row = GT + (size_t)e * n;
    for (int f = 0; f < nt; f++) {
      double g = blob_kernel(c + 3 * e, s[e], c + 3 * f, s[f]);
      for (int b = 0; b < 4; b++) {
        int l = M->tet[4 * f + b];
        row[l] += g * 0.25 * M->tetV[f] / M->V[l];
      }
    }
  }
  /* S[k][l] = sum_{e contains k} T_ek GT[e][l] */
#pragma omp parallel for schedule(dynamic, 16)
  for (int k = 0; k < n; k++) {
    double *Sk = S + (size_t)k * n;
    for (int l = 0; l < n; l++) Sk[l] = 0.0;
    for (int q = M->n2t_ptr[k]; q < M->n2t_ptr[k + 1]; q++) {
      int e = M->n2t[q];
      double w = 0.25 * M->tetV[e] / M->V[k];
      const double *row = GT + (size_t)e * n;
      for (int l = 0; l < n; l++) Sk[l] += w * row[l];
    }
  }
  free(c); free(s); free(GT);
  return OR_OK;
}

/* A single entry S_kl by the double sum over the two node supports (for spot checks). */
double or_demag_S_entry(const or_mesh *M, double beta, int k, int l) {
  double acc = 0.0;
  for (int q = M->n2t_ptr[k]; q < M->n2t_ptr[k + 1]; q++) {
    int e = M->n2t[q];
    double ce[3] = {0, 0, 0};
    for (int a = 0; a < 4; a++) {
      int i = M->tet[4 * e + a];
      ce[0] += 0.25 * M->x[i]; ce[1] += 0.25 * M->y[i]; ce[2] += 0.25 * M->z[i];
    }
    double se = beta * cbrt(M->tetV[e]);
    for (int r = M->n2t_ptr[l]; r < M->n2t_ptr[l + 1]; r++) {
      int f = M->n2t[r];
      double cf[3] = {0, 0, 0};
      for (int a = 0; a < 4; a++) {
        int i = M->tet[4 * f + a];
        cf[0] += 0.25 * M->x[i]; cf[1] += 0.25 * M->y[i]; cf[2] += 0.25 * M->z[i];
      }
      double sf = beta * cbrt(M->tetV[f]);
      acc += (0.25 * M->tetV[e] / M->V[k]) * (0.25 * M->tetV[f] / M->V[l]) *
             blob_kernel(ce, se, cf, sf);
    }
  }
  return acc;
}

/* ------------------------------------------------------------------------------------------ */
/* Applied field (Sec. II.A/II.C: head field moved down-track, scaled by the rise; plus H_ext)  */
/* ------------------------------------------------------------------------------------------ */
static double rise(const or_field *F, double t) {
  if (F->t_rise <= 0.0) return 1.0;
  double r = t / F->t_rise;
  return r < 1.0 ? r : 1.0;
}

/* Field grid (the precomputed head field handed to the recording simulation, Sec. II.A):
 * trilinear interpolation of the node vectors at the field-frame point s; zero outside the box
 * spanned by the nodes.  Node (i, j, k) sits at g_origin + g_h (i, j, k). */
static void grid_field(const or_field *F, const double *s, double *G) {
  const int n[3] = {F->nx, F->ny, F->nz};
  int lo[3];
  double f[3];
  G[0] = G[1] = G[2] = 0.0;
  for (int a = 0; a < 3; a++) {
    double u = (s[a] - F->g_origin[a]) / F->g_h;
    if (u < 0.0 || u > (double)(n[a] - 1)) return;
    int i = (int)floor(u);
    if (i > n[a] - 2) i = n[a] - 2;
    lo[a] = i;
    f[a] = u - i;
  }
  size_t per_comp = (size_t)n[0] * n[1] * n[2];
  for (int corner = 0; corner < 8; corner++) {
    int ix = lo[0] + (corner & 1), iy = lo[1] + ((corner >> 1) & 1), iz = lo[2] + ((corner >> 2) & 1);
    double w = ((corner & 1) ? f[0] : 1.0 - f[0]) * (((corner >> 1) & 1) ? f[1] : 1.0 - f[1]) *
               (((corner >> 2) & 1) ? f[2] : 1.0 - f[2]);
    size_t node = ((size_t)iz * n[1] + iy) * n[0] + ix;
    for (int c = 0; c < 3; c++) G[c] += w * (double)F->grid[c * per_comp + node];
  }
}

static void applied_B(const or_field *F, double t, double x, double y, double z, double *B) {
  double amp = F->B_peak * rise(F, t);
  double dir[3] = {F->dir[0], F->dir[1], F->dir[2]};
  if (F->kind == OR_FIELD_POLE) {
    double sx = x - F->x_off[0] - F->v[0] * t;
    double sy = y - F->x_off[1] - F->v[1] * t;
    double fx = 0.5 * (1.0 - tanh(sx / F->L_grad));
    double fy = 0.5 * (tanh((sy + 0.5 * F->W_pole) / F->L_grad) - tanh((sy - 0.5 * F->W_pole) / F->L_grad));
    amp *= fx * fy;
  } else if (F->kind == OR_FIELD_GRID) {
    double sp[3] = {x - F->x_off[0] - F->v[0] * t, y - F->x_off[1] - F->v[1] * t, z - F->x_off[2] - F->v[2] * t};
    grid_field(F, sp, dir);
  }
  for (int c = 0; c < 3; c++) B[c] = amp * dir[c] + F->B_ext[c];
}

/* ------------------------------------------------------------------------------------------ */
/* Effective field B = mu0 H_eff (tesla) of one instance, term by term, and its energy         */
/*   exchange    B_ex,i  = -(2 A_L / (Ms_L V_i)) (K m)_i                                       */
/*   anisotropy  B_an,i  = (2 K_L / Ms_L) (m_i . u_L) u_L                                      */
/*   interlayer  B_int,i = (A_int / delta) a_p / (Ms_L V_i) m_partner                          */
/*   demag       b = D (Ms m), u = S b, B_d,j = -(mu0 / V_j) (D^T u)_j                         */
/*   Zeeman      B_app(x_i + offset, t)                                                       */
/*   dipoles     B_dip (uniform over the island, supplied by the caller)                      */
/* E = E_ex + E_an + E_int + E_d + E_Z with each term the energy whose negative variational    */
/* derivative, divided by the node moment w_i = Ms_L V_i, is the field above.                 */
/* ------------------------------------------------------------------------------------------ */
typedef struct { double *b, *u, *Km, *Dtu; } or_work;

static void field_terms(const or_mesh *M, const double *S, const or_material *mat,
                        const or_field *F, const double *off, double t, const double *m,
                        const double *Bdip, double *Btot, double *terms, double *E, or_work *W) {
  int n = M->n;
  const double *mx = m, *my = m + n, *mz = m + 2 * n;
  /* exchange operator K m and charges b = D (Ms m) */
  for (int i = 0; i < n; i++) {
    double k0 = 0, k1 = 0, k2 = 0, bb = 0;
    for (int q = M->rowptr[i]; q < M->rowptr[i + 1]; q++) {
      int j = M->col[q];
      double Msj = mat->Ms[M->layer[j] ? 1 : 0];
      k0 += M->K[q] * mx[j]; k1 += M->K[q] * my[j]; k2 += M->K[q] * mz[j];
      bb += Msj * (M->D[3 * q] * mx[j] + M->D[3 * q + 1] * my[j] + M->D[3 * q + 2] * mz[j]);
    }
    W->Km[i] = k0; W->Km[n + i] = k1; W->Km[2 * n + i] = k2;
    W->b[i] = bb;
  }
  /* potentials u = S b (dense) */
  if (S) {
    for (int k = 0; k < n; k++) {
      double acc = 0.0;
      const double *Sk = S + (size_t)k * n;
      for (int l = 0; l < n; l++) acc += Sk[l] * W->b[l];
      W->u[k] = acc;
    }
  } else {
    for (int k = 0; k < n; k++) W->u[k] = 0.0;
  }
  double Eex = 0, Ean = 0, Eint = 0, Ed = 0, EZ = 0;
  /* (D^T u)_j = sum_k D_{k,j} u_k: walk rows k, scatter to columns j */
  double *Dtu = W->Dtu;
  for (int i = 0; i < 3 * n; i++) Dtu[i] = 0.0;
  for (int k = 0; k < n; k++)
    for (int q = M->rowptr[k]; q < M->rowptr[k + 1]; q++) {
      int j = M->col[q];
      Dtu[j] += M->D[3 * q] * W->u[k];
      Dtu[n + j] += M->D[3 * q + 1] * W->u[k];
      Dtu[2 * n + j] += M->D[3 * q + 2] * W->u[k];
    }
  for (int i = 0; i < n; i++) {
    int L = M->layer[i] ? 1 : 0;
    double Ms = mat->Ms[L], Vi = M->V[i], w = Ms * Vi;
    double mi[3] = {mx[i], my[i], mz[i]};
    double bex[3], ban[3], bint[3] = {0, 0, 0}, bd[3], bz[3];
    double cex = -2.0 * mat->A[L] / (Ms * Vi);
    for (int c = 0; c < 3; c++) bex[c] = cex * W->Km[c * n + i];
    const double *u = mat->axis[L];
    double mu = mi[0] * u[0] + mi[1] * u[1] + mi[2] * u[2];
    for (int c = 0; c < 3; c++) ban[c] = 2.0 * mat->K[L] / Ms * mu * u[c];
    int p = M->ifidx[i];
    if (p >= 0) {
      int j = M->ifpart[i];
      double cint = mat->A_int / mat->delta_int * M->aif[p] / w;
      bint[0] = cint * mx[j]; bint[1] = cint * my[j]; bint[2] = cint * mz[j];
    }
    for (int c = 0; c < 3; c++) bd[c] = -OR_MU0 / Vi * Dtu[c * n + i];
    applied_B(F, t, M->x[i] + off[0], M->y[i] + off[1], M->z[i] + off[2], bz);
    for (int c = 0; c < 3; c++) {
      double bdip = Bdip ? Bdip[c] : 0.0;
      Btot[c * n + i] = bex[c] + ban[c] + bint[c] + bd[c] + bz[c] + bdip;
      if (terms) {
        terms[(0 * 3 + c) * n + i] = bex[c];
        terms[(1 * 3 + c) * n + i] = ban[c];
        terms[(2 * 3 + c) * n + i] = bint[c];
        terms[(3 * 3 + c) * n + i] = bd[c];
        terms[(4 * 3 + c) * n + i] = bz[c];
      }
    }
    if (E) {
      Eex += mat->A[L] * (mi[0] * W->Km[i] + mi[1] * W->Km[n + i] + mi[2] * W->Km[2 * n + i]);
      Ean += -mat->K[L] * Vi * mu * mu;
      if (p >= 0 && L == 0) {
        int j = M->ifpart[i];
        Eint += -mat->A_int / mat->delta_int * M->aif[p] * (mi[0] * mx[j] + mi[1] * my[j] + mi[2] * mz[j]);
      }
      EZ += -w * (mi[0] * bz[0] + mi[1] * bz[1] + mi[2] * bz[2]);
      Ed += 0.5 * OR_MU0 * W->b[i] * W->u[i];
    }
  }
  if (E) { E[0] = Eex; E[1] = Ean; E[2] = Eint; E[3] = Ed; E[4] = EZ; }
}

static void instance_moment(const or_mesh *M, const or_material *mat, const double *m, double *mu) {
  int n = M->n;
  mu[0] = mu[1] = mu[2] = 0.0;
  for (int i = 0; i < n; i++) {
    double w = mat->Ms[M->layer[i] ? 1 : 0] * M->V[i];
    mu[0] += w * m[i]; mu[1] += w * m[n + i]; mu[2] += w * m[2 * n + i];
  }
}

/* Point-dipole field (tesla) at r_J from moment mu at r_I: mu0 (3 (mu.rhat) rhat - mu)/(4 pi r^3) */
static void dipole_B(const double *rJ, const double *rI, const double *mu, double *B) {
  double d[3] = {rJ[0] - rI[0], rJ[1] - rI[1], rJ[2] - rI[2]};
  double r = sqrt(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]);
  double rh[3] = {d[0] / r, d[1] / r, d[2] / r};
  double mr = mu[0] * rh[0] + mu[1] * rh[1] + mu[2] * rh[2];
  double c = OR_MU0 / (4.0 * OR_PI * r * r * r);
  for (int k = 0; k < 3; k++) B[k] = c * (3.0 * mr * rh[k] - mu[k]);
}

/* Exported single-instance field/energy evaluation (used by the pins). */
int or_fields(const or_mesh *M, const double *S, const or_material *mat, const or_field *F,
              const double *off, double t, const double *m, const double *Bdip, double *Btot,
              double *terms, double *E) {
  int n = M->n;
  or_work W;
  W.b = malloc(sizeof(double) * n); W.u = malloc(sizeof(double) * n);
  W.Km = malloc(sizeof(double) * 3 * n); W.Dtu = malloc(sizeof(double) * 3 * n);
  double zero[3] = {0, 0, 0};
  field_terms(M, S, mat, F, off ? off : zero, t, m, Bdip, Btot, terms, E, &W);
  free(W.b); free(W.u); free(W.Km); free(W.Dtu);
  return OR_OK;
}

/* ------------------------------------------------------------------------------------------ */
/* LLG right-hand side (Landau-Lifshitz form of the Gilbert equation, Sec. II.A):              */
/*   dm/dt = -gamma/(1+alpha^2) [ m x B + alpha m x (m x B) ]                                 */
/* prec = 0 drops the precession term m x B: the damping term alone moves m down the energy   */
/* (the relaxation used by the string method for the energy barrier of Sec. II.C).            */
/* ------------------------------------------------------------------------------------------ */
static void llg_rhs(int n, double alpha, double prec, const double *m, const double *B, double *dm) {
  double gp = OR_GAMMA / (1.0 + alpha * alpha);
  for (int i = 0; i < n; i++) {
    double mi[3] = {m[i], m[n + i], m[2 * n + i]};
    double b[3] = {B[i], B[n + i], B[2 * n + i]};
    double mxb[3], mxmxb[3];
    cross3(mi, b, mxb);
    cross3(mi, mxb, mxmxb);
    for (int c = 0; c < 3; c++) dm[c * n + i] = -gp * (prec * mxb[c] + alpha * mxmxb[c]);
  }
}

int or_llg_rhs(int n, double alpha, const double *m, const double *B, double *dm) {
  llg_rhs(n, alpha, 1.0, m, B, dm);
  return OR_OK;
}

/* ------------------------------------------------------------------------------------------ */
/* Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11) and Box-Muller Gaussians                  */
/* ------------------------------------------------------------------------------------------ */
static void philox_round(uint32_t *c, const uint32_t *k) {
  uint64_t p0 = (uint64_t)0xD2511F53u * c[0];
  uint64_t p1 = (uint64_t)0xCD9E8D57u * c[2];
  uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
  uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
  uint32_t n0 = hi1 ^ c[1] ^ k[0];
  uint32_t n2 = hi0 ^ c[3] ^ k[1];
  c[0] = n0; c[1] = lo1; c[2] = n2; c[3] = lo0;
}

void or_philox4x32_10(const uint32_t *ctr, const uint32_t *key, uint32_t *out) {
  uint32_t c[4] = {ctr[0], ctr[1], ctr[2], ctr[3]};
  uint32_t k[2] = {key[0], key[1]};
  for (int r = 0; r < 10; r++) {
    if (r > 0) { k[0] += 0x9E3779B9u; k[1] += 0xBB67AE85u; }
    philox_round(c, k);
  }
  out[0] = c[0]; out[1] = c[1]; out[2] = c[2]; out[3] = c[3];
}

/* Three standard normals for (key, step, node): counter = (step_lo, step_hi, node, 0);
 * uniforms u = (x + 1/2) 2^-32 lie in (0,1); Box-Muller on (u0,u1) and (u2,u3). */
void or_gauss3(const uint32_t *key, uint64_t step, uint32_t node, double *g) {
  uint32_t ctr[4] = {(uint32_t)step, (uint32_t)(step >> 32), node, 0u}, x[4];
  or_philox4x32_10(ctr, key, x);
  double u[4];
  for (int i = 0; i < 4; i++) u[i] = ((double)x[i] + 0.5) * (1.0 / 4294967296.0);
  double r0 = sqrt(-2.0 * log(u[0])), r1 = sqrt(-2.0 * log(u[2]));
  g[0] = r0 * cos(2.0 * OR_PI * u[1]);
  g[1] = r0 * sin(2.0 * OR_PI * u[1]);
  g[2] = r1 * cos(2.0 * OR_PI * u[3]);
}

/* ------------------------------------------------------------------------------------------ */
/* Systems and time integration                                                               */
/* ------------------------------------------------------------------------------------------ */
typedef struct {
  const or_mesh *M;
  const double *S;
  int R;                       /* instances in this system (>1 only when dipole-coupled) */
  const or_material *mat;      /* [R] */
  const or_field *fld;         /* [R] */
  const double *off;           /* [R][3] */
  int coupled;
  or_work W;
  double *Bbuf;                /* [3n] */
  double *Bdip;                /* [R][3] */
  double *mom;                 /* [R][3] */
  int relax;                   /* drop the precession term */
} or_system;

static void sys_init(or_system *Y) {
  int n = Y->M->n;
  Y->W.b = malloc(sizeof(double) * n); Y->W.u = malloc(sizeof(double) * n);
  Y->W.Km = malloc(sizeof(double) * 3 * n); Y->W.Dtu = malloc(sizeof(double) * 3 * n);
  Y->Bbuf = malloc(sizeof(double) * 3 * n);
  Y->Bdip = calloc(3 * Y->R, sizeof(double));
  Y->mom = calloc(3 * Y->R, sizeof(double));
}

static void sys_free(or_system *Y) {
  free(Y->W.b); free(Y->W.u); free(Y->W.Km); free(Y->W.Dtu); free(Y->Bbuf); free(Y->Bdip); free(Y->mom);
}

static void sys_dipoles(or_system *Y, const double *y) {
  int n = Y->M->n, R = Y->R;
  for (int r = 0; r < 3 * R; r++) Y->Bdip[r] = 0.0;
  if (!Y->coupled || R < 2) return;
  for (int r = 0; r < R; r++) instance_moment(Y->M, &Y->mat[r], y + (size_t)r * 3 * n, Y->mom + 3 * r);
  for (int J = 0; J < R; J++) {
    double rJ[3] = {Y->M->centroid[0] + Y->off[3 * J], Y->M->centroid[1] + Y->off[3 * J + 1],
                    Y->M->centroid[2] + Y->off[3 * J + 2]};
    for (int I = 0; I < R; I++) {
      if (I == J) continue;
      double rI[3] = {Y->M->centroid[0] + Y->off[3 * I], Y->M->centroid[1] + Y->off[3 * I + 1],
                      Y->M->centroid[2] + Y->off[3 * I + 2]};
      double B[3];
      dipole_B(rJ, rI, Y->mom + 3 * I, B);
      for (int c = 0; c < 3; c++) Y->Bdip[3 * J + c] += B[c];
    }
  }
}

/* dy/dt for the whole system; Bth (may be NULL) is an extra per-node field [R][3][n]. */
static void sys_rhs(or_system *Y, double t, const double *y, const double *Bth, double *dy) {
  int n = Y->M->n;
  sys_dipoles(Y, y);
  for (int r = 0; r < Y->R; r++) {
    const double *m = y + (size_t)r * 3 * n;
    field_terms(Y->M, Y->S, &Y->mat[r], &Y->fld[r], Y->off + 3 * r, t, m, Y->Bdip + 3 * r,
                Y->Bbuf, NULL, NULL, &Y->W);
    if (Bth) for (int i = 0; i < 3 * n; i++) Y->Bbuf[i] += Bth[(size_t)r * 3 * n + i];
    llg_rhs(n, Y->mat[r].alpha, Y->relax ? 0.0 : 1.0, m, Y->Bbuf, dy + (size_t)r * 3 * n);
  }
}

/* Total energy of instance r (J), dipole term split half/half between partners. */
static double sys_energy(or_system *Y, double t, const double *y, int r) {
  int n = Y->M->n;
  double E[5];
  sys_dipoles(Y, y);
  field_terms(Y->M, Y->S, &Y->mat[r], &Y->fld[r], Y->off + 3 * r, t, y + (size_t)r * 3 * n, NULL,
              Y->Bbuf, NULL, E, &Y->W);
  double mu[3];
  instance_moment(Y->M, &Y->mat[r], y + (size_t)r * 3 * n, mu);
  double Edip = -0.5 * (mu[0] * Y->Bdip[3 * r] + mu[1] * Y->Bdip[3 * r + 1] + mu[2] * Y->Bdip[3 * r + 2]);
  return E[0] + E[1] + E[2] + E[3] + E[4] + Edip;
}

/* Observables: volume-weighted layer means of m_z and the moment-weighted mean of m. */
static void observe(const or_mesh *M, const or_material *mat, const double *m, double *obs) {
  int n = M->n;
  double ms = 0, mh = 0, vs = 0, vh = 0, w = 0, a[3] = {0, 0, 0};
  for (int i = 0; i < n; i++) {
    int L = M->layer[i] ? 1 : 0;
    double wi = mat->Ms[L] * M->V[i];
    if (L) { mh += M->V[i] * m[2 * n + i]; vh += M->V[i]; }
    else { ms += M->V[i] * m[2 * n + i]; vs += M->V[i]; }
    w += wi; a[0] += wi * m[i]; a[1] += wi * m[n + i]; a[2] += wi * m[2 * n + i];
  }
  obs[0] = a[0] / w; obs[1] = a[1] / w; obs[2] = a[2] / w;
  obs[3] = vs > 0 ? ms / vs : 0.0;
  obs[4] = vh > 0 ? mh / vh : 0.0;
}

typedef struct {
  double prev_t, prev_v;
  int crossed;
  double t_sw;
} or_cross;

static void cross_update(or_cross *C, double t, double v) {
  if (!C->crossed && v <= 0.0) {
    C->crossed = 1;
    if (C->prev_v <= 0.0 || t == C->prev_t) C->t_sw = t;
    else C->t_sw = C->prev_t + (t - C->prev_t) * C->prev_v / (C->prev_v - v);
  }
  C->prev_t = t; C->prev_v = v;
}

static void save_traj(or_system *Y, const double *y, double t, double dt, double err, double *traj,
                      int64_t cap, int64_t *ntraj) {
  int n = Y->M->n;
  for (int r = 0; r < Y->R; r++) {
    if (!traj || ntraj[r] >= cap) continue;
    double obs[5], B[3];
    observe(Y->M, &Y->mat[r], y + (size_t)r * 3 * n, obs);
    applied_B(&Y->fld[r], t, Y->M->centroid[0] + Y->off[3 * r], Y->M->centroid[1] + Y->off[3 * r + 1],
              Y->M->centroid[2] + Y->off[3 * r + 2], B);
    double *s = traj + ((size_t)r * cap + ntraj[r]) * 9;
    s[0] = t; s[1] = obs[0]; s[2] = obs[1]; s[3] = obs[2]; s[4] = obs[3]; s[5] = obs[4];
    s[6] = sqrt(B[0] * B[0] + B[1] * B[1] + B[2] * B[2]); s[7] = dt; s[8] = err;
    ntraj[r]++;
  }
}

/* Dormand-Prince 5(4) coefficients (Dormand & Prince 1980), written as exact fractions. */
static const double DP_C[7] = {0.0, 1.0 / 5, 3.0 / 10, 4.0 / 5, 8.0 / 9, 1.0, 1.0};
static const double DP_A[7][6] = {
    {0, 0, 0, 0, 0, 0},
    {1.0 / 5, 0, 0, 0, 0, 0},
    {3.0 / 40, 9.0 / 40, 0, 0, 0, 0},
    {44.0 / 45, -56.0 / 15, 32.0 / 9, 0, 0, 0},
    {19372.0 / 6561, -25360.0 / 2187, 64448.0 / 6561, -212.0 / 729, 0, 0},
    {9017.0 / 3168, -355.0 / 33, 46732.0 / 5247, 49.0 / 176, -5103.0 / 18656, 0},
    {35.0 / 384, 0, 500.0 / 1113, 125.0 / 192, -2187.0 / 6784, 11.0 / 84}};
/* error weights e = b - bhat */
static const double DP_E[7] = {71.0 / 57600, 0, -71.0 / 16695, 71.0 / 1920, -17253.0 / 339200,
                               22.0 / 525, -1.0 / 40};

void or_dp5_tableau(double *c, double *a, double *e) {
  memcpy(c, DP_C, sizeof(DP_C));
  memcpy(a, DP_A, sizeof(DP_A));
  memcpy(e, DP_E, sizeof(DP_E));
}

static int all_finite(const double *y, size_t len) {
  for (size_t i = 0; i < len; i++) if (!isfinite(y[i])) return 0;
  return 1;
}

static void finalize_results(or_system *Y, const double *y, double t, or_cross *cr, or_result *res) {
  int n = Y->M->n;
  for (int r = 0; r < Y->R; r++) {
    double obs[5];
    observe(Y->M, &Y->mat[r], y + (size_t)r * 3 * n, obs);
    res[r].mz_soft = obs[3]; res[r].mz_hard = obs[4];
    res[r].switched = obs[4] < 0.0;
    res[r].t_reached = t;
    res[r].t_sw = cr[r].crossed ? cr[r].t_sw : NAN;
    if (cr[r].crossed) {
      double B[3];
      applied_B(&Y->fld[r], cr[r].t_sw, Y->M->centroid[0] + Y->off[3 * r], Y->M->centroid[1] + Y->off[3 * r + 1],
                Y->M->centroid[2] + Y->off[3 * r + 2], B);
      res[r].B_sw = sqrt(B[0] * B[0] + B[1] * B[1] + B[2] * B[2]);
    } else {
      res[r].B_sw = NAN;
    }
    res[r].energy = all_finite(y + (size_t)r * 3 * n, 3 * (size_t)n) ? sys_energy(Y, t, y, r) : NAN;
  }
}

static void renormalize(int n, int R, double *y, double *maxdev) {
  for (int r = 0; r < R; r++) {
    double *m = y + (size_t)r * 3 * n;
    for (int i = 0; i < n; i++) {
      double l = sqrt(m[i] * m[i] + m[n + i] * m[n + i] + m[2 * n + i] * m[2 * n + i]);
      double d = fabs(1.0 - l);
      if (d > *maxdev) *maxdev = d;
      m[i] /= l; m[n + i] /= l; m[2 * n + i] /= l;
    }
  }
}

/* Dormand-Prince 5(4), FSAL.  Adaptive (error-controlled) or fixed step.  The error norm is the
 * RMS over every component of the system of e / (atol + rtol max(|y_n|, |y_n+1|)); a step is
 * accepted when the norm is <= 1 and the next step is dt * clamp(0.9 err^-1/5, 0.2, 5) with
 * growth capped at 1 on the step after a rejection.  |m| is restored after every accepted step. */
static void run_dp5(or_system *Y, const or_opts *o, double *y, or_result *res, double *traj,
                    int64_t cap, int64_t *ntraj) {
  int n = Y->M->n, R = Y->R;
  size_t len = (size_t)R * 3 * n;
  double *k[7], *ys = malloc(sizeof(double) * len), *y5 = malloc(sizeof(double) * len);
  for (int s = 0; s < 7; s++) k[s] = malloc(sizeof(double) * len);
  int fixed = o->integrator == OR_DP5_FIXED;
  double t = 0.0, dt = fixed ? o->dt_fixed : o->dt0, facmax = 5.0, maxdev = 0.0;
  double dtmin_used = INFINITY, dtmax_used = 0.0, err = 0.0;
  int64_t nacc = 0, nrej = 0, istep = 0;
  int status = OR_OK;
  or_cross *cr = calloc(R, sizeof(or_cross));
  for (int r = 0; r < R; r++) {
    double obs[5];
    observe(Y->M, &Y->mat[r], y + (size_t)r * 3 * n, obs);
    cr[r].prev_t = 0.0; cr[r].prev_v = obs[4];
    if (obs[4] <= 0.0) { cr[r].crossed = 1; cr[r].t_sw = 0.0; }
  }
  int64_t nfix = fixed ? (int64_t)ceil(o->t_end / o->dt_fixed - 1e-9) : 0;
  save_traj(Y, y, 0.0, 0.0, 0.0, traj, cap, ntraj);
  if (!all_finite(y, len)) status = OR_ENONFINITE;
  else sys_rhs(Y, t, y, NULL, k[0]);
  while (status == OR_OK) {
    double h;
    int last = 0;
    if (fixed) {
      if (istep >= nfix) break;
      t = istep * o->dt_fixed;
      double t1 = (istep + 1) * o->dt_fixed;
      if (t1 >= o->t_end || istep + 1 == nfix) { t1 = o->t_end; last = 1; }
      h = t1 - t;
    } else {
      if (t >= o->t_end) break;
      h = dt;
      if (t + h >= o->t_end) { h = o->t_end - t; last = 1; }
    }
    for (int s = 1; s < 7; s++) {
      for (size_t i = 0; i < len; i++) {
        double acc = 0.0;
        for (int j = 0; j < s; j++) acc += DP_A[s][j] * k[j][i];
        ys[i] = y[i] + h * acc;
      }
      sys_rhs(Y, t + DP_C[s] * h, ys, NULL, k[s]);
    }
    memcpy(y5, ys, sizeof(double) * len); /* stage 7 input is the 5th-order solution */
    double sum = 0.0;
    for (size_t i = 0; i < len; i++) {
      double e = 0.0;
      for (int j = 0; j < 7; j++) e += DP_E[j] * k[j][i];
      e *= h;
      double sc = o->atol + o->rtol * fmax(fabs(y[i]), fabs(y5[i]));
      sum += (e / sc) * (e / sc);
    }
    err = sqrt(sum / (double)len);
    if (!isfinite(err) || !all_finite(y5, len)) { status = OR_ENONFINITE; break; }
    if (fixed || err <= 1.0) {
      memcpy(y, y5, sizeof(double) * len);
      renormalize(n, R, y, &maxdev);
      double *tmp = k[0]; k[0] = k[6]; k[6] = tmp;   /* FSAL */
      t = last ? o->t_end : t + h;
      nacc++; istep++;
      if (h < dtmin_used) dtmin_used = h;
      if (h > dtmax_used) dtmax_used = h;
      for (int r = 0; r < R; r++) {
        double obs[5];
        observe(Y->M, &Y->mat[r], y + (size_t)r * 3 * n, obs);
        cross_update(&cr[r], t, obs[4]);
      }
      if ((o->save_every > 0 && nacc % o->save_every == 0) || last)
        save_traj(Y, y, t, h, err, traj, cap, ntraj);
      if (!fixed) {
        double fac = err == 0.0 ? facmax : fmin(facmax, fmax(0.2, 0.9 * pow(err, -0.2)));
        dt = h * fac;
        facmax = 5.0;
      }
      if (last) break;
    } else {
      nrej++;
      dt = h * fmax(0.2, 0.9 * pow(err, -0.2));
      facmax = 1.0;
    }
    if (!fixed && dt < o->dt_min) { status = OR_ESTEPUNDERFLOW; break; }
    if (o->max_steps > 0 && nacc + nrej >= o->max_steps) { status = OR_EMAXSTEPS; break; }
  }
  finalize_results(Y, y, t, cr, res);
  for (int r = 0; r < R; r++) {
    res[r].status = status;
    res[r].n_accept = nacc; res[r].n_reject = nrej;
    res[r].dt_min_used = nacc ? dtmin_used : 0.0;
    res[r].dt_max_used = dtmax_used;
    res[r].max_norm_dev = maxdev;
  }
  for (int s = 0; s < 7; s++) free(k[s]);
  free(ys); free(y5); free(cr);
}

/* Stochastic Heun (Stratonovich) with a Langevin thermal field.  Per step the field on node i
 * is B_th = sqrt(2 alpha kB T / (gamma w_i dt)) xi, xi ~ N(0,1)^3 drawn from Philox with
 * key = the instance seed and counter = (step, node); the same xi serves predictor and corrector. */
static void run_heun(or_system *Y, const or_opts *o, const uint64_t *seeds, double *y,
                     or_result *res, double *traj, int64_t cap, int64_t *ntraj) {
  int n = Y->M->n, R = Y->R;
  size_t len = (size_t)R * 3 * n;
  double *k1 = malloc(sizeof(double) * len), *k2 = malloc(sizeof(double) * len);
  double *yp = malloc(sizeof(double) * len), *Bth = malloc(sizeof(double) * len);
  double dt = o->dt_fixed, maxdev = 0.0, t = 0.0;
  int64_t nsteps = (int64_t)ceil(o->t_end / dt - 1e-9), nacc = 0;
  int status = OR_OK;
  or_cross *cr = calloc(R, sizeof(or_cross));
  for (int r = 0; r < R; r++) {
    double obs[5];
    observe(Y->M, &Y->mat[r], y + (size_t)r * 3 * n, obs);
    cr[r].prev_t = 0.0; cr[r].prev_v = obs[4];
    if (obs[4] <= 0.0) { cr[r].crossed = 1; cr[r].t_sw = 0.0; }
  }
  save_traj(Y, y, 0.0, 0.0, 0.0, traj, cap, ntraj);
  for (int64_t st = 0; st < nsteps && status == OR_OK; st++) {
    t = st * dt;
    double t1 = (st + 1 == nsteps) ? o->t_end : (st + 1) * dt;
    double h = t1 - t;
    for (int r = 0; r < R; r++) {
      uint32_t key[2] = {(uint32_t)seeds[r], (uint32_t)(seeds[r] >> 32)};
      const or_material *mat = &Y->mat[r];
      for (int i = 0; i < n; i++) {
        double g[3];
        or_gauss3(key, (uint64_t)st, (uint32_t)i, g);
        double w = mat->Ms[Y->M->layer[i] ? 1 : 0] * Y->M->V[i];
        double sig = o->temperature > 0.0 ? sqrt(2.0 * mat->alpha * OR_KB * o->temperature / (OR_GAMMA * w * h)) : 0.0;
        for (int c = 0; c < 3; c++) Bth[(size_t)r * 3 * n + c * n + i] = sig * g[c];
      }
    }
    sys_rhs(Y, t, y, Bth, k1);
    for (size_t i = 0; i < len; i++) yp[i] = y[i] + h * k1[i];
    sys_rhs(Y, t1, yp, Bth, k2);
    for (size_t i = 0; i < len; i++) y[i] = y[i] + 0.5 * h * (k1[i] + k2[i]);
    if (!all_finite(y, len)) { status = OR_ENONFINITE; break; }
    renormalize(n, R, y, &maxdev);
    t = t1;
    nacc++;
    for (int r = 0; r < R; r++) {
      double obs[5];
      observe(Y->M, &Y->mat[r], y + (size_t)r * 3 * n, obs);
      cross_update(&cr[r], t, obs[4]);
    }
    if ((o->save_every > 0 && nacc % o->save_every == 0) || st + 1 == nsteps)
      save_traj(Y, y, t, h, 0.0, traj, cap, ntraj);
  }
  finalize_results(Y, y, t, cr, res);
  for (int r = 0; r < R; r++) {
    res[r].status = status; res[r].n_accept = nacc; res[r].n_reject = 0;
    res[r].dt_min_used = dt; res[r].dt_max_used = dt; res[r].max_norm_dev = maxdev;
  }
  free(k1); free(k2); free(yp); free(Bth); free(cr);
}

/* Runs R instances on one mesh.  coupled != 0: one system with inter-island point dipoles and a
 * shared clock; otherwise R independent systems (OpenMP across them).
 * m (in/out): [R][3][n]; traj: [R][cap][9] = (t, <mx>, <my>, <mz>, <mz>_soft, <mz>_hard,
 * |B_app(centroid)|, dt, err); ntraj: [R]. */
int or_run(const or_mesh *M, const double *S, int R, const or_material *mats,
           const or_field *flds, const double *offsets, int coupled, const uint64_t *seeds,
           const or_opts *o, double *m, or_result *res, double *traj, int64_t cap,
           int64_t *ntraj) {
  if (!M || R <= 0 || !o) return OR_EINVAL;
  if (o->t_end < 0.0) return OR_EINVAL;
  if ((o->integrator == OR_DP5_FIXED || o->integrator == OR_HEUN) && !(o->dt_fixed > 0.0)) return OR_EINVAL;
  if (o->integrator == OR_DP45 && !(o->dt0 > 0.0)) return OR_EINVAL;
  int n = M->n;
  double zero3[3] = {0, 0, 0};
  for (int r = 0; r < R; r++) if (ntraj) ntraj[r] = 0;
  if (coupled && R > 1) {
    or_system Y = {M, S, R, mats, flds, offsets, 1};
    Y.relax = o->relax;
    sys_init(&Y);
    if (o->integrator == OR_HEUN) run_heun(&Y, o, seeds, m, res, traj, cap, ntraj);
    else run_dp5(&Y, o, m, res, traj, cap, ntraj);
    sys_free(&Y);
  } else {
#pragma omp parallel for schedule(dynamic, 1)
    for (int r = 0; r < R; r++) {
      or_system Y = {M, S, 1, mats + r, flds + r, offsets ? offsets + 3 * r : zero3, 0};
      Y.relax = o->relax;
      sys_init(&Y);
      double *trr = traj ? traj + (size_t)r * cap * 9 : NULL;
      int64_t *ntr = ntraj ? ntraj + r : NULL;
      if (o->integrator == OR_HEUN) run_heun(&Y, o, seeds + r, m + (size_t)r * 3 * n, res + r, trr, cap, ntr);
      else run_dp5(&Y, o, m + (size_t)r * 3 * n, res + r, trr, cap, ntr);
      sys_free(&Y);
    }
  }
  return OR_OK;
}

int or_num_threads(void) {
#ifdef _OPENMP
  return omp_get_max_threads();
#else
  return 1;
#endif
}
