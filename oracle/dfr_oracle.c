/*
 * dfr_oracle.c -- plain FP64 CPU oracle for the direct-flux-reconstruction (DFR)
 * right-hand side of the covariant shallow-water equations on the rotated
 * cubed sphere, and for its complex-step Jacobian-vector product.
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the reference the GPU library is
 * checked against.  Only the test-suite, the smoke check and the CPU-baseline
 * leg of the benchmark load it.  It shares no code with the library.
 *
 * Written from the paper (Gaudreault, Charron, Dallerit, Tokman, "High-order
 * numerical solutions to the shallow-water equations on the rotated
 * cubed-sphere grid", JCP 2022, arXiv 2101.05617):
 *   - equations of motion ........................ Sec. 2, Eqs. (1)-(2)
 *   - tensor-density form of the fluxes ........... App. D, Eq. (136)
 *   - 1-D DFR: GL points, Lagrange basis, extended
 *     flux polynomial and its derivative ......... Sec. 3.1, Eqs. (7)-(14)
 *   - tensor-product extension .................... Sec. 3.2
 *   - Riemann solver: Rusanov (named in Sec. 3.1); wave speeds from
 *     the flux-Jacobian eigenvalues ............... App. E, Eqs. (147)-(148)
 *   - Riemann solver: AUSM with double Froude-number
 *     splitting (the paper's choice) .............. App. D, Eqs. (136)-(143)
 *   - metric terms, Christoffel symbols ........... App. B, Eqs. (59)-(80)
 *   - rotated panel angles ....................... App. B, Eqs. (81)-(95)
 *   - panel-interface vector relations ........... App. C, Eqs. (100)-(135)
 *   - complex-step Jacobian-vector product ........ Sec. 4, Eq. (28)
 *   - relative vorticity, Coriolis parameter and the
 *     integrals of mass, total energy and potential
 *     enstrophy ................................. Sec. 5.4, Eqs. (43)-(46)
 *
 * Everything is written out element by element with no blocking or fusion.
 * Complex arithmetic is C99 `double complex` (the literal complex step).
 *
 * Readings where the paper is silent (same list as the design notes):
 *   R1  Riemann flux: Rusanov on the tensor densities q^mu; lambda is the max
 *       over the two sides of |u^n| + sqrt(h^nn g H).
 *   R2  Face states are extrapolated from the stored nodal (H, H u^1, H u^2)
 *       with the Lagrange basis of Eq. (7); the neighbour's contravariant
 *       momentum is converted to the receiving panel's basis with App. C, and
 *       the flux is formed in the receiving panel's coordinates.
 *   R3  Non-analytic operations under the complex step take the branch of
 *       the real evaluation at Re q: |z| := z if z_r >= 0 else -z ;
 *       max(a,b) := a if a_r >= b_r else b, where z_r, a_r, b_r are computed
 *       in real arithmetic from the real parts of the traced states (so an
 *       O(eps^2) real part of a complex quotient can never pick a branch).
 *   R4  Arctangents of Eqs. (81)-(95) are evaluated with atan2(num, den); the
 *       special case phi0 = alpha0 = 0 uses the stated pole values.
 *   R5  Orography derivative dh_B/dx^j: element-local collocation derivative
 *       of the nodal h_B (Lagrange basis on the GL points).
 *   R6  Panel connectivity and edge orientation are those of the unrotated
 *       layout implied by App. B/C (panels 0-3 equatorial west->east,
 *       4 north, 5 south); rotation does not change them.
 *   A1  AUSM split functions (App. D defers them to the original AUSM of
 *       Liou and Steffen, J. Comput. Phys. 107, 1993): the Froude-number
 *       split M^+- = +-(M +- 1)^2/4 for |M| <= 1, (M +- |M|)/2 otherwise,
 *       and the pressure weights P^+- / P = (M +- 1)^2 (2 -+ M)/4 for
 *       |M| <= 1, (1 +- sign M)/2 otherwise (the cubic form of that paper).
 *   A2  The "+" parts are taken on the low-coordinate side of the face and
 *       the "-" parts on the high side, each with its own Froude number
 *       M = u^n / a^n and gravity-wave speed a^n = sqrt(h^nn g_r H) (App. E).
 *   A3  Branches (|M| <= 1, sign M, max/min of Eqs. 142-143) follow the real
 *       evaluation, as in R3; when the split Froude number is exactly zero
 *       the advective part is taken from the low side.
 *   A4  The pressure component of the mass flux vanishes (h^{0n} = 0).
 *   V1  The derivatives of Eq. (43) are element-local collocation derivatives
 *       of the nodal covariant velocity g_jk u^k (as in R5); integrals over
 *       the sphere use the GL quadrature of each element with the area
 *       element sqrt(g) dx^1 dx^2.
 */
#include <complex.h>
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

typedef double complex cplx;

#define ORC_MAXNS 12
#define ORC_PI 3.14159265358979323846

enum { ORC_OK = 0, ORC_EINVAL = -1, ORC_ENOMEM = -2, ORC_ENONFINITE = -4, ORC_EDEPTH = -5 };

typedef struct orc_grid {
  int ne, ns;
  double a, omega, g;
  double lam[6], phi[6], alp[6];   /* panel angles, App. B */
  double xi[ORC_MAXNS], w[ORC_MAXNS];
  double lm[ORC_MAXNS], lp[ORC_MAXNS];          /* l_k(-1), l_k(+1), Eq. (8) */
  double Dt[ORC_MAXNS][ORC_MAXNS + 2];          /* l~'_n(xi_k), Eq. (13) */
  double Dgl[ORC_MAXNS][ORC_MAXNS];             /* l'_k(xi_m) on GL points (R5) */
  double *dhb;                                  /* NULL or 2*N: dh_B/dx^1, dh_B/dx^2 */
  int riemann;                                  /* 0: Rusanov, 1: AUSM */
} orc_grid;

/* ------------------------------------------------------------------------ */
/* Indexing: field-major, then panel, element row, element column, node row,  */
/* node column (x^1 fastest).                                                */
static inline int64_t orc_idx(const orc_grid *G, int f, int p, int ej, int ei, int nj, int ni) {
  int64_t ne = G->ne, ns = G->ns;
  return (((((int64_t)f * 6 + p) * ne + ej) * ne + ei) * ns + nj) * ns + ni;
}
int64_t orc_num_nodes(const orc_grid *G) { return 6LL * G->ne * G->ne * G->ns * G->ns; }

/* ------------------------------------------------------------------------ */
/* Gauss-Legendre points: roots of P_ns (Sec. 3.1), by Newton's method on the  */
/* three-term recurrence; weights 2/((1-x^2) P'_ns(x)^2).                    */
static void legendre(int n, double x, double *P, double *dP) {
  double p0 = 1.0, p1 = x;
  if (n == 0) { *P = 1.0; *dP = 0.0; return; }
  for (int k = 2; k <= n; ++k) {
    double p2 = ((2.0 * k - 1.0) * x * p1 - (k - 1.0) * p0) / k;
    p0 = p1; p1 = p2;
  }
  *P = p1;
  *dP = n * (x * p1 - p0) / (x * x - 1.0);
}

static void gauss_legendre(int n, double *x, double *w) {
  for (int k = 0; k < n; ++k) {
    /* k-th root in increasing order */
    double z = -cos(ORC_PI * (k + 0.75) / (n + 0.5));
    for (int it = 0; it < 100; ++it) {
      double P, dP;
      legendre(n, z, &P, &dP);
      double dz = P / dP;
      z -= dz;
      if (fabs(dz) < 1e-16) break;
    }
    double P, dP;
    legendre(n, z, &P, &dP);
    x[k] = z;
    w[k] = 2.0 / ((1.0 - z * z) * dP * dP);
  }
}

/* Lagrange basis on nodes t[0..n-1] evaluated at s (Eq. 8). */
static double lagrange(const double *t, int n, int k, double s) {
  double v = 1.0;
  for (int l = 0; l < n; ++l)
    if (l != k) v *= (s - t[l]) / (t[k] - t[l]);
  return v;
}

/* Derivative of the Lagrange basis polynomial n on nodes t, at s: Eq. (13). */
static double lagrange_deriv(const double *t, int npts, int n, double s) {
  double sum = 0.0;
  for (int i = 0; i < npts; ++i) {
    if (i == n) continue;
    double prod = 1.0 / (t[n] - t[i]);
    for (int m = 0; m < npts; ++m) {
      if (m == i || m == n) continue;
      prod *= (s - t[m]) / (t[n] - t[m]);
    }
    sum += prod;
  }
  return sum;
}

/* ------------------------------------------------------------------------ */
/* Panel angles (lambda_p, phi_p, alpha_p), Eqs. (81)-(95), reading R4.      */
void orc_panel_angles(double l0, double f0, double a0, double *lam, double *phi, double *alp) {
  double cl = cos(l0), sl = sin(l0), cf = cos(f0), sf = sin(f0), ca = cos(a0), sa = sin(a0);
  lam[0] = l0; phi[0] = f0; alp[0] = a0;
  lam[1] = atan2(cl * ca + sl * sf * sa, cl * sf * sa - sl * ca);   /* (81) */
  phi[1] = -asin(cf * sa);                                        /* (82) */
  alp[1] = atan2(sf, cf * ca);                                    /* (83) */
  lam[2] = l0 + ORC_PI;                                           /* (84) */
  phi[2] = -f0;                                                   /* (85) */
  alp[2] = -a0;                                                   /* (86) */
  lam[3] = -atan2(cl * ca + sl * sf * sa, sl * ca - cl * sf * sa);  /* (87) */
  phi[3] = asin(cf * sa);                                         /* (88) */
  alp[3] = -atan2(sf, cf * ca);                                   /* (89) */
  if (f0 == 0.0 && a0 == 0.0) {
    /* pole special case stated after Eq. (95) */
    lam[4] = 0.0; phi[4] = 0.5 * ORC_PI; alp[4] = -l0;
    lam[5] = 0.0; phi[5] = -0.5 * ORC_PI; alp[5] = l0;
  } else {
    lam[4] = atan2(cl * sa - sl * sf * ca, -cl * sf * ca - sl * sa);  /* (90) */
    phi[4] = asin(cf * ca);                                         /* (91) */
    alp[4] = atan2(cf * sa, -sf);                                   /* (92) */
    lam[5] = atan2(sl * sf * ca - cl * sa, cl * sf * ca + sl * sa);   /* (93) */
    phi[5] = -asin(cf * ca);                                        /* (94) */
    alp[5] = atan2(cf * sa, sf);                                    /* (95) */
  }
}

/* ------------------------------------------------------------------------ */
/* Coordinates.  Element edges are equiangular: x^i in [-pi/4, pi/4], ne      */
/* elements of width Delta = pi/(2 ne).  Node abscissa by the affine map Eq 5. */
static inline double orc_delta(const orc_grid *G) { return 0.5 * ORC_PI / G->ne; }
static inline double node_x(const orc_grid *G, int e, int k) {
  double D = orc_delta(G);
  double lo = -0.25 * ORC_PI + e * D;
  return lo + 0.5 * (1.0 + G->xi[k]) * D;
}
static inline double edge_x(const orc_grid *G, int e) { return -0.25 * ORC_PI + e * orc_delta(G); }

/* Metric, Eqs. (67)-(70). */
typedef struct { double sg, h11, h12, h22; } metric_t;
static metric_t metric_at(const orc_grid *G, double X, double Y) {
  metric_t m;
  double a2 = G->a * G->a;
  double d2 = 1.0 + X * X + Y * Y;
  double d = sqrt(d2);
  m.sg = a2 * (1.0 + X * X) * (1.0 + Y * Y) / (d2 * d);
  m.h11 = d2 / (a2 * (1.0 + X * X));
  m.h12 = X * Y * d2 / (a2 * (1.0 + X * X) * (1.0 + Y * Y));
  m.h22 = d2 / (a2 * (1.0 + Y * Y));
  return m;
}

/* Christoffel symbols.  c0[i][j] = Gamma^{i+1}_{0 (j+1)} (Eqs. 71-74);       */
/* cs[i][j][k] = Gamma^{i+1}_{(j+1)(k+1)} (Eqs. 75-80).                       */
static void christoffel_at(const orc_grid *G, int p, double X, double Y, double c0[2][2], double cs[2][2][2]) {
  double d2 = 1.0 + X * X + Y * Y;
  double fac = sin(G->phi[p]) - X * cos(G->phi[p]) * sin(G->alp[p]) + Y * cos(G->phi[p]) * cos(G->alp[p]);
  double Om = G->omega;
  c0[0][0] = Om * X * Y / d2 * fac;                 /* (71) */
  c0[0][1] = -Om * (1.0 + Y * Y) / d2 * fac;        /* (72) */
  c0[1][0] = Om * (1.0 + X * X) / d2 * fac;         /* (73) */
  c0[1][1] = -Om * X * Y / d2 * fac;                /* (74) */
  cs[0][0][0] = 2.0 * X * Y * Y / d2;               /* (75) */
  cs[0][0][1] = cs[0][1][0] = -Y * (1.0 + Y * Y) / d2; /* (76) */
  cs[0][1][1] = 0.0;                                /* (77) */
  cs[1][0][0] = 0.0;                                /* (78) */
  cs[1][0][1] = cs[1][1][0] = -X * (1.0 + X * X) / d2; /* (79) */
  cs[1][1][1] = 2.0 * X * X * Y / d2;               /* (80) */
}

/* ------------------------------------------------------------------------ */
/* Panel connectivity (reading R6).  Edges: 0=W (x^1 low), 1=E (x^1 high),    */
/* 2=S (x^2 low), 3=N (x^2 high).  rev=1 when the along-edge coordinates run */
/* in opposite directions on the two panels.                                 */
enum { EW = 0, EE = 1, ES = 2, EN = 3 };
typedef struct { int q, edge, rev; } nbr_t;
static const nbr_t CONN[6][4] = {
  /* panel 0 */ { {3, EE, 0}, {1, EW, 0}, {5, EN, 0}, {4, ES, 0} },
  /* panel 1 */ { {0, EE, 0}, {2, EW, 0}, {5, EE, 1}, {4, EE, 0} },
  /* panel 2 */ { {1, EE, 0}, {3, EW, 0}, {5, ES, 1}, {4, EN, 1} },
  /* panel 3 */ { {2, EE, 0}, {0, EW, 0}, {5, EW, 0}, {4, EW, 1} },
  /* panel 4 */ { {3, EN, 1}, {1, EN, 0}, {0, EN, 0}, {2, EN, 1} },
  /* panel 5 */ { {3, ES, 0}, {1, ES, 1}, {2, ES, 1}, {0, ES, 0} },
};

/* App. C contravariant relations.  Returns the 2x2 matrix M with            */
/* A_(dst) = M A_(src) for the interface between panels dst and src, where   */
/* t = 2s/(1+s^2) and s is the along-edge tangent named in the paper (Y for   */
/* the equatorial pairs; X "defined on panel q" for the polar pairs).        */
static void appc_matrix(int dst, int src, double s, double M[2][2]) {
  double t = 2.0 * s / (1.0 + s * s);
  double F[2][2];   /* forward relation as printed, and which way it maps */
  int fwd_dst, fwd_src;
  /* equatorial: (p,q) = (0,1),(1,2),(2,3),(3,0): A_(p) from A_(q), Eqs. (100)-(101) */
  if (dst < 4 && src < 4) {
    fwd_dst = ((src + 3) % 4 == dst) ? dst : src;
    fwd_src = (fwd_dst == dst) ? src : dst;
    F[0][0] = 1.0; F[0][1] = 0.0;
    F[1][0] = t;   F[1][1] = 1.0;
  } else {
    int pole = (dst >= 4) ? dst : src;
    int q = (dst >= 4) ? src : dst;
    fwd_dst = pole; fwd_src = q;
    if (pole == 4) {
      switch (q) {
        case 0: F[0][0] = 1.0;  F[0][1] = -t;  F[1][0] = 0.0;  F[1][1] = 1.0;  break; /* (104)-(105) */
        case 1: F[0][0] = 0.0;  F[0][1] = -1.0; F[1][0] = 1.0;  F[1][1] = -t;  break; /* (108)-(109) */
        case 2: F[0][0] = -1.0; F[0][1] = t;   F[1][0] = 0.0;  F[1][1] = -1.0; break; /* (112)-(113) */
        default: F[0][0] = 0.0; F[0][1] = 1.0; F[1][0] = -1.0; F[1][1] = t;   break; /* (116)-(117) */
      }
    } else {
      switch (q) {
        case 0: F[0][0] = 1.0;  F[0][1] = t;   F[1][0] = 0.0;  F[1][1] = 1.0;  break; /* (120)-(121) */
        case 1: F[0][0] = 0.0;  F[0][1] = 1.0; F[1][0] = -1.0; F[1][1] = -t;  break; /* (124)-(125) */
        case 2: F[0][0] = -1.0; F[0][1] = -t;  F[1][0] = 0.0;  F[1][1] = -1.0; break; /* (128)-(129) */
        default: F[0][0] = 0.0; F[0][1] = -1.0; F[1][0] = 1.0; F[1][1] = t;   break; /* (132)-(133) */
      }
    }
  }
  if (fwd_dst == dst && fwd_src == src) {
    memcpy(M, F, sizeof(F));
  } else {
    /* inverse of the printed relation */
    double det = F[0][0] * F[1][1] - F[0][1] * F[1][0];
    M[0][0] = F[1][1] / det;  M[0][1] = -F[0][1] / det;
    M[1][0] = -F[1][0] / det; M[1][1] = F[0][0] / det;
  }
}

/* ------------------------------------------------------------------------ */
/* Grid construction.                                                        */
orc_grid *orc_create(int ne, int ns, double a, double omega, double g,
                     double lam0, double phi0, double alp0, const double *hB) {
  if (ne < 1 || ns < 1 || ns > ORC_MAXNS) return NULL;
  orc_grid *G = (orc_grid *)calloc(1, sizeof(orc_grid));
  if (!G) return NULL;
  G->ne = ne; G->ns = ns; G->a = a; G->omega = omega; G->g = g;
  orc_panel_angles(lam0, phi0, alp0, G->lam, G->phi, G->alp);
  gauss_legendre(ns, G->xi, G->w);
  for (int k = 0; k < ns; ++k) {
    G->lm[k] = lagrange(G->xi, ns, k, -1.0);
    G->lp[k] = lagrange(G->xi, ns, k, 1.0);
  }
  /* extended points {-1, xi_1..xi_ns, +1} (Sec. 3.1, after Eq. 10) */
  double ext[ORC_MAXNS + 2];
  ext[0] = -1.0;
  for (int k = 0; k < ns; ++k) ext[k + 1] = G->xi[k];
  ext[ns + 1] = 1.0;
  for (int k = 0; k < ns; ++k)
    for (int n = 0; n < ns + 2; ++n) G->Dt[k][n] = lagrange_deriv(ext, ns + 2, n, G->xi[k]);
  for (int m = 0; m < ns; ++m)
    for (int k = 0; k < ns; ++k) G->Dgl[m][k] = lagrange_deriv(G->xi, ns, k, G->xi[m]);
  G->dhb = NULL;
  if (hB) {
    int64_t N = orc_num_nodes(G);
    G->dhb = (double *)malloc(sizeof(double) * 2 * N);
    if (!G->dhb) { free(G); return NULL; }
    double s = 2.0 / orc_delta(G);
    for (int p = 0; p < 6; ++p)
      for (int ej = 0; ej < ne; ++ej)
        for (int ei = 0; ei < ne; ++ei)
          for (int nj = 0; nj < ns; ++nj)
            for (int ni = 0; ni < ns; ++ni) {
              double d1 = 0.0, d2 = 0.0;
              for (int k = 0; k < ns; ++k) {
                d1 += G->Dgl[ni][k] * hB[orc_idx(G, 0, p, ej, ei, nj, k)];
                d2 += G->Dgl[nj][k] * hB[orc_idx(G, 0, p, ej, ei, k, ni)];
              }
              int64_t i0 = orc_idx(G, 0, p, ej, ei, nj, ni);
              G->dhb[i0] = s * d1;
              G->dhb[N + i0] = s * d2;
            }
  }
  return G;
}

void orc_destroy(orc_grid *G) {
  if (!G) return;
  free(G->dhb);
  free(G);
}

/* Accessors used by the tests. */
void orc_get_operators(const orc_grid *G, double *xi, double *w, double *lm, double *lp, double *Dt) {
  int ns = G->ns;
  for (int k = 0; k < ns; ++k) { xi[k] = G->xi[k]; w[k] = G->w[k]; lm[k] = G->lm[k]; lp[k] = G->lp[k]; }
  for (int k = 0; k < ns; ++k)
    for (int n = 0; n < ns + 2; ++n) Dt[k * (ns + 2) + n] = G->Dt[k][n];
}
void orc_get_panels(const orc_grid *G, double *out18) {
  for (int p = 0; p < 6; ++p) { out18[3 * p] = G->lam[p]; out18[3 * p + 1] = G->phi[p]; out18[3 * p + 2] = G->alp[p]; }
}
void orc_appc_matrix(int dst, int src, double s, double *M4) {
  double M[2][2];
  appc_matrix(dst, src, s, M);
  M4[0] = M[0][0]; M4[1] = M[0][1]; M4[2] = M[1][0]; M4[3] = M[1][1];
}
void orc_connectivity(int p, int edge, int *q, int *qedge, int *rev) {
  *q = CONN[p][edge].q; *qedge = CONN[p][edge].edge; *rev = CONN[p][edge].rev;
}

/* Panel frame: centre e_c, and e_1, e_2 obtained by turning east/north by   */
/* alpha_p; this is the frame for which Eqs. (59)-(60) read X = P.e1/P.ec,   */
/* Y = P.e2/P.ec.  The inverse map is P = (e_c + X e_1 + Y e_2)/delta.       */
static void panel_frame(const orc_grid *G, int p, double ec[3], double e1[3], double e2[3]) {
  double lp = G->lam[p], fp = G->phi[p], ap = G->alp[p];
  double E[3] = { -sin(lp), cos(lp), 0.0 };
  double Nn[3] = { -sin(fp) * cos(lp), -sin(fp) * sin(lp), cos(fp) };
  ec[0] = cos(fp) * cos(lp); ec[1] = cos(fp) * sin(lp); ec[2] = sin(fp);
  for (int i = 0; i < 3; ++i) {
    e1[i] = cos(ap) * E[i] - sin(ap) * Nn[i];
    e2[i] = sin(ap) * E[i] + cos(ap) * Nn[i];
  }
}

/* Unit position P and the coordinate basis dP/dx^1, dP/dx^2 at every node  */
/* (unit sphere).  Used to build synthetic inputs and by geometry pins.      */
void orc_node_frames(const orc_grid *G, double *P, double *B1, double *B2) {
  int ne = G->ne, ns = G->ns;
  for (int p = 0; p < 6; ++p) {
    double ec[3], e1[3], e2[3];
    panel_frame(G, p, ec, e1, e2);
    for (int ej = 0; ej < ne; ++ej)
      for (int ei = 0; ei < ne; ++ei)
        for (int nj = 0; nj < ns; ++nj)
          for (int ni = 0; ni < ns; ++ni) {
            double X = tan(node_x(G, ei, ni)), Y = tan(node_x(G, ej, nj));
            double d2 = 1.0 + X * X + Y * Y, d = sqrt(d2);
            int64_t n = orc_idx(G, 0, p, ej, ei, nj, ni);
            for (int c = 0; c < 3; ++c) {
              double r = ec[c] + X * e1[c] + Y * e2[c];
              P[3 * n + c] = r / d;
              /* dP/dX = e1/d - r X/d^3 ; dX/dx^1 = 1 + X^2 */
              B1[3 * n + c] = (1.0 + X * X) * (e1[c] / d - r * X / (d2 * d));
              B2[3 * n + c] = (1.0 + Y * Y) * (e2[c] / d - r * Y / (d2 * d));
            }
          }
  }
}

/* Geometry at every node: sqrt(g), h^11, h^12, h^22, Gamma^i_0j, Gamma^i_jk. */
void orc_node_metric(const orc_grid *G, double *out /* N x 16 */) {
  int ne = G->ne, ns = G->ns;
  for (int p = 0; p < 6; ++p)
    for (int ej = 0; ej < ne; ++ej)
      for (int ei = 0; ei < ne; ++ei)
        for (int nj = 0; nj < ns; ++nj)
          for (int ni = 0; ni < ns; ++ni) {
            double X = tan(node_x(G, ei, ni)), Y = tan(node_x(G, ej, nj));
            metric_t m = metric_at(G, X, Y);
            double c0[2][2], cs[2][2][2];
            christoffel_at(G, p, X, Y, c0, cs);
            double *o = out + 16 * orc_idx(G, 0, p, ej, ei, nj, ni);
            o[0] = m.sg; o[1] = m.h11; o[2] = m.h12; o[3] = m.h22;
            o[4] = c0[0][0]; o[5] = c0[0][1]; o[6] = c0[1][0]; o[7] = c0[1][1];
            o[8] = cs[0][0][0]; o[9] = cs[0][0][1]; o[10] = cs[0][1][1];
            o[11] = cs[1][0][0]; o[12] = cs[1][0][1]; o[13] = cs[1][1][1];
            o[14] = X; o[15] = Y;
          }
}

/* ------------------------------------------------------------------------ */
/* Complex helpers for the non-analytic operations (reading R3).            */
/* zr, ar, br: the same quantities evaluated in real arithmetic at Re q.      */
static inline cplx cs_abs(cplx z, double zr) { return zr >= 0.0 ? z : -z; }
static inline cplx cs_max(cplx a, cplx b, double ar, double br) { return ar >= br ? a : b; }

/* State trace at one face point of element (p,ej,ei): extrapolation of the  */
/* three stored fields along the line normal to `edge`, Eq. (7) at xi=+-1.    */
static void face_trace(const orc_grid *G, const cplx *Q, int p, int ej, int ei, int edge, int t, cplx out[3]) {
  int ns = G->ns;
  for (int f = 0; f < 3; ++f) {
    cplx s = 0.0;
    for (int k = 0; k < ns; ++k) {
      int64_t id;
      double wgt;
      switch (edge) {
        case EW: id = orc_idx(G, f, p, ej, ei, t, k); wgt = G->lm[k]; break;
        case EE: id = orc_idx(G, f, p, ej, ei, t, k); wgt = G->lp[k]; break;
        case ES: id = orc_idx(G, f, p, ej, ei, k, t); wgt = G->lm[k]; break;
        default: id = orc_idx(G, f, p, ej, ei, k, t); wgt = G->lp[k]; break;
      }
      s += wgt * Q[id];
    }
    out[f] = s;
  }
}

/* Normal flux sqrt(g) T^{mu n} from tensor densities q (Eq. 136).           */
static void normal_flux(const orc_grid *G, const cplx q[3], double sg, const double h[2][2], int n, cplx F[3]) {
  F[0] = q[1 + n];
  for (int i = 0; i < 2; ++i)
    F[1 + i] = q[1 + i] * q[1 + n] / q[0] + G->g * h[i][n] * q[0] * q[0] / (2.0 * sg);
}

/* Rusanov common flux at one face point (reading R1).  qL, qR: densities on */
/* the low and high sides (in the receiving panel's basis).                  */
static void rusanov(const orc_grid *G, const cplx qL[3], const cplx qR[3], double sg, const double h[2][2], int n, cplx Fs[3]) {
  cplx FL[3], FR[3];
  normal_flux(G, qL, sg, h, n, FL);
  normal_flux(G, qR, sg, h, n, FR);
  /* wave speed |u^n| + sqrt(h^nn g H), Eqs. (147)-(148) */
  cplx uL = qL[1 + n] / qL[0], uR = qR[1 + n] / qR[0];
  cplx HL = qL[0] / sg, HR = qR[0] / sg;
  /* branches of |.| and max(.,.) are those of the real evaluation at Re q
     (reading R3): real quotients, so that no O(eps^2) real part can decide */
  double uLr = creal(qL[1 + n]) / creal(qL[0]), uRr = creal(qR[1 + n]) / creal(qR[0]);
  double cLr = fabs(uLr) + sqrt(h[n][n] * G->g * (creal(qL[0]) / sg));
  double cRr = fabs(uRr) + sqrt(h[n][n] * G->g * (creal(qR[0]) / sg));
  cplx cL = cs_abs(uL, uLr) + csqrt(h[n][n] * G->g * HL);
  cplx cR = cs_abs(uR, uRr) + csqrt(h[n][n] * G->g * HR);
  cplx lam = cs_max(cL, cR, cLr, cRr);
  for (int m = 0; m < 3; ++m) Fs[m] = 0.5 * (FL[m] + FR[m]) - 0.5 * lam * (qR[m] - qL[m]);
}

/* AUSM split functions of the Froude number and of the pressure weight      */
/* (reading A1), on a real M.                                                */
void orc_ausm_split(double M, double *Mp, double *Mm, double *Pp, double *Pm) {
  if (fabs(M) <= 1.0) {
    *Mp = 0.25 * (M + 1.0) * (M + 1.0);
    *Mm = -0.25 * (M - 1.0) * (M - 1.0);
    *Pp = 0.25 * (M + 1.0) * (M + 1.0) * (2.0 - M);
    *Pm = 0.25 * (M - 1.0) * (M - 1.0) * (2.0 + M);
  } else {
    *Mp = 0.5 * (M + fabs(M));
    *Mm = 0.5 * (M - fabs(M));
    *Pp = M > 0.0 ? 1.0 : 0.0;
    *Pm = M > 0.0 ? 0.0 : 1.0;
  }
}

/* The same split on a complex M whose real part Mr (computed in real         */
/* arithmetic, reading A3) picks the branch: "+" parts (low side) or "-".      */
static void ausm_split_c(cplx M, double Mr, int plus, cplx *Ms, cplx *Ps) {
  if (fabs(Mr) <= 1.0) {
    if (plus) { *Ms = 0.25 * (M + 1.0) * (M + 1.0); *Ps = 0.25 * (M + 1.0) * (M + 1.0) * (2.0 - M); }
    else { *Ms = -0.25 * (M - 1.0) * (M - 1.0); *Ps = 0.25 * (M - 1.0) * (M - 1.0) * (2.0 + M); }
  } else if (Mr > 0.0) {
    *Ms = plus ? M : 0.0;
    *Ps = plus ? 1.0 : 0.0;
  } else {
    *Ms = plus ? 0.0 : M;
    *Ps = plus ? 0.0 : 1.0;
  }
}

/* AUSM common flux with double Froude-number splitting, Eqs. (137)-(143):   */
/* sqrt(g) T^{mu n} = M^n A^{mu n} + P^{mu n}, A^{mu n} = q^mu a^n,            */
/* P^{mu n} = g_r h^{mu n} (q^0)^2 / (2 sqrt g).  qL: low side ("+"), qR:      */
/* high side ("-"), both in the receiving panel's basis.                      */
static void ausm(const orc_grid *G, const cplx qL[3], const cplx qR[3], double sg, const double h[2][2], int n, cplx Fs[3]) {
  cplx HL = qL[0] / sg, HR = qR[0] / sg;
  cplx aL = csqrt(h[n][n] * G->g * HL), aR = csqrt(h[n][n] * G->g * HR);   /* App. E */
  cplx ML = (qL[1 + n] / qL[0]) / aL, MR = (qR[1 + n] / qR[0]) / aR;
  double MLr = (creal(qL[1 + n]) / creal(qL[0])) / sqrt(h[n][n] * G->g * (creal(qL[0]) / sg));
  double MRr = (creal(qR[1 + n]) / creal(qR[0])) / sqrt(h[n][n] * G->g * (creal(qR[0]) / sg));
  cplx Mp, Mm, Pp, Pm;
  ausm_split_c(ML, MLr, 1, &Mp, &Pp);
  ausm_split_c(MR, MRr, 0, &Mm, &Pm);
  double sL[4], sR[4];                 /* real splits: M+, M-, P+, P- */
  orc_ausm_split(MLr, &sL[0], &sL[1], &sL[2], &sL[3]);
  orc_ausm_split(MRr, &sR[0], &sR[1], &sR[2], &sR[3]);
  cplx m = Mp + Mm;                    /* Eq. (138) on the two sides */
  double mr = sL[0] + sR[1];
  for (int mu = 0; mu < 3; ++mu) {
    cplx AL = qL[mu] * aL, AR = qR[mu] * aR;
    cplx PL = 0.0, PR = 0.0;
    if (mu > 0) {
      PL = G->g * h[mu - 1][n] * qL[0] * qL[0] / (2.0 * sg);
      PR = G->g * h[mu - 1][n] * qR[0] * qR[0] / (2.0 * sg);
    }
    /* Eqs. (140)-(143): max[0, m] A^+ + min[0, m] A^- + P^+ + P^- */
    cplx adv = mr >= 0.0 ? m * AL : m * AR;
    Fs[mu] = adv + Pp * PL + Pm * PR;
  }
}

/* Common flux of the grid's Riemann solver; qL on the low side.             */
static void common_flux(const orc_grid *G, const cplx qL[3], const cplx qR[3], double sg, const double h[2][2], int n, cplx Fs[3]) {
  if (G->riemann == 1) ausm(G, qL, qR, sg, h, n, Fs);
  else rusanov(G, qL, qR, sg, h, n, Fs);
}

/* Real common flux at one face point, for the tests: qL, qR tensor          */
/* densities, h4 = (h^11, h^12, h^21, h^22), n the normal direction.          */
void orc_common_flux(const orc_grid *G, const double *qL, const double *qR, double sg, const double *h4, int n, double *F) {
  cplx a[3], b[3], Fs[3];
  double h[2][2] = { { h4[0], h4[1] }, { h4[2], h4[3] } };
  for (int k = 0; k < 3; ++k) { a[k] = qL[k]; b[k] = qR[k]; }
  common_flux(G, a, b, sg, h, n, Fs);
  for (int k = 0; k < 3; ++k) F[k] = creal(Fs[k]);
}

void orc_set_riemann(orc_grid *G, int solver) { G->riemann = solver; }

/* Common flux on face `edge` of element (p,ej,ei) at face point t, in the    */
/* element's own coordinates.                                                */
static void face_flux(const orc_grid *G, const cplx *Q, int p, int ej, int ei, int edge, int t, cplx Fs[3]) {
  int ne = G->ne;
  /* own trace */
  cplx own[3];
  face_trace(G, Q, p, ej, ei, edge, t, own);
  /* neighbour element, its touching face, and the matching face point */
  int q = p, qej = ej, qei = ei, qedge, qt = t;
  int interior = 1;
  switch (edge) {
    case EW: if (ei > 0) { qei = ei - 1; qedge = EE; } else interior = 0; break;
    case EE: if (ei < ne - 1) { qei = ei + 1; qedge = EW; } else interior = 0; break;
    case ES: if (ej > 0) { qej = ej - 1; qedge = EN; } else interior = 0; break;
    default: if (ej < ne - 1) { qej = ej + 1; qedge = ES; } else interior = 0; break;
  }
  int along_e = (edge == EW || edge == EE) ? ej : ei;   /* element index along the edge */
  if (!interior) {
    nbr_t nb = CONN[p][edge];
    q = nb.q; qedge = nb.edge;
    int ae = nb.rev ? ne - 1 - along_e : along_e;
    qt = nb.rev ? G->ns - 1 - t : t;
    switch (qedge) {
      case EW: qei = 0; qej = ae; break;
      case EE: qei = ne - 1; qej = ae; break;
      case ES: qej = 0; qei = ae; break;
      default: qej = ne - 1; qei = ae; break;
    }
  }
  cplx nbv[3];
  face_trace(G, Q, q, qej, qei, qedge, qt, nbv);
  if (!interior) {
    /* App. C: convert the neighbour's contravariant momentum to this panel */
    double s;
    if (p < 4 && q < 4) {
      /* the along-edge tangent Y is common to both sides */
      s = tan(node_x(G, ej, t));
    } else if (p < 4) {
      /* X defined on the equatorial panel = own along-edge tangent */
      s = tan(node_x(G, ei, t));
    } else {
      /* X defined on the equatorial neighbour panel q (its N or S edge) */
      s = tan(node_x(G, qei, qt));
    }
    double M[2][2];
    appc_matrix(p, q, s, M);
    cplx m1 = M[0][0] * nbv[1] + M[0][1] * nbv[2];
    cplx m2 = M[1][0] * nbv[1] + M[1][1] * nbv[2];
    nbv[1] = m1; nbv[2] = m2;
  }
  /* face-point coordinates on the own panel */
  double X, Y;
  switch (edge) {
    case EW: X = tan(edge_x(G, ei)); Y = tan(node_x(G, ej, t)); break;
    case EE: X = tan(edge_x(G, ei + 1)); Y = tan(node_x(G, ej, t)); break;
    case ES: X = tan(node_x(G, ei, t)); Y = tan(edge_x(G, ej)); break;
    default: X = tan(node_x(G, ei, t)); Y = tan(edge_x(G, ej + 1)); break;
  }
  metric_t m = metric_at(G, X, Y);
  double h[2][2] = { { m.h11, m.h12 }, { m.h12, m.h22 } };
  cplx qo[3], qn[3];
  for (int f = 0; f < 3; ++f) { qo[f] = m.sg * own[f]; qn[f] = m.sg * nbv[f]; }
  int n = (edge == EW || edge == EE) ? 0 : 1;
  if (edge == EW || edge == ES) common_flux(G, qn, qo, m.sg, h, n, Fs);
  else common_flux(G, qo, qn, m.sg, h, n, Fs);
}

/* The right-hand side at the nodes of element (p, ej, ei).                 */
static void element_rhs(const orc_grid *G, const cplx *Q, cplx *dQ, int p, int ej, int ei) {
  int ns = G->ns;
  int64_t N = orc_num_nodes(G);
  double D = orc_delta(G);
  cplx F1[3 * ORC_MAXNS * ORC_MAXNS], F2[3 * ORC_MAXNS * ORC_MAXNS];
  cplx FW[3 * ORC_MAXNS], FE[3 * ORC_MAXNS], FS[3 * ORC_MAXNS], FN[3 * ORC_MAXNS];
  /* nodal fluxes sqrt(g) T^{mu j} (Eq. 136) */
  for (int nj = 0; nj < ns; ++nj)
    for (int ni = 0; ni < ns; ++ni) {
      double X = tan(node_x(G, ei, ni)), Y = tan(node_x(G, ej, nj));
      metric_t m = metric_at(G, X, Y);
      double h[2][2] = { { m.h11, m.h12 }, { m.h12, m.h22 } };
      cplx q[3];
      for (int f = 0; f < 3; ++f) q[f] = m.sg * Q[orc_idx(G, f, p, ej, ei, nj, ni)];
      cplx f1[3], f2[3];
      normal_flux(G, q, m.sg, h, 0, f1);
      normal_flux(G, q, m.sg, h, 1, f2);
      for (int f = 0; f < 3; ++f) {
        F1[(f * ns + nj) * ns + ni] = f1[f];
        F2[(f * ns + nj) * ns + ni] = f2[f];
      }
    }
  /* common fluxes at the four faces */
  for (int t = 0; t < ns; ++t) {
    face_flux(G, Q, p, ej, ei, EW, t, FW + 3 * t);
    face_flux(G, Q, p, ej, ei, EE, t, FE + 3 * t);
    face_flux(G, Q, p, ej, ei, ES, t, FS + 3 * t);
    face_flux(G, Q, p, ej, ei, EN, t, FN + 3 * t);
  }
  /* derivative of the continuous flux polynomial (Eqs. 12, 14) and sources */
  for (int nj = 0; nj < ns; ++nj)
    for (int ni = 0; ni < ns; ++ni) {
      double X = tan(node_x(G, ei, ni)), Y = tan(node_x(G, ej, nj));
      metric_t m = metric_at(G, X, Y);
      double h[2][2] = { { m.h11, m.h12 }, { m.h12, m.h22 } };
      double c0[2][2], csy[2][2][2];
      christoffel_at(G, p, X, Y, c0, csy);
      cplx q[3];
      for (int f = 0; f < 3; ++f) q[f] = m.sg * Q[orc_idx(G, f, p, ej, ei, nj, ni)];
      int64_t n0 = orc_idx(G, 0, p, ej, ei, nj, ni);
      for (int f = 0; f < 3; ++f) {
        /* x^1 direction: extended points {W face, row nodes, E face} */
        cplx d1 = G->Dt[ni][0] * FW[3 * nj + f] + G->Dt[ni][ns + 1] * FE[3 * nj + f];
        for (int k = 0; k < ns; ++k) d1 += G->Dt[ni][k + 1] * F1[(f * ns + nj) * ns + k];
        cplx d2 = G->Dt[nj][0] * FS[3 * ni + f] + G->Dt[nj][ns + 1] * FN[3 * ni + f];
        for (int k = 0; k < ns; ++k) d2 += G->Dt[nj][k + 1] * F2[(f * ns + k) * ns + ni];
        cplx rhs = -(2.0 / D) * (d1 + d2);
        if (f > 0) {
          int i = f - 1;
          /* Coriolis: -2 sqrt(g) Gamma^i_{j0} H u^j = -2 Gamma^i_{0j} q^j */
          cplx src = 0.0;
          for (int j = 0; j < 2; ++j) src += -2.0 * c0[i][j] * q[1 + j];
          /* metric: -sqrt(g) Gamma^i_jk (H u^j u^k + g h^jk H^2 / 2) */
          for (int j = 0; j < 2; ++j)
            for (int k = 0; k < 2; ++k)
              src += -csy[i][j][k] * (q[1 + j] * q[1 + k] / q[0] + 0.5 * G->g * h[j][k] * q[0] * q[0] / m.sg);
          /* orography: -sqrt(g) H g h^ij dh_B/dx^j */
          if (G->dhb)
            for (int j = 0; j < 2; ++j) src += -q[0] * G->g * h[i][j] * G->dhb[(int64_t)j * N + n0];
          rhs += src;
        }
        dQ[(int64_t)f * N + n0] = rhs / m.sg;
      }
    }
}

/* Complex right-hand side dQ/dt = F(Q) for Q = (H, H u^1, H u^2).  Elements
   are independent (each writes only its own nodes), so the loop over them
   may run on several threads (OpenMP, OMP_NUM_THREADS) with results that do
   not depend on the thread count. */
int orc_rhs_complex(const orc_grid *G, const cplx *Q, cplx *dQ) {
  int ne = G->ne;
  int64_t N = orc_num_nodes(G);
  for (int64_t i = 0; i < 3 * N; ++i)
    if (!isfinite(creal(Q[i])) || !isfinite(cimag(Q[i]))) return ORC_ENONFINITE;
  for (int64_t i = 0; i < N; ++i)
    if (!(creal(Q[i]) > 0.0)) return ORC_EDEPTH;
  int64_t nel = 6LL * ne * ne;
#pragma omp parallel for schedule(static)
  for (int64_t e = 0; e < nel; ++e) {
    int ei = (int)(e % ne), ej = (int)((e / ne) % ne), p = (int)(e / ((int64_t)ne * ne));
    element_rhs(G, Q, dQ, p, ej, ei);
  }
  return ORC_OK;
}

/* Real right-hand side: the complex evaluation at a real state.             */
int orc_rhs(const orc_grid *G, const double *Q, double *dQ) {
  int64_t n3 = 3 * orc_num_nodes(G);
  cplx *z = (cplx *)malloc(sizeof(cplx) * n3), *r = (cplx *)malloc(sizeof(cplx) * n3);
  if (!z || !r) { free(z); free(r); return ORC_ENOMEM; }
  for (int64_t i = 0; i < n3; ++i) z[i] = Q[i];
  int rc = orc_rhs_complex(G, z, r);
  if (rc == ORC_OK)
    for (int64_t i = 0; i < n3; ++i) dQ[i] = creal(r[i]);
  free(z); free(r);
  return rc;
}

/* Complex-step Jacobian-vector product, Eq. (28): Im F(Q + i eps V) / eps.  */
int orc_jvp(const orc_grid *G, const double *Q, const double *V, double eps, double *JV) {
  int64_t n3 = 3 * orc_num_nodes(G);
  if (!(eps > 0.0)) return ORC_EINVAL;
  cplx *z = (cplx *)malloc(sizeof(cplx) * n3), *r = (cplx *)malloc(sizeof(cplx) * n3);
  if (!z || !r) { free(z); free(r); return ORC_ENOMEM; }
  for (int64_t i = 0; i < n3; ++i) z[i] = Q[i] + I * (eps * V[i]);
  int rc = orc_rhs_complex(G, z, r);
  if (rc == ORC_OK)
    for (int64_t i = 0; i < n3; ++i) JV[i] = cimag(r[i]) / eps;
  free(z); free(r);
  return rc;
}

/* Complex RHS on split real/imaginary planes (used by pins on the complex   */
/* step itself, e.g. its independence of eps).                               */
int orc_rhs_split(const orc_grid *G, const double *re, const double *im, double *ore, double *oim) {
  int64_t n3 = 3 * orc_num_nodes(G);
  cplx *z = (cplx *)malloc(sizeof(cplx) * n3), *r = (cplx *)malloc(sizeof(cplx) * n3);
  if (!z || !r) { free(z); free(r); return ORC_ENOMEM; }
  for (int64_t i = 0; i < n3; ++i) z[i] = re[i] + I * im[i];
  int rc = orc_rhs_complex(G, z, r);
  if (rc == ORC_OK)
    for (int64_t i = 0; i < n3; ++i) { ore[i] = creal(r[i]); oim[i] = cimag(r[i]); }
  free(z); free(r);
  return rc;
}

/* Quadrature weights w_m w_n sqrt(g) (Delta/2)^2 at every node: the global  */
/* integral of Eq. (42) including the constant element Jacobian.             */
void orc_mass_weights(const orc_grid *G, double *wq) {
  int ne = G->ne, ns = G->ns;
  double D = orc_delta(G);
  for (int p = 0; p < 6; ++p)
    for (int ej = 0; ej < ne; ++ej)
      for (int ei = 0; ei < ne; ++ei)
        for (int nj = 0; nj < ns; ++nj)
          for (int ni = 0; ni < ns; ++ni) {
            double X = tan(node_x(G, ei, ni)), Y = tan(node_x(G, ej, nj));
            metric_t m = metric_at(G, X, Y);
            wq[orc_idx(G, 0, p, ej, ei, nj, ni)] = G->w[ni] * G->w[nj] * m.sg * 0.25 * D * D;
          }
}

/* ------------------------------------------------------------------------ */
/* Diagnostics of Sec. 5.4.  Per node: relative vorticity zeta (Eq. 43),     */
/* Coriolis parameter f (Eq. 46); integrals over the sphere of H, of the      */
/* total energy (1/2)[H g_ij u^i u^j + g_r((H + h_B)^2 - h_B^2)] and of the   */
/* potential enstrophy (zeta + f)^2 / (2H).  hB: NULL or N nodal values;     */
/* zeta, fcor: NULL or N values; out3: mass, energy, potential enstrophy.    */
int orc_diagnostics(const orc_grid *G, const double *Q, const double *hB, double *zeta, double *fcor, double *out3) {
  int ne = G->ne, ns = G->ns;
  int64_t N = orc_num_nodes(G);
  for (int64_t i = 0; i < 3 * N; ++i)
    if (!isfinite(Q[i])) return ORC_ENONFINITE;
  for (int64_t i = 0; i < N; ++i)
    if (!(Q[i] > 0.0)) return ORC_EDEPTH;
  double D = orc_delta(G), a2 = G->a * G->a;
  double v1[ORC_MAXNS][ORC_MAXNS], v2[ORC_MAXNS][ORC_MAXNS];   /* covariant g_jk u^k, [nj][ni] */
  double mass = 0.0, energy = 0.0, enstrophy = 0.0;
  for (int p = 0; p < 6; ++p)
    for (int ej = 0; ej < ne; ++ej)
      for (int ei = 0; ei < ne; ++ei) {
        for (int nj = 0; nj < ns; ++nj)
          for (int ni = 0; ni < ns; ++ni) {
            double X = tan(node_x(G, ei, ni)), Y = tan(node_x(G, ej, nj));
            double d2 = 1.0 + X * X + Y * Y;
            double g11 = a2 * (1.0 + X * X) * (1.0 + X * X) * (1.0 + Y * Y) / (d2 * d2);   /* (64) */
            double g12 = -a2 * X * Y * (1.0 + X * X) * (1.0 + Y * Y) / (d2 * d2);          /* (65) */
            double g22 = a2 * (1.0 + X * X) * (1.0 + Y * Y) * (1.0 + Y * Y) / (d2 * d2);   /* (66) */
            int64_t i0 = orc_idx(G, 0, p, ej, ei, nj, ni);
            double H = Q[i0], u1 = Q[N + i0] / H, u2 = Q[2 * N + i0] / H;
            v1[nj][ni] = g11 * u1 + g12 * u2;
            v2[nj][ni] = g12 * u1 + g22 * u2;
          }
        for (int nj = 0; nj < ns; ++nj)
          for (int ni = 0; ni < ns; ++ni) {
            double X = tan(node_x(G, ei, ni)), Y = tan(node_x(G, ej, nj));
            metric_t m = metric_at(G, X, Y);
            double d2 = 1.0 + X * X + Y * Y;
            /* element-local derivatives (reading V1) */
            double d1v2 = 0.0, d2v1 = 0.0;
            for (int k = 0; k < ns; ++k) {
              d1v2 += G->Dgl[ni][k] * v2[nj][k];
              d2v1 += G->Dgl[nj][k] * v1[k][ni];
            }
            double z = (2.0 / D) * (d1v2 - d2v1) / m.sg;                               /* (43) */
            double fac = sin(G->phi[p]) - X * cos(G->phi[p]) * sin(G->alp[p]) + Y * cos(G->phi[p]) * cos(G->alp[p]);
            double f = 2.0 * G->omega / sqrt(d2) * fac;                                 /* (46) */
            int64_t i0 = orc_idx(G, 0, p, ej, ei, nj, ni);
            double H = Q[i0], u1 = Q[N + i0] / H, u2 = Q[2 * N + i0] / H;
            double hb = hB ? hB[i0] : 0.0;
            double ke = H * (u1 * v1[nj][ni] + u2 * v2[nj][ni]);
            double e = 0.5 * (ke + G->g * ((H + hb) * (H + hb) - hb * hb));
            double zs = (z + f) * (z + f) / (2.0 * H);
            double wgt = G->w[ni] * G->w[nj] * m.sg * 0.25 * D * D;
            mass += wgt * H;
            energy += wgt * e;
            enstrophy += wgt * zs;
            if (zeta) zeta[i0] = z;
            if (fcor) fcor[i0] = f;
          }
      }
  out3[0] = mass;
  out3[1] = energy;
  out3[2] = enstrophy;
  return ORC_OK;
}
