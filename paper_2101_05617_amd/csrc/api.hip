// Host side of the library: grid set-up (Gauss-Legendre operators, rotated
// cubed-sphere frames, panel connectivity and interface maps, tangent
// tables), context management and the right-hand-side / J*v entry points.
//
// Geometry is built here from first principles, independently of any other
// implementation: the six panels of the unrotated cube are rotated as one rigid
// body so that panel 0 has centre (lambda0, phi0) and turn alpha0 (App. B); the
// gnomonic coordinates are X = P.e1/P.ec, Y = P.e2/P.ec (App. B, Eqs. 59-60);
// neighbours and edge orientations are found by matching Cartesian points;
// the contravariant interface maps (App. C) are the Jacobians between the two
// panels' coordinate bases at each face point.
#include "dfrsw_internal.h"

#include <algorithm>
#include <atomic>
#include <cmath>
#include <cstring>
#include <mutex>

namespace dfrsw {

static thread_local std::string g_last_error;
void set_error(const std::string &msg) { g_last_error = msg; }

int set_expm_lds_limit(int m);
size_t expm_lds_bytes(int m);

// ---------------------------------------------------------------------------
// Gauss-Legendre points and weights (roots of P_ns), symmetric by construction
static void gauss_legendre_sym(int ns, std::vector<double> &x, std::vector<double> &w) {
  x.assign(ns, 0.0);
  w.assign(ns, 0.0);
  const long double pi = 3.141592653589793238462643383279503L;
  for (int k = 0; k < (ns + 1) / 2; ++k) {
    long double z = std::cos(pi * (k + 0.75L) / (ns + 0.5L));   // k-th largest root
    long double dp = 0.0L;
    for (int it = 0; it < 60; ++it) {
      long double p0 = 1.0L, p1 = z;
      for (int l = 2; l <= ns; ++l) {
        long double p2 = ((2 * l - 1) * z * p1 - (l - 1) * p0) / l;
        p0 = p1;
        p1 = p2;
      }
      if (ns == 1) { p1 = z; p0 = 1.0L; }
      dp = ns * (z * p1 - p0) / (z * z - 1.0L);
      long double dz = p1 / dp;
      z -= dz;
      if (std::fabs((double)dz) < 1e-19) break;
    }
    long double p0 = 1.0L, p1 = z;
    for (int l = 2; l <= ns; ++l) {
      long double p2 = ((2 * l - 1) * z * p1 - (l - 1) * p0) / l;
      p0 = p1;
      p1 = p2;
    }
    dp = ns * (z * p1 - p0) / (z * z - 1.0L);
    const long double wk = 2.0L / ((1.0L - z * z) * dp * dp);
    x[ns - 1 - k] = (double)z;
    x[k] = -(double)z;
    w[k] = w[ns - 1 - k] = (double)wk;
  }
  if (ns % 2 == 1) x[ns / 2] = 0.0;
}

// barycentric weights of a node set
static std::vector<long double> bary(const std::vector<long double> &t) {
  std::vector<long double> b(t.size(), 1.0L);
  for (size_t j = 0; j < t.size(); ++j)
    for (size_t k = 0; k < t.size(); ++k)
      if (k != j) b[j] /= (t[j] - t[k]);
  return b;
}

static void build_ops(int ns, const std::vector<double> &xi, Ops1D &ops) {
  std::memset(&ops, 0, sizeof(ops));
  // extended points {-1, xi_1..xi_ns, +1}; differentiation matrix from the
  // barycentric formula D_ij = (b_j/b_i)/(t_i - t_j), D_ii = -sum_{j!=i} D_ij
  std::vector<long double> t(ns + 2);
  t[0] = -1.0L;
  for (int k = 0; k < ns; ++k) t[k + 1] = xi[k];
  t[ns + 1] = 1.0L;
  std::vector<long double> b = bary(t);
  for (int i = 1; i <= ns; ++i) {
    long double diag = 0.0L;
    for (int j = 0; j < ns + 2; ++j) {
      if (j == i) continue;
      long double d = (b[j] / b[i]) / (t[i] - t[j]);
      ops.Dt[i - 1][j] = (double)d;
      diag -= d;
    }
    ops.Dt[i - 1][i] = (double)diag;
  }
  // Lagrange basis on the GL points at -1 and +1 (barycentric form)
  std::vector<long double> g(ns);
  for (int k = 0; k < ns; ++k) g[k] = xi[k];
  std::vector<long double> bg = bary(g);
  for (int side = 0; side < 2; ++side) {
    const long double s = side ? 1.0L : -1.0L;
    long double den = 0.0L;
    for (int k = 0; k < ns; ++k) den += bg[k] / (s - g[k]);
    for (int k = 0; k < ns; ++k) {
      const long double v = (bg[k] / (s - g[k])) / den;
      (side ? ops.lp : ops.lm)[k] = (double)v;
    }
  }
}

// GL collocation derivative matrix (for the orography gradient)
static std::vector<double> gl_deriv(int ns, const std::vector<double> &xi) {
  std::vector<long double> g(xi.begin(), xi.end());
  std::vector<long double> b = bary(g);
  std::vector<double> D(ns * ns, 0.0);
  for (int i = 0; i < ns; ++i) {
    long double diag = 0.0L;
    for (int j = 0; j < ns; ++j) {
      if (j == i) continue;
      long double d = (b[j] / b[i]) / (g[i] - g[j]);
      D[i * ns + j] = (double)d;
      diag -= d;
    }
    D[i * ns + i] = (double)diag;
  }
  return D;
}

// ---------------------------------------------------------------------------
// cube frames
static inline double dot3(const double *a, const double *b) { return a[0] * b[0] + a[1] * b[1] + a[2] * b[2]; }

static void build_frames(double l0, double f0, double a0, double ec[6][3], double e1[6][3], double e2[6][3]) {
  // unrotated cube: panels 0..3 on the equator west to east, 4 north, 5 south
  static const double C0[6][3] = {{1, 0, 0}, {0, 1, 0}, {-1, 0, 0}, {0, -1, 0}, {0, 0, 1}, {0, 0, -1}};
  static const double A0[6][3] = {{0, 1, 0}, {-1, 0, 0}, {0, -1, 0}, {1, 0, 0}, {0, 1, 0}, {0, 1, 0}};
  static const double B0[6][3] = {{0, 0, 1}, {0, 0, 1}, {0, 0, 1}, {0, 0, 1}, {-1, 0, 0}, {1, 0, 0}};
  // rotation taking the unrotated panel-0 frame (x, y, z) to the frame at
  // centre (l0, f0) turned by a0: columns ec0, e10, e20
  const double E[3] = {-std::sin(l0), std::cos(l0), 0.0};
  const double Nn[3] = {-std::sin(f0) * std::cos(l0), -std::sin(f0) * std::sin(l0), std::cos(f0)};
  double R[3][3];
  for (int i = 0; i < 3; ++i) {
    R[i][0] = (i == 0 ? std::cos(f0) * std::cos(l0) : i == 1 ? std::cos(f0) * std::sin(l0) : std::sin(f0));
    R[i][1] = std::cos(a0) * E[i] - std::sin(a0) * Nn[i];
    R[i][2] = std::sin(a0) * E[i] + std::cos(a0) * Nn[i];
  }
  for (int p = 0; p < 6; ++p)
    for (int i = 0; i < 3; ++i) {
      ec[p][i] = R[i][0] * C0[p][0] + R[i][1] * C0[p][1] + R[i][2] * C0[p][2];
      e1[p][i] = R[i][0] * A0[p][0] + R[i][1] * A0[p][1] + R[i][2] * A0[p][2];
      e2[p][i] = R[i][0] * B0[p][0] + R[i][1] * B0[p][1] + R[i][2] * B0[p][2];
    }
}

static void point_on(const Ctx &c, int p, double X, double Y, double P[3]) {
  double r[3], n2 = 0.0;
  for (int i = 0; i < 3; ++i) {
    r[i] = c.ec[p][i] + X * c.e1[p][i] + Y * c.e2[p][i];
    n2 += r[i] * r[i];
  }
  const double inv = 1.0 / std::sqrt(n2);
  for (int i = 0; i < 3; ++i) P[i] = r[i] * inv;
}

// coordinate basis dP/dx^1, dP/dx^2 on panel p at P (unit sphere)
static void basis_at(const Ctx &c, int p, const double P[3], double B1[3], double B2[3]) {
  const double pc = dot3(P, c.ec[p]);
  const double X = dot3(P, c.e1[p]) / pc, Y = dot3(P, c.e2[p]) / pc;
  double r[3], n2 = 0.0;
  for (int i = 0; i < 3; ++i) {
    r[i] = c.ec[p][i] + X * c.e1[p][i] + Y * c.e2[p][i];
    n2 += r[i] * r[i];
  }
  const double nr = std::sqrt(n2);
  for (int i = 0; i < 3; ++i) {
    const double u = r[i] / nr;
    B1[i] = (1.0 + X * X) * (c.e1[p][i] - u * dot3(r, c.e1[p]) / nr) / nr;
    B2[i] = (1.0 + Y * Y) * (c.e2[p][i] - u * dot3(r, c.e2[p]) / nr) / nr;
  }
}

static void edge_xy(int edge, double s, double &X, double &Y) {
  switch (edge) {
    case 0: X = -1.0; Y = s; break;
    case 1: X = 1.0; Y = s; break;
    case 2: X = s; Y = -1.0; break;
    default: X = s; Y = 1.0; break;
  }
}

static int build_connectivity(Ctx &c) {
  for (int p = 0; p < 6; ++p)
    for (int e = 0; e < 4; ++e) {
      double X, Y, P0[3], P1[3];
      edge_xy(e, 0.0, X, Y);
      point_on(c, p, X, Y, P0);
      edge_xy(e, 0.5, X, Y);
      point_on(c, p, X, Y, P1);
      int found = 0;
      for (int q = 0; q < 6 && !found; ++q) {
        if (q == p) continue;
        for (int f = 0; f < 4 && !found; ++f) {
          double Q0[3], Qa[3], Qb[3];
          edge_xy(f, 0.0, X, Y);
          point_on(c, q, X, Y, Q0);
          double d0 = 0.0;
          for (int i = 0; i < 3; ++i) d0 += (P0[i] - Q0[i]) * (P0[i] - Q0[i]);
          if (d0 > 1e-20) continue;
          edge_xy(f, 0.5, X, Y);
          point_on(c, q, X, Y, Qa);
          edge_xy(f, -0.5, X, Y);
          point_on(c, q, X, Y, Qb);
          double da = 0.0, db = 0.0;
          for (int i = 0; i < 3; ++i) {
            da += (P1[i] - Qa[i]) * (P1[i] - Qa[i]);
            db += (P1[i] - Qb[i]) * (P1[i] - Qb[i]);
          }
          if (da < 1e-20 || db < 1e-20) {
            c.ga.nb_q[p][e] = q;
            c.ga.nb_e[p][e] = f;
            c.ga.nb_rev[p][e] = (da < 1e-20) ? 0 : 1;
            found = 1;
          }
        }
      }
      if (!found) {
        set_error("panel connectivity could not be established");
        return DFR_E_INVAL;
      }
    }
  return DFR_OK;
}

static const double PI = 3.14159265358979323846;

// element-edge and node abscissae x in [-pi/4, pi/4]
static double node_abscissa(const Ctx &c, int e, int k) {
  const double D = 0.5 * PI / c.ne;
  return -0.25 * PI + e * D + 0.5 * (1.0 + c.xi[k]) * D;
}
static double edge_abscissa(const Ctx &c, int e) { return -0.25 * PI + e * (0.5 * PI / c.ne); }

static int setup_geometry(Ctx &c, const double *hB) {
  gauss_legendre_sym(c.ns, c.xi, c.wgl);
  build_ops(c.ns, c.xi, c.ops);
  build_frames(c.lam0, c.phi0, c.alp0, c.ec, c.e1, c.e2);
  GridArgs &g = c.ga;
  std::memset(&g, 0, sizeof(g));
  g.ne = c.ne;
  g.nelem = c.nelem;
  g.n = c.n;
  g.g_red = c.gravity / (c.radius * c.radius);
  g.omega = c.omega;
  g.two_over_delta = 2.0 / (0.5 * PI / c.ne);
  const double zhat[3] = {0.0, 0.0, 1.0};
  for (int p = 0; p < 6; ++p) {
    // Coriolis factor of Eqs. (71)-(74): z . (ec + X e1 + Y e2)
    g.cA[p] = dot3(zhat, c.ec[p]);
    g.cB[p] = dot3(zhat, c.e1[p]);
    g.cC[p] = dot3(zhat, c.e2[p]);
  }
  int rc = build_connectivity(c);
  if (rc) return rc;

  const int ne = c.ne, ns = c.ns;
  std::vector<Tan3> tn(ne * ns);
  for (int e = 0; e < ne; ++e)
    for (int k = 0; k < ns; ++k) {
      const double X = std::tan(node_abscissa(c, e, k));
      tn[e * ns + k] = {X, 1.0 + X * X, 1.0 / (1.0 + X * X), 0.0};
    }
  std::vector<double> te(ne + 1);
  for (int e = 0; e <= ne; ++e) te[e] = std::tan(edge_abscissa(c, e));
  te[0] = -1.0;
  te[ne] = 1.0;

  // contravariant maps own <- neighbour at every panel-edge face point
  std::vector<double> xf((size_t)6 * 4 * ne * ns * 4);
  for (int p = 0; p < 6; ++p)
    for (int e = 0; e < 4; ++e) {
      const int q = g.nb_q[p][e];
      for (int a = 0; a < ne; ++a)
        for (int t = 0; t < ns; ++t) {
          const double s = tn[a * ns + t].x;
          double X, Y, P[3], b1[3], b2[3], n1[3], n2[3];
          edge_xy(e, s, X, Y);
          point_on(c, p, X, Y, P);
          basis_at(c, p, P, b1, b2);
          basis_at(c, q, P, n1, n2);
          const double g11 = dot3(b1, b1), g12 = dot3(b1, b2), g22 = dot3(b2, b2);
          const double det = g11 * g22 - g12 * g12;
          // A_own = G^{-1} [b_i . n_j] A_nbr
          const double r11 = dot3(b1, n1), r12 = dot3(b1, n2), r21 = dot3(b2, n1), r22 = dot3(b2, n2);
          double *M = &xf[(((size_t)p * 4 + e) * ne * ns + a * ns + t) * 4];
          M[0] = (g22 * r11 - g12 * r21) / det;
          M[1] = (g22 * r12 - g12 * r22) / det;
          M[2] = (g11 * r21 - g12 * r11) / det;
          M[3] = (g11 * r22 - g12 * r12) / det;
          // the maps are exact integers or 2s/(1+s^2) up to rounding; snap
          // entries that are within rounding of 0 or +-1
          for (int k = 0; k < 4; ++k) {
            if (std::fabs(M[k]) < 1e-13) M[k] = 0.0;
            if (std::fabs(std::fabs(M[k]) - 1.0) < 1e-13) M[k] = M[k] > 0 ? 1.0 : -1.0;
          }
        }
    }

  DFR_HIP(hipMalloc(&c.d_tnode, sizeof(Tan3) * tn.size()));
  DFR_HIP(hipMemcpy(c.d_tnode, tn.data(), sizeof(Tan3) * tn.size(), hipMemcpyHostToDevice));
  DFR_HIP(hipMalloc(&c.d_tedge, sizeof(double) * te.size()));
  DFR_HIP(hipMemcpy(c.d_tedge, te.data(), sizeof(double) * te.size(), hipMemcpyHostToDevice));
  DFR_HIP(hipMalloc(&c.d_xform, sizeof(double) * xf.size()));
  DFR_HIP(hipMemcpy(c.d_xform, xf.data(), sizeof(double) * xf.size(), hipMemcpyHostToDevice));
  g.tnode = c.d_tnode;
  g.tedge = c.d_tedge;
  g.xform = c.d_xform;

  // collocation data of the diagnostics
  {
    const std::vector<double> D = gl_deriv(ns, c.xi);
    std::memset(&c.dops, 0, sizeof(c.dops));
    for (int k = 0; k < ns; ++k) {
      c.dops.w[k] = c.wgl[k];
      for (int j = 0; j < ns; ++j) c.dops.Dg[k][j] = D[k * ns + j];
    }
  }
  if (hB) {
    DFR_HIP(hipMalloc(&c.d_hB, sizeof(double) * c.n));
    DFR_HIP(hipMemcpy(c.d_hB, hB, sizeof(double) * c.n, hipMemcpyHostToDevice));
  }
  if (hB) {
    // orography source (g/a^2) a^2 h^ij d_j h_B per node, derivative by GL collocation
    const std::vector<double> D = gl_deriv(ns, c.xi);
    const double s = g.two_over_delta;
    const int64_t N = c.n;
    std::vector<double> o(2 * N);
    for (int p = 0; p < 6; ++p)
      for (int ej = 0; ej < ne; ++ej)
        for (int ei = 0; ei < ne; ++ei) {
          const int64_t base = (((int64_t)p * ne + ej) * ne + ei) * ns * ns;
          for (int nj = 0; nj < ns; ++nj)
            for (int ni = 0; ni < ns; ++ni) {
              double d1 = 0.0, d2 = 0.0;
              for (int k = 0; k < ns; ++k) {
                d1 += D[ni * ns + k] * hB[base + nj * ns + k];
                d2 += D[nj * ns + k] * hB[base + k * ns + ni];
              }
              d1 *= s;
              d2 *= s;
              const Tan3 tx = tn[ei * ns + ni], ty = tn[ej * ns + nj];
              const double d2m = 1.0 + tx.x * tx.x + ty.x * ty.x;
              const double e11 = d2m * tx.rax, e22 = d2m * ty.rax, e12 = tx.x * ty.x * d2m * tx.rax * ty.rax;
              o[base + nj * ns + ni] = g.g_red * (e11 * d1 + e12 * d2);
              o[N + base + nj * ns + ni] = g.g_red * (e12 * d1 + e22 * d2);
            }
        }
    DFR_HIP(hipMalloc(&c.d_orog, sizeof(double) * o.size()));
    DFR_HIP(hipMemcpy(c.d_orog, o.data(), sizeof(double) * o.size(), hipMemcpyHostToDevice));
    g.orog = c.d_orog;
  }
  DFR_HIP(hipMalloc(&c.d_err, sizeof(int)));
  DFR_HIP(hipMemset(c.d_err, 0, sizeof(int)));
  g.err_flag = c.d_err;
  return DFR_OK;
}

// admissible element tiles: TX, TY divide ne, one thread per node (<= 1024),
// dynamic LDS within the device limit
std::vector<std::pair<int, int>> tile_candidates(const Ctx &c) {
  std::vector<std::pair<int, int>> out;
  const int nn = c.ns * c.ns;
  for (int tx = 1; tx <= c.ne; ++tx) {
    if (c.ne % tx) continue;
    for (int ty = 1; ty <= c.ne; ++ty) {
      if (c.ne % ty) continue;
      if (tx * ty * nn > 1024) continue;
      if (dfr_lds_bytes(c.ns, tx, ty, false) > c.lds_limit) continue;
      out.push_back({tx, ty});
    }
  }
  return out;
}

// default tile: the largest (then squarest) tile that still gives two
// workgroups per compute unit; on small grids, the one with most workgroups
static void default_tile(Ctx &c) {
  const auto cand = tile_candidates(c);
  int best = -1;
  long best_key = -1;
  for (size_t k = 0; k < cand.size(); ++k) {
    const int tx = cand[k].first, ty = cand[k].second;
    const long nb = 6L * (c.ne / tx) * (c.ne / ty);
    const long nel = (long)tx * ty;
    long key;
    if (nb >= 512) key = (1L << 40) + nel * 1000 - std::abs(tx - ty);
    else key = nb * 1000 + nel;
    if (key > best_key) {
      best_key = key;
      best = (int)k;
    }
  }
  c.tile_tx = c.ar_tx = cand[best].first;
  c.tile_ty = c.ar_ty = cand[best].second;
}

static int alloc_workspace(Ctx &c) {
  const int64_t n3 = c.n3;
  DFR_HIP(hipMalloc(&c.d_diag, sizeof(double) * (3 * diag_blocks(&c) + 3)));
  // largest grid of any tile (1 x 1 tiles) or of the vector kernels
  const int64_t nb = std::max<int64_t>(6LL * c.ne * c.ne + 8, 8192);
  DFR_HIP(hipMalloc(&c.d_partials, sizeof(double) * 2 * nb));
  DFR_HIP(hipMalloc(&c.d_partials2, sizeof(double) * 2 * nb));
  DFR_HIP(hipMalloc(&c.d_counter, sizeof(unsigned)));
  DFR_HIP(hipMemset(c.d_counter, 0, sizeof(unsigned)));
  DFR_HIP(hipMalloc(&c.d_kd, sizeof(KDev)));
  DFR_HIP(hipMemset(c.d_kd, 0, sizeof(KDev)));
  DFR_HIP(hipHostMalloc((void **)&c.mail, sizeof(HostMail), hipHostMallocCoherent | hipHostMallocMapped));
  std::memset(c.mail, 0, sizeof(HostMail));
  DFR_HIP(hipHostGetDevicePointer((void **)&c.d_mail, c.mail, 0));
  DFR_HIP(hipMalloc(&c.d_V, sizeof(double) * (MAX_M + 1) * n3));
  DFR_HIP(hipMalloc(&c.d_W, sizeof(double) * MAX_P * n3));
  DFR_HIP(hipMalloc(&c.d_qf32, sizeof(float) * n3));
  DFR_HIP(hipMalloc(&c.d_tmp, sizeof(double) * n3));
  // the small exponential keeps four padded m x m FP64 matrices in LDS
  int lds = 0, lds_optin = 0;
  (void)hipDeviceGetAttribute(&lds, hipDeviceAttributeMaxSharedMemoryPerBlock, c.device);
  (void)hipDeviceGetAttribute(&lds_optin, hipDeviceAttributeSharedMemPerBlockOptin, c.device);
  lds = std::max(lds, lds_optin) - 1024;
  // the DFR kernel's static LDS (operators, halo table, reduction) stays below 8 KB
  c.lds_limit = (size_t)lds - 8192;
  default_tile(c);
  {
    const int rc = dfr_set_lds_limits(&c, c.lds_limit);
    if (rc) return rc;
  }
  c.max_m = MAX_M;   // largest Krylov dimension whose exponential fits in LDS
  while (c.max_m > 2 && expm_lds_bytes(c.max_m) > (size_t)lds) --c.max_m;
  if (expm_lds_bytes(c.max_m) > (size_t)lds) {
    set_error("device LDS too small for the Krylov exponential");
    return DFR_E_INVAL;
  }
  int rc = set_expm_lds_limit(c.max_m);
  if (rc) return rc;
  return DFR_OK;
}

static void free_ctx(Ctx &c) {
  (void)hipFree(c.d_tnode);
  (void)hipFree(c.d_tedge);
  (void)hipFree(c.d_xform);
  (void)hipFree(c.d_orog);
  (void)hipFree(c.d_hB);
  (void)hipFree(c.d_diag);
  (void)hipFree(c.d_err);
  (void)hipFree(c.d_partials);
  (void)hipFree(c.d_partials2);
  (void)hipFree(c.d_counter);
  (void)hipFree(c.d_kd);
  if (c.mail) (void)hipHostFree(c.mail);
  (void)hipFree(c.d_V);
  (void)hipFree(c.d_W);
  (void)hipFree(c.d_qf32);
  (void)hipFree(c.d_tmp);
}

bool timing_slot(KTimer *t, int kind, double units, hipEvent_t *start, hipEvent_t *stop) {
  if (!t->on || !((t->kinds >> kind) & 1u)) return false;
  if (t->used == t->pool.size()) {
    KTimer::EvPair e{};
    if (hipEventCreate(&e.a) != hipSuccess || hipEventCreate(&e.b) != hipSuccess) {
      t->on = false;
      return false;
    }
    t->pool.push_back(e);
  }
  KTimer::EvPair &e = t->pool[t->used];
  e.kind = kind;
  e.units = units;
  *start = e.a;
  *stop = e.b;
  return true;
}

void timing_fold(KTimer &t) {
  if (t.used == 0) return;
  (void)hipEventSynchronize(t.pool[t.used - 1].b);
  for (size_t k = 0; k < t.used; ++k) {
    float ms = 0.f;
    if (hipEventElapsedTime(&ms, t.pool[k].a, t.pool[k].b) == hipSuccess) {
      t.t_ms[t.pool[k].kind] += ms;
      t.t_n[t.pool[k].kind] += 1;
      t.t_units[t.pool[k].kind] += t.pool[k].units;
    }
  }
  t.used = 0;
}

void timing_done(KTimer *t) {
  // fold finished pairs back periodically so the pool stays small
  if (++t->used >= 4096) timing_fold(*t);
}

void timing_reset(KTimer &t, bool on) {
  timing_fold(t);
  for (int k = 0; k < DFR_K_NKINDS; ++k) {
    t.t_ms[k] = 0.0;
    t.t_n[k] = 0;
    t.t_units[k] = 0.0;
  }
  t.on = on;
}

void timing_free(KTimer &t) {
  for (auto &e : t.pool) {
    (void)hipEventDestroy(e.a);
    (void)hipEventDestroy(e.b);
  }
  t.pool.clear();
  t.used = 0;
}

// Wait for the kernel result numbered seq in the context's host mail: poll
// its sequence number, and the stream's status every 256 polls (an idle
// stream without the number, or a stream error, ends the wait).
int mail_wait(Ctx &c, unsigned seq) {
  volatile unsigned *s = &c.mail->seq;
  for (unsigned it = 1;; ++it) {
    if (*s == seq) break;
    if ((it & 255) == 0) {
      const hipError_t q = hipStreamQuery(c.stream);
      if (q == hipSuccess) {
        if (*s == seq) break;
        set_error("a kernel result did not reach the host");
        return DFR_E_HIP;
      }
      if (q != hipErrorNotReady) {
        set_error(std::string("HIP error: ") + hipGetErrorString(q));
        return DFR_E_HIP;
      }
    }
#if defined(__x86_64__)
    __builtin_ia32_pause();
#endif
  }
  std::atomic_thread_fence(std::memory_order_acquire);
  return DFR_OK;
}

// The flags latched by the kernels (bit 0: a non-finite input, bit 1: a
// non-positive depth), read and cleared in stream order; when it returns,
// every earlier operation on the stream has finished.
int latched_error(Ctx &c) {
  const unsigned seq = ++c.mail_seq;
  int rc = launch_err_mail(&c, seq);
  if (!rc) rc = mail_wait(c, seq);
  if (rc) return rc;
  const int flag = c.mail->err;
  if (flag) {
    if (flag & 1) {
      set_error("non-finite value in an input state");
      return DFR_E_NONFINITE;
    }
    set_error("non-positive fluid depth H");
    return DFR_E_DEPTH;
  }
  return DFR_OK;
}

}  // namespace dfrsw

namespace dfrsw {
// mean duration (ms) of `reps` launches after two untimed ones
template <typename F>
static int time_launches(Ctx &c, hipEvent_t e0, hipEvent_t e1, int reps, F launch, float *ms) {
  int rc = DFR_OK;
  // two untimed launches, then the fastest of three timed rounds
  for (int r = 0; r < 2 && !rc; ++r) rc = launch();
  float best = 1e30f;
  for (int round = 0; round < 3 && !rc; ++round) {
    (void)hipEventRecord(e0, c.stream);
    for (int r = 0; r < reps && !rc; ++r) rc = launch();
    if (rc) break;
    (void)hipEventRecord(e1, c.stream);
    (void)hipEventSynchronize(e1);
    float t = 0.f;
    (void)hipEventElapsedTime(&t, e0, e1);
    best = std::min(best, t / reps);
  }
  if (rc) return rc;
  *ms = best;
  return DFR_OK;
}

// a plain streaming copy, 16 bytes per lane, grid-stride (measurement only)
__global__ __launch_bounds__(512) void stream_copy_kernel(const float4 *__restrict__ a, float4 *__restrict__ b,
                                                          size_t n) {
  for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x)
    b[i] = a[i];
}

}  // namespace dfrsw

using namespace dfrsw;

extern "C" {

const char *dfr_last_error(void) { return g_last_error.c_str(); }

int dfr_stream_copy(const void *src, void *dst, size_t bytes, void *hip_stream) {
  if (!src || !dst || (bytes % 16) || ((uintptr_t)src % 16) || ((uintptr_t)dst % 16)) {
    set_error("dfr_stream_copy: null pointer, or a pointer or size not a multiple of 16 bytes");
    return DFR_E_INVAL;
  }
  const size_t n = bytes / 16;
  if (n == 0) return DFR_OK;
  const size_t blocks = std::min<size_t>(131072, (n + 511) / 512);
  hipLaunchKernelGGL(stream_copy_kernel, dim3((unsigned)blocks), dim3(512), 0, (hipStream_t)hip_stream,
                     (const float4 *)src, (float4 *)dst, n);
  DFR_HIP(hipGetLastError());
  return DFR_OK;
}

int dfr_create(const dfr_grid_desc *d, void *stream, dfr_ctx **out) {
  if (!d || !out) {
    set_error("null argument");
    return DFR_E_INVAL;
  }
  *out = nullptr;
  if (d->ne < 1 || d->p < 1 || d->p > MAX_NS - 1 || !(d->radius > 0.0) || !(d->gravity >= 0.0) ||
      !std::isfinite(d->omega)) {
    set_error("invalid grid descriptor (need ne >= 1, 1 <= p <= 7, radius > 0, gravity >= 0)");
    return DFR_E_INVAL;
  }
  dfr_ctx *h = new (std::nothrow) dfr_ctx();
  if (!h) return DFR_E_NOMEM;
  Ctx &c = h->c;
  c.ne = d->ne;
  c.p_deg = d->p;
  c.ns = d->p + 1;
  c.nelem = 6LL * c.ne * c.ne;
  c.n = c.nelem * c.ns * c.ns;
  c.n3 = 3 * c.n;
  c.radius = d->radius;
  c.omega = d->omega;
  c.gravity = d->gravity;
  c.lam0 = d->lambda0;
  c.phi0 = d->phi0;
  c.alp0 = d->alpha0;
  c.stream = (hipStream_t)stream;
  if (hipGetDevice(&c.device) != hipSuccess) {
    set_error("no HIP device");
    delete h;
    return DFR_E_HIP;
  }
  int rc = setup_geometry(c, d->hB);
  if (!rc) rc = alloc_workspace(c);
  if (!rc) rc = scratch_init(c.device);
  if (rc) {
    free_ctx(c);
    delete h;
    return rc;
  }
  *out = h;
  return DFR_OK;
}

int dfr_create_ode(int problem, int n, void *stream, dfr_ctx **out) {
  if (!out) return DFR_E_INVAL;
  *out = nullptr;
  const int nmax = problem == DFR_ODE_ADR ? 256 : 65536;
  if (problem < DFR_ODE_ADR || problem > DFR_ODE_SEMILINEAR || n < 3 || n > nmax) {
    set_error("dfr_create_ode: unknown problem or size out of range");
    return DFR_E_INVAL;
  }
  dfr_ctx *h = new (std::nothrow) dfr_ctx();
  if (!h) return DFR_E_NOMEM;
  Ctx &c = h->c;
  OdeArgs &o = c.ode;
  o.kind = problem;
  o.n = n;
  if (problem == DFR_ODE_ADR) {          // Sec. 5.1: eps = 1/100, alpha = -10, gamma = 100
    o.len = (int64_t)n * n;
    o.h = 1.0 / (n - 1);
    o.eps = 1.0 / 100.0;
    o.alpha = -10.0;
    o.gamma = 100.0;
  } else if (problem == DFR_ODE_BURGERS) {   // eps = 1e-3
    o.len = n;
    o.h = 1.0 / (n + 1);
    o.eps = 1e-3;
  } else {                                   // semilinear parabolic, time appended
    o.len = n + 1;
    o.h = 1.0 / (n + 1);
    double s = 0.0;
    for (int i = 1; i <= n; ++i) {
      const double x = i * o.h;
      s += x * (1.0 - x);
    }
    o.isum = o.h * s;
  }
  c.ode_kind = problem;
  c.ne = 1;
  c.p_deg = 1;
  c.ns = 2;
  c.nelem = 1;
  c.n = o.len;
  c.n3 = o.len;
  c.radius = c.omega = c.gravity = 1.0;
  c.stream = (hipStream_t)stream;
  int rc = DFR_OK;
  if (hipGetDevice(&c.device) != hipSuccess) {
    set_error("no HIP device");
    rc = DFR_E_HIP;
  }
  if (!rc && (hipMalloc(&c.d_err, sizeof(int)) != hipSuccess || hipMemset(c.d_err, 0, sizeof(int)) != hipSuccess)) {
    set_error("dfr_create_ode: out of device memory");
    rc = DFR_E_NOMEM;
  }
  c.ga.err_flag = c.d_err;
  if (!rc) rc = alloc_workspace(c);
  if (!rc) rc = scratch_init(c.device);
  if (rc) {
    free_ctx(c);
    delete h;
    return rc;
  }
  *out = h;
  return DFR_OK;
}

int64_t dfr_num_unknowns(const dfr_ctx *h) { return h ? h->c.n3 : -1; }

int dfr_timing_enable(dfr_ctx *h, int enable) {
  if (!h) return DFR_E_INVAL;
  timing_reset(h->c.tm, enable != 0);
  return DFR_OK;
}

int dfr_timing_read(dfr_ctx *h, int kind, double *total_ms, int64_t *launches) {
  if (!h || kind < 0 || kind >= DFR_K_NKINDS || !total_ms || !launches) return DFR_E_INVAL;
  KTimer &t = h->c.tm;
  timing_fold(t);
  *total_ms = t.t_ms[kind];
  *launches = t.t_n[kind];
  return DFR_OK;
}

int dfr_destroy(dfr_ctx *h) {
  if (!h) return DFR_OK;
  (void)hipStreamSynchronize(h->c.stream);
  timing_free(h->c.tm);
  free_ctx(h->c);
  delete h;
  return DFR_OK;
}

int64_t dfr_num_nodes(const dfr_ctx *h) { return h ? h->c.n : -1; }

int dfr_node_frames(const dfr_ctx *h, double *P, double *B1, double *B2) {
  if (h && h->c.ode_kind) {
    set_error("dfr_node_frames: a grid context is required (this one holds a test problem)");
    return DFR_E_INVAL;
  }
  if (!h || !P || !B1 || !B2) {
    set_error("null argument");
    return DFR_E_INVAL;
  }
  const Ctx &c = h->c;
  const int ne = c.ne, ns = c.ns;
  for (int p = 0; p < 6; ++p)
    for (int ej = 0; ej < ne; ++ej)
      for (int ei = 0; ei < ne; ++ei)
        for (int nj = 0; nj < ns; ++nj)
          for (int ni = 0; ni < ns; ++ni) {
            const int64_t n = ((((int64_t)p * ne + ej) * ne + ei) * ns + nj) * ns + ni;
            const double X = std::tan(node_abscissa(c, ei, ni)), Y = std::tan(node_abscissa(c, ej, nj));
            point_on(c, p, X, Y, P + 3 * n);
            basis_at(c, p, P + 3 * n, B1 + 3 * n, B2 + 3 * n);
          }
  return DFR_OK;
}

int dfr_set_tile(dfr_ctx *h, int tx, int ty) {
  if (h && h->c.ode_kind) {
    set_error("dfr_set_tile: a grid context is required (this one holds a test problem)");
    return DFR_E_INVAL;
  }
  if (!h) return DFR_E_INVAL;
  Ctx &c = h->c;
  for (const auto &t : tile_candidates(c))
    if (t.first == tx && t.second == ty) {
      c.tile_tx = c.ar_tx = tx;
      c.tile_ty = c.ar_ty = ty;
      return DFR_OK;
    }
  set_error("tile not admissible (TX, TY must divide ne, TX*TY*(p+1)^2 <= 1024, LDS within limit)");
  return DFR_E_INVAL;
}

int dfr_set_riemann(dfr_ctx *h, int solver) {
  if (h && h->c.ode_kind) {
    set_error("dfr_set_riemann: a grid context is required (this one holds a test problem)");
    return DFR_E_INVAL;
  }
  if (!h || (solver != DFR_RUSANOV && solver != DFR_AUSM)) {
    set_error("dfr_set_riemann: solver must be DFR_RUSANOV or DFR_AUSM");
    return DFR_E_INVAL;
  }
  h->c.ga.riemann = solver;
  return DFR_OK;
}

int dfr_get_riemann(const dfr_ctx *h, int *solver) {
  if (!h || !solver) return DFR_E_INVAL;
  *solver = h->c.ga.riemann;
  return DFR_OK;
}

int dfr_get_tile(const dfr_ctx *h, int *tx, int *ty) {
  if (!h || !tx || !ty) return DFR_E_INVAL;
  *tx = h->c.tile_tx;
  *ty = h->c.tile_ty;
  return DFR_OK;
}

int dfr_get_krylov_tile(const dfr_ctx *h, int *tx, int *ty) {
  if (!h || !tx || !ty) return DFR_E_INVAL;
  *tx = h->c.ar_tx;
  *ty = h->c.ar_ty;
  return DFR_OK;
}

int dfr_autotune(dfr_ctx *h, dfr_precision prec, int *tile_tx, int *tile_ty) {
  if (h && h->c.ode_kind) {
    set_error("dfr_autotune: a grid context is required (this one holds a test problem)");
    return DFR_E_INVAL;
  }
  if (!h || (prec != DFR_FP64 && prec != DFR_FP32_JV && prec != DFR_FP32_JV_BASIS32)) return DFR_E_INVAL;
  Ctx &c = h->c;
  const int64_t n3 = c.n3;
  // a smooth positive state and a direction in the Krylov workspace (and
  // FP32 copies of the direction and of a previous vector for an FP32 basis)
  double *q = c.d_V, *v = c.d_V + n3, *w = c.d_V + 2 * n3;
  float *vf = reinterpret_cast<float *>(c.d_V + 3 * n3), *pf = vf + n3, *wf = pf + n3;
  int rc = launch_fill(&c, q, v);
  if (rc) return rc;
  const bool fp32 = prec != DFR_FP64, b32 = prec == DFR_FP32_JV_BASIS32;
  if (fp32) {
    rc = launch_copy_to_f32(&c, n3, q, (float *)c.d_qf32);
    if (rc) return rc;
  }
  if (b32) {
    rc = launch_copy_to_f32(&c, n3, v, vf);
    if (!rc) rc = launch_copy_to_f32(&c, n3, q, pf);
    if (rc) return rc;
  }
  const double eps = fp32 ? 1e-20 : 1e-150;
  // the Krylov form: start of a sweep with four b-columns, kept interleaved
  // as KIOPS keeps them, and a previous vector (the KIOPS state is
  // re-initialised by every sweep)
  ArnoldiArgs ar{};
  ar.on = 1;
  ar.j = 0;
  ar.p = std::min(4, MAX_P);
  ar.start = 1;
  {
    const double *cols[4] = {v, v, v, v};
    rc = launch_w_interleave(&c, n3, ar.p, 1.0, cols, c.d_W, b32);
    if (rc) return rc;
  }
  for (int k = 0; k < ar.p; ++k) ar.W[k] = c.d_W;
  ar.wil = 1;
  ar.vprev = b32 ? (const void *)pf : (const void *)q;
  ar.pin = q;
  ar.np_in = 1;
  ar.pout = c.d_partials;
  ar.kd = c.d_kd;
  ar.tol = 0.0;
  ar.ybot[0] = 1.0;
  DFR_HIP(hipMemsetAsync(&c.d_kd->happy, 0, sizeof(int), c.stream));
  hipEvent_t e0, e1;
  DFR_HIP(hipEventCreate(&e0));
  DFR_HIP(hipEventCreate(&e1));
  const int keep[4] = {c.tile_tx, c.tile_ty, c.ar_tx, c.ar_ty};
  float best = 1e30f, best_ar = 1e30f;
  int bt[4] = {keep[0], keep[1], keep[2], keep[3]};
  const bool was_timing = c.tm.on;
  c.tm.on = false;
  for (const auto &t : tile_candidates(c)) {
    c.tile_tx = c.ar_tx = t.first;
    c.tile_ty = c.ar_ty = t.second;
    float ms = 0.f;
    rc = time_launches(c, e0, e1, 5, [&] {
      return launch_dfr(&c, q, (const float *)c.d_qf32, v, nullptr, eps, true, fp32, w, nullptr);
    }, &ms);
    if (rc) break;
    if (ms < best) {
      best = ms;
      bt[0] = t.first;
      bt[1] = t.second;
    }
    c.basis32 = b32;
    rc = time_launches(c, e0, e1, 5, [&] {
      return launch_dfr(&c, q, (const float *)c.d_qf32, b32 ? (const void *)vf : (const void *)v, nullptr, eps, true,
                        fp32, b32 ? (void *)wf : (void *)w, &ar);
    }, &ms);
    c.basis32 = false;
    if (rc) break;
    if (ms < best_ar) {
      best_ar = ms;
      bt[2] = t.first;
      bt[3] = t.second;
    }
  }
  c.tm.on = was_timing;
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  const int *use = rc ? keep : bt;
  c.tile_tx = use[0];
  c.tile_ty = use[1];
  c.ar_tx = use[2];
  c.ar_ty = use[3];
  if (tile_tx) *tile_tx = c.tile_tx;
  if (tile_ty) *tile_ty = c.tile_ty;
  return rc ? rc : latched_error(c);
}

int dfr_sync(dfr_ctx *h) {
  if (!h) return DFR_E_INVAL;
  DFR_HIP(hipStreamSynchronize(h->c.stream));
  return latched_error(h->c);
}

int dfr_diagnostics(dfr_ctx *h, const double *q, double *zeta, double *fcor, double *host_out3) {
  if (h && h->c.ode_kind) {
    set_error("dfr_diagnostics: a grid context is required (this one holds a test problem)");
    return DFR_E_INVAL;
  }
  if (!h || !q || !host_out3 || zeta == q || fcor == q || (zeta && zeta == fcor)) {
    set_error("invalid argument");
    return DFR_E_INVAL;
  }
  Ctx &c = h->c;
  int rc = launch_check_state(&c, q);
  if (!rc) rc = launch_diagnostics(&c, q, zeta, fcor);
  if (rc) return rc;
  DFR_HIP(hipMemcpyAsync(host_out3, c.d_diag + 3 * diag_blocks(&c), 3 * sizeof(double), hipMemcpyDeviceToHost,
                         c.stream));
  DFR_HIP(hipStreamSynchronize(c.stream));
  return latched_error(c);
}

int dfr_rhs(dfr_ctx *h, const double *q, double *dqdt) {
  if (!h || !q || !dqdt || q == dqdt) {
    set_error("invalid argument");
    return DFR_E_INVAL;
  }
  return launch_dfr(&h->c, q, nullptr, nullptr, nullptr, 0.0, false, false, dqdt, nullptr);
}

int dfr_jvp_complex_step(dfr_ctx *h, const double *q, const double *v, double eps, dfr_precision prec, double *jv) {
  if (h && h->c.ode_kind && prec != DFR_FP64) {
    set_error("dfr_jvp_complex_step: test problems take the exact Jacobian in FP64 (DFR_FP64)");
    return DFR_E_INVAL;
  }
  if (!h || !q || !v || !jv || jv == q || jv == v || !eps_prec_ok(eps, prec)) {
    set_error("dfr_jvp_complex_step: invalid argument (an FP32 form needs eps >= DFR_FP32_EPS_MIN)");
    return DFR_E_INVAL;
  }
  Ctx &c = h->c;
  if (prec != DFR_FP64) {
    int rc = launch_copy_to_f32(&c, c.n3, q, (float *)c.d_qf32);
    if (rc) return rc;
    return launch_dfr(&c, nullptr, (const float *)c.d_qf32, v, nullptr, eps, true, true, jv, nullptr);
  }
  return launch_dfr(&c, q, nullptr, v, nullptr, eps, true, false, jv, nullptr);
}

}  // extern "C"
