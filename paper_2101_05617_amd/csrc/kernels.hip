// HIP kernels for gfx950 (CDNA4, wave64): fused DFR right-hand side /
// complex-step Jacobian-vector product, the Krylov (KIOPS) vector kernels and
// the one-workgroup small matrix exponential.
//
// Method references (Gaudreault, Charron, Dallerit, Tokman, arXiv 2101.05617):
//   covariant shallow-water equations       Sec. 2, Eqs. (1)-(2); App. D Eq. (136)
//   1-D DFR and its tensor-product use      Sec. 3.1-3.2, Eqs. (7)-(14)
//   metric terms and Christoffel symbols    App. B, Eqs. (67)-(80)
//   Rusanov flux, wave speeds               Sec. 3.1; App. E, Eqs. (147)-(148)
//   panel-interface vector relations        App. C
//   complex-step J v                        Sec. 4, Eq. (28)
//   phi-combination by Krylov projection    Sec. 4, Eqs. (26), (29)
#include "dfrsw_internal.h"

#include <cmath>

namespace dfrsw {

int launch_dots_finalize(Ctx *c, int np, const ArnoldiArgs &ar);

// ---------------------------------------------------------------------------
// complex arithmetic on (re, im) pairs: the complex step evaluates F on
// z = q + i eps v; products keep the eps^2 terms (exact complex arithmetic)
template <typename T>
struct cx {
  T r, i;
};
template <typename T>
__device__ __forceinline__ cx<T> operator+(cx<T> a, cx<T> b) { return {a.r + b.r, a.i + b.i}; }
template <typename T>
__device__ __forceinline__ cx<T> operator-(cx<T> a, cx<T> b) { return {a.r - b.r, a.i - b.i}; }
template <typename T>
__device__ __forceinline__ cx<T> operator-(cx<T> a) { return {-a.r, -a.i}; }
template <typename T>
__device__ __forceinline__ cx<T> operator*(T s, cx<T> a) { return {s * a.r, s * a.i}; }
template <typename T>
__device__ __forceinline__ cx<T> cmul(cx<T> a, cx<T> b) {
  return {a.r * b.r - a.i * b.i, a.r * b.i + a.i * b.r};
}
template <typename T>
__device__ __forceinline__ T wave_sum(T v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

// block-wide sum over BLOCK threads in a fixed order (deterministic)
__device__ __forceinline__ double block_sum(double v, double *red) {
  v = wave_sum(v);
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  __syncthreads();
  if (lane == 0) red[wv] = v;
  __syncthreads();
  double s = 0.0;
  if (threadIdx.x == 0)
    for (int k = 0; k < (int)(blockDim.x >> 6); ++k) s += red[k];
  return s;   // valid in thread 0
}

// XCD-aware logical block: consecutive logical blocks land on the same XCD
// (the dispatcher places block b on XCD b % 8), so neighbouring elements
// share an L2.
__device__ __forceinline__ int64_t logical_block(int64_t nlogical) {
  const int64_t b = blockIdx.x, per = (gridDim.x + 7) / 8;
  int64_t lb = (b % 8) * per + b / 8;
  return lb < nlogical ? lb : -1;
}

// sum of partials[k*stride + off], k < np, in a fixed order; valid in thread 0
__device__ double reduce_partials(const double *partials, int np, int stride, int off, double *red) {
  double s = 0.0;
  for (int k = threadIdx.x; k < np; k += blockDim.x) s += partials[(int64_t)k * stride + off];
  return block_sum(s, red);
}

// ---------------------------------------------------------------------------
// Arnoldi finalisation after w = A~ v_j has been formed and its inner products
// with the last two top vectors reduced: classical Gram-Schmidt coefficients
// h_{j,j}, h_{j-1,j} (incomplete orthogonalisation, iop = 2) including the
// bottom blocks, and the bottom block of the new vector.
__device__ void arnoldi_dot_finalize(const ArnoldiArgs &ar, int np, double *red) {
  KDev *kd = ar.kd;
  const int j = ar.j, p = ar.p;
  const double d0 = reduce_partials(ar.partials, np, 2, 0, red);
  const double d1 = reduce_partials(ar.partials, np, 2, 1, red);
  if (threadIdx.x == 0) {
    const double *bj = kd->bot + j * MAX_P;
    double wb[MAX_P];
    for (int k = 0; k < p; ++k) wb[k] = (k + 1 < p) ? bj[k + 1] : 0.0;   // K v_j^bot (upper shift)
    double hjj = d0, hpj = d1;
    for (int k = 0; k < p; ++k) hjj += bj[k] * wb[k];
    const int ld = MAX_M + 2;
    kd->H[j * ld + j] = hjj;
    const bool two = (j >= 1) && (ar.vprev != nullptr);   // iop = 2
    if (two) {
      const double *bp = kd->bot + (j - 1) * MAX_P;
      for (int k = 0; k < p; ++k) hpj += bp[k] * wb[k];
      kd->H[(j - 1) * ld + j] = hpj;
    } else {
      hpj = 0.0;
    }
    double nb2 = 0.0;
    double *bn = kd->bot + (j + 1) * MAX_P;
    for (int k = 0; k < p; ++k) {
      double v = wb[k] - hjj * bj[k];
      if (two) v -= hpj * kd->bot[(j - 1) * MAX_P + k];
      bn[k] = v;
      nb2 += v * v;
    }
    kd->wnorm2_bot = nb2;
  }
}

// ---------------------------------------------------------------------------
// fast reciprocal and reciprocal square root: hardware estimate refined by
// Newton steps (two in FP64, the estimate being good to ~2^-23)
__device__ __forceinline__ double frcp(double x) {
  double r = __builtin_amdgcn_rcp(x);
  r = fma(fma(-x, r, 1.0), r, r);
  r = fma(fma(-x, r, 1.0), r, r);
  return r;
}
__device__ __forceinline__ float frcp(float x) { return __builtin_amdgcn_rcpf(x); }
__device__ __forceinline__ double frsqrt(double x) {
  double r = __builtin_amdgcn_rsq(x);
  const double h = 0.5 * x;
  r = fma(r, fma(-h * r, r, 0.5), r);
  r = fma(r, fma(-h * r, r, 0.5), r);
  return r;
}
__device__ __forceinline__ float frsqrt(float x) { return __builtin_amdgcn_rsqf(x); }

// Complex reciprocal and principal square root (Re > 0) on z = a + i b with
// |b| << |a|: the terms of relative size (b/a)^2 are dropped, which leaves the
// result of exact complex arithmetic unchanged in floating point whenever
// |b/a| < 2^-27 (FP64) / 2^-12 (FP32); the complex step keeps b = O(eps |v|).
template <typename T>
__device__ __forceinline__ cx<T> crcp1(cx<T> z) {
  const T r = frcp(z.r);
  return {r, -z.i * r * r};
}
template <typename T>
__device__ __forceinline__ cx<T> csqrt1(cx<T> z) {
  const T rs = frsqrt(z.r);
  return {z.r * rs, T(0.5) * z.i * rs};
}

// physical flux through an x^n = const face per unit sqrt(g)/a^2, and the
// Rusanov wave speed |u^n| + sqrt(h^nn g H), for Q = (H, H u^1, H u^2)
template <typename T>
__device__ __forceinline__ void side_flux1(const cx<T> Q[3], int n, T eta_1n, T eta_2n, T eta_nn, T gred,
                                           cx<T> f[3], cx<T> &c) {
  const cx<T> rH = crcp1(Q[0]);
  const cx<T> Mn = (n == 0) ? Q[1] : Q[2];
  const cx<T> un = cmul(Mn, rH);
  const cx<T> H2h = (T(0.5) * gred) * cmul(Q[0], Q[0]);
  f[0] = Mn;
  f[1] = cmul(Q[1], un) + eta_1n * H2h;
  f[2] = cmul(Q[2], un) + eta_2n * H2h;
  // |u^n| with the branch of the real evaluation: sign(Re H u^n), H > 0
  const cx<T> au = (Mn.r >= T(0)) ? un : -un;
  c = au + csqrt1((eta_nn * gred) * Q[0]);
}

// ---------------------------------------------------------------------------
// The fused DFR kernel.  A block takes `epb` consecutive elements of one
// element row of one panel (epb divides ne), one thread per GL node.
//  Phase 1 (per node): metric terms from 1-D tangent tables (App. B), nodal
//    fluxes (Eq. 136) and sources (Eq. 2) in complex arithmetic; state and
//    fluxes staged in LDS.
//  Phase 2a (per element, face, face point, field): own trace and neighbour
//    trace (Eq. 7 at +-1); the east/west neighbours inside the block come from
//    LDS, the others from global memory (L2-resident halo).
//  Phase 2b (per element, face, face point): App. C map of the neighbour's
//    momentum at panel edges, Rusanov common flux.
//  Phase 3 (per node): extended-point derivative of Eq. (12) in both
//    directions, sources, division by sqrt(g); output Re (F) or Im/eps (J v),
//    optionally with the Arnoldi epilogue (W-columns, partial inner products).
template <int NS, typename T>
struct DfrSmem {
  static constexpr int NN = NS * NS;
  static constexpr int EPB = BLOCK / NN;
  cx<T> F1[EPB][3][NN];
  cx<T> F2[EPB][3][NN];
  cx<T> Z[EPB][3][NN];
  cx<T> Tr[EPB][4][3][NS];      // own traces; overwritten by the common fluxes
  cx<T> Nb[EPB][4][3][NS];      // neighbour traces
  T D[NS][NS + 2];
  T lm[NS], lp[NS];
  double red[BLOCK / 64];
};

template <int NS, typename T, typename TQ, bool CS>
__global__ __launch_bounds__(BLOCK) void dfr_kernel(const GridArgs g, const Ops1D ops, const int epb,
                                                     const TQ *__restrict__ q, const double *__restrict__ v,
                                                     const double *__restrict__ vscale, double eps,
                                                     double *__restrict__ out, const ArnoldiArgs ar) {
  using S = DfrSmem<NS, T>;
  constexpr int NN = S::NN;
  __shared__ S sm;

  if (ar.on && ar.kd->happy) return;   // uniform: the sub-step ended in a happy breakdown

  const int tid = threadIdx.x;
  const int ne = g.ne;
  const int N = (int)g.n;
  const int bpr = ne / epb;            // blocks per element row
  const int nlog = 6 * ne * bpr;
  const int lb = (int)logical_block(nlog);
  if (lb < 0) {                        // uniform: padding block of the XCD mapping
    if (ar.on && tid == 0) {
      ar.partials[blockIdx.x * 2 + 0] = 0.0;
      ar.partials[blockIdx.x * 2 + 1] = 0.0;
    }
    return;
  }
  const int row = lb / bpr;            // panel * ne + element row
  const int p = row / ne, ej = row - p * ne;
  const int ei0 = (lb - row * bpr) * epb;
  const int ebase = row * ne + ei0;    // first element of the block

  for (int k = tid; k < NS * (NS + 2); k += BLOCK) sm.D[k / (NS + 2)][k % (NS + 2)] = (T)ops.Dt[k / (NS + 2)][k % (NS + 2)];
  if (tid < NS) {
    sm.lm[tid] = (T)ops.lm[tid];
    sm.lp[tid] = (T)ops.lp[tid];
  }

  const int s = tid / NN, node = tid - s * NN, nj = node / NS, ni = node - nj * NS;
  const bool active = s < epb;
  const int ei = ei0 + s;
  const int gidx = (ebase + s) * NN + node;
  const T gred = (T)g.g_red;
  const double vs = (CS && vscale) ? *vscale : 1.0;
  const double eps_vs = eps * vs;

  cx<T> src1 = {T(0), T(0)}, src2 = {T(0), T(0)};
  T rs = T(0);
  double vtrue[3] = {0.0, 0.0, 0.0};

  // ---- phase 1
  if (active) {
    const Tan3 tx = g.tnode[ei * NS + ni], ty = g.tnode[ej * NS + nj];
    const T X = (T)tx.x, ax = (T)tx.ax, rax = (T)tx.rax;
    const T Y = (T)ty.x, ay = (T)ty.ax, ray = (T)ty.rax;
    const T d2 = ax + Y * Y;
    const T rd = frsqrt(d2);
    const T rd2 = rd * rd;
    const T sg = ax * ay * rd2 * rd;          // sqrt(g)/a^2, Eq. (70)
    rs = d2 * (d2 * rd) * rax * ray;          // a^2/sqrt(g)
    const T e11 = d2 * rax, e22 = d2 * ray, e12 = X * Y * e11 * ray;   // a^2 h^ij, Eqs. (67)-(69)
    const T cf = (T)g.omega * ((T)g.cA[p] + X * (T)g.cB[p] + Y * (T)g.cC[p]) * rd2;
    const T xy = X * Y;
    const T G101 = xy * cf, G102 = -ay * cf, G201 = ax * cf, G202 = -xy * cf;   // Eqs. (71)-(74)
    const T G111 = T(2) * xy * Y * rd2, G112 = -Y * ay * rd2;                  // Eqs. (75)-(76)
    const T G212 = -X * ax * rd2, G222 = T(2) * xy * X * rd2;                  // Eqs. (79)-(80)

    cx<T> Qz[3];
#pragma unroll
    for (int f = 0; f < 3; ++f) {
      const T qr = (T)q[f * N + gidx];
      T qi = T(0);
      if (CS) {
        const double vv = vs * v[f * N + gidx];
        vtrue[f] = vv;
        qi = (T)(eps * vv);
      }
      Qz[f] = {qr, qi};
      sm.Z[s][f][node] = Qz[f];
    }
    const cx<T> H = Qz[0], M1 = Qz[1], M2 = Qz[2];
    if (!(H.r > T(0))) atomicOr(g.err_flag, 2);
    const cx<T> rH = crcp1(H);
    const cx<T> u1 = cmul(M1, rH), u2 = cmul(M2, rH);
    const cx<T> H2h = (T(0.5) * gred) * cmul(H, H);
    const cx<T> m11 = cmul(M1, u1), m12 = cmul(M1, u2), m22 = cmul(M2, u2);
    const cx<T> f12 = m12 + e12 * H2h;
    sm.F1[s][0][node] = sg * M1;
    sm.F1[s][1][node] = sg * (m11 + e11 * H2h);
    sm.F1[s][2][node] = sg * f12;
    sm.F2[s][0][node] = sg * M2;
    sm.F2[s][1][node] = sg * f12;
    sm.F2[s][2][node] = sg * (m22 + e22 * H2h);
    // sources per unit sqrt(g): Coriolis -2 Gamma^i_0j H u^j, metric -Gamma^i_jk H u^j u^k
    // (the h^jk Gamma^i_jk term vanishes identically on the cubed sphere, App. B)
    src1 = -(T(2) * (G101 * M1 + G102 * M2) + (G111 * m11 + (T(2) * G112) * m12));
    src2 = -(T(2) * (G201 * M1 + G202 * M2) + ((T(2) * G212) * m12 + G222 * m22));
    if (g.orog) {
      src1 = src1 - (T)g.orog[gidx] * H;
      src2 = src2 - (T)g.orog[N + gidx] * H;
    }
  }
  __syncthreads();

  // ---- phase 2a: traces, task = ((f * epb + s) * 4 + face) * NS + t
  const int ntr = 3 * epb * 4 * NS;
  for (int task = tid; task < ntr; task += BLOCK) {
    const int t = task % NS;
    const int r1 = task / NS;
    const int face = r1 & 3;
    const int r2 = r1 >> 2;
    const int fs = r2 % epb, f = r2 / epb;
    const int fei = ei0 + fs;
    // own trace along the line normal to the face
    const T *wl = (face == 0 || face == 2) ? sm.lm : sm.lp;
    cx<T> acc = {T(0), T(0)};
#pragma unroll
    for (int k = 0; k < NS; ++k) acc = acc + wl[k] * sm.Z[fs][f][(face < 2) ? (t * NS + k) : (k * NS + t)];
    sm.Tr[fs][face][f][t] = acc;
    // neighbour trace
    cx<T> nb = {T(0), T(0)};
    if (face == 0 && fs > 0) {
#pragma unroll
      for (int k = 0; k < NS; ++k) nb = nb + sm.lp[k] * sm.Z[fs - 1][f][t * NS + k];
    } else if (face == 1 && fs < epb - 1) {
#pragma unroll
      for (int k = 0; k < NS; ++k) nb = nb + sm.lm[k] * sm.Z[fs + 1][f][t * NS + k];
    } else {
      int q_p = p, q_ej = ej, q_ei = fei, q_face, q_t = t;
      bool edge = false;
      if (face == 0) { if (fei > 0) { q_ei = fei - 1; q_face = 1; } else edge = true; }
      else if (face == 1) { if (fei < ne - 1) { q_ei = fei + 1; q_face = 0; } else edge = true; }
      else if (face == 2) { if (ej > 0) { q_ej = ej - 1; q_face = 3; } else edge = true; }
      else { if (ej < ne - 1) { q_ej = ej + 1; q_face = 2; } else edge = true; }
      if (edge) {
        const int along = (face < 2) ? ej : fei;
        q_p = g.nb_q[p][face];
        q_face = g.nb_e[p][face];
        const int rev = g.nb_rev[p][face];
        const int qa = rev ? ne - 1 - along : along;
        q_t = rev ? NS - 1 - t : t;
        if (q_face == 0) { q_ei = 0; q_ej = qa; }
        else if (q_face == 1) { q_ei = ne - 1; q_ej = qa; }
        else if (q_face == 2) { q_ej = 0; q_ei = qa; }
        else { q_ej = ne - 1; q_ei = qa; }
      }
      const T *wq = (q_face == 0 || q_face == 2) ? sm.lm : sm.lp;
      const int first = f * N + ((q_p * ne + q_ej) * ne + q_ei) * NN + ((q_face < 2) ? q_t * NS : q_t);
      const int stride = (q_face < 2) ? 1 : NS;
#pragma unroll
      for (int k = 0; k < NS; ++k) {
        const int id = first + k * stride;
        T zi = T(0);
        if (CS) zi = (T)(eps_vs * v[id]);
        nb = nb + wq[k] * cx<T>{(T)q[id], zi};
      }
    }
    sm.Nb[fs][face][f][t] = nb;
  }
  __syncthreads();

  // ---- phase 2b: common fluxes, task = (s * 4 + face) * NS + t
  const int nfl = epb * 4 * NS;
  for (int task = tid; task < nfl; task += BLOCK) {
    const int t = task % NS;
    const int r1 = task / NS;
    const int face = r1 & 3, fs = r1 >> 2;
    const int fei = ei0 + fs;
    cx<T> own[3], nb[3];
#pragma unroll
    for (int f = 0; f < 3; ++f) {
      own[f] = sm.Tr[fs][face][f][t];
      nb[f] = sm.Nb[fs][face][f][t];
    }
    const bool edge = (face == 0 && fei == 0) || (face == 1 && fei == ne - 1) || (face == 2 && ej == 0) ||
                      (face == 3 && ej == ne - 1);
    if (edge) {
      const int along = (face < 2) ? ej : fei;
      const double *M = g.xform + (((p * 4 + face) * ne + along) * NS + t) * 4;
      const T m00 = (T)M[0], m01 = (T)M[1], m10 = (T)M[2], m11 = (T)M[3];
      const cx<T> a1 = m00 * nb[1] + m01 * nb[2];
      const cx<T> a2 = m10 * nb[1] + m11 * nb[2];
      nb[1] = a1;
      nb[2] = a2;
    }
    // metric at the face point
    T X, Y, ax, ay, rax, ray;
    if (face < 2) {
      const double xe = g.tedge[fei + (face == 1)];
      const Tan3 ty = g.tnode[ej * NS + t];
      X = (T)xe; ax = T(1) + X * X; rax = frcp(ax);
      Y = (T)ty.x; ay = (T)ty.ax; ray = (T)ty.rax;
    } else {
      const double ye = g.tedge[ej + (face == 3)];
      const Tan3 tx = g.tnode[fei * NS + t];
      X = (T)tx.x; ax = (T)tx.ax; rax = (T)tx.rax;
      Y = (T)ye; ay = T(1) + Y * Y; ray = frcp(ay);
    }
    const T d2 = ax + Y * Y;
    const T rd = frsqrt(d2);
    const T sg = ax * ay * rd * rd * rd;
    const int n = (face < 2) ? 0 : 1;
    const T e11 = d2 * rax, e22 = d2 * ray, e12 = X * Y * e11 * ray;
    const T eta1n = n == 0 ? e11 : e12, eta2n = n == 0 ? e12 : e22, etann = n == 0 ? e11 : e22;
    const bool own_low = (face == 1 || face == 3);
    cx<T> fL[3], fR[3], cL, cR;
    const cx<T> *QL = own_low ? own : nb;
    const cx<T> *QR = own_low ? nb : own;
    side_flux1(QL, n, eta1n, eta2n, etann, gred, fL, cL);
    side_flux1(QR, n, eta1n, eta2n, etann, gred, fR, cR);
    const cx<T> lam = (cL.r >= cR.r) ? cL : cR;
#pragma unroll
    for (int f = 0; f < 3; ++f) {
      const cx<T> F = T(0.5) * (fL[f] + fR[f]) - T(0.5) * cmul(lam, QR[f] - QL[f]);
      sm.Tr[fs][face][f][t] = sg * F;
    }
  }
  __syncthreads();

  // ---- phase 3: derivative of the continuous flux polynomial (Eqs. 12, 14)
  double w[3] = {0.0, 0.0, 0.0};
  if (active) {
    const T scale = -(T)g.two_over_delta * rs;
    const T invE = CS ? (T)(1.0 / eps) : T(1);
#pragma unroll
    for (int f = 0; f < 3; ++f) {
      cx<T> d1 = sm.D[ni][0] * sm.Tr[s][0][f][nj] + sm.D[ni][NS + 1] * sm.Tr[s][1][f][nj];
      cx<T> d2 = sm.D[nj][0] * sm.Tr[s][2][f][ni] + sm.D[nj][NS + 1] * sm.Tr[s][3][f][ni];
#pragma unroll
      for (int k = 0; k < NS; ++k) {
        d1 = d1 + sm.D[ni][k + 1] * sm.F1[s][f][nj * NS + k];
        d2 = d2 + sm.D[nj][k + 1] * sm.F2[s][f][k * NS + ni];
      }
      cx<T> r = scale * (d1 + d2);
      if (f == 1) r = r + src1;
      if (f == 2) r = r + src2;
      w[f] = CS ? (double)(r.i * invE) : (double)r.r;
    }
    if (!ar.on) {
#pragma unroll
      for (int f = 0; f < 3; ++f) out[f * N + gidx] = w[f];
    }
  }
  if (!ar.on) return;

  // ---- Arnoldi epilogue: w += sum_k W_k c_k ; partial <v_j, w>, <v_{j-1}, w>
  double d0 = 0.0, d1 = 0.0;
  if (active) {
    const double *c = ar.kd->bot + ar.j * MAX_P;
#pragma unroll
    for (int f = 0; f < 3; ++f) {
      const int id = f * N + gidx;
      double acc = w[f];
      for (int k = 0; k < ar.p; ++k) acc += ar.W[k][id] * c[k];
      out[id] = acc;
      d0 += acc * vtrue[f];
      if (ar.vprev) d1 += acc * ar.vprev[id];
    }
  }
  const double b0 = block_sum(d0, sm.red);
  const double b1 = block_sum(d1, sm.red);
  if (tid == 0) {
    ar.partials[blockIdx.x * 2 + 0] = b0;
    ar.partials[blockIdx.x * 2 + 1] = b1;
  }
}

// one block: reduce the J v kernel's partial inner products (fixed order)
__global__ __launch_bounds__(BLOCK) void arnoldi_dots_finalize_kernel(int np, const ArnoldiArgs ar) {
  __shared__ double red[BLOCK / 64];
  if (ar.kd->happy) return;
  arnoldi_dot_finalize(ar, np, red);
}

// first Arnoldi step of a sub-step whose top block is identically zero:
// w = W c (no J v), same epilogue
__global__ __launch_bounds__(BLOCK) void arnoldi_first_kernel(int64_t n3, const ArnoldiArgs ar, double *out) {
  if (ar.kd->happy) return;
  const double *c = ar.kd->bot + ar.j * MAX_P;
  for (int64_t i = (int64_t)blockIdx.x * BLOCK + threadIdx.x; i < n3; i += (int64_t)gridDim.x * BLOCK) {
    double acc = 0.0;
    for (int k = 0; k < ar.p; ++k) acc += ar.W[k][i] * c[k];
    out[i] = acc;
  }
  // the top block of v_j is zero, so both inner products vanish
  if (threadIdx.x == 0) {
    ar.partials[blockIdx.x * 2 + 0] = 0.0;
    ar.partials[blockIdx.x * 2 + 1] = 0.0;
  }
}

// Gram-Schmidt update and normalisation:
//   w <- w - h_jj sigma_j v~_j - h_{j-1,j} v_{j-1};  v_j <- sigma_j v~_j (stored normalised)
//   h_{j+1,j} = ||w|| (top and bottom), sigma_{j+1} = 1/h_{j+1,j}; happy breakdown if < tol
__global__ __launch_bounds__(BLOCK) void arnoldi_update_kernel(int64_t n3, int j, double *w, double *vj,
                                                               const double *vprev, double *partials, KDev *kd) {
  __shared__ double red[BLOCK / 64];
  if (kd->happy) return;
  const int ld = MAX_M + 2;
  const double hjj = kd->H[j * ld + j];
  const double hpj = (j >= 1 && vprev) ? kd->H[(j - 1) * ld + j] : 0.0;
  const double sj = kd->sigma[j];
  double acc = 0.0;
  for (int64_t i = (int64_t)blockIdx.x * BLOCK + threadIdx.x; i < n3; i += (int64_t)gridDim.x * BLOCK) {
    const double vv = sj * vj[i];
    double x = w[i] - hjj * vv;
    if (vprev) x -= hpj * vprev[i];
    w[i] = x;
    vj[i] = vv;
    acc += x * x;
  }
  const double b = block_sum(acc, red);
  if (threadIdx.x == 0) partials[blockIdx.x * 2] = b;
}

// one block: h_{j+1,j} = ||w|| (top and bottom blocks), sigma_{j+1} = 1/h_{j+1,j},
// normalised bottom block; happy breakdown if the norm is below tol
__global__ __launch_bounds__(BLOCK) void arnoldi_norm_finalize_kernel(int np, int j, int p, const double *partials,
                                                                      KDev *kd, double tol) {
  __shared__ double red[BLOCK / 64];
  if (kd->happy) return;
  const double s = reduce_partials(partials, np, 2, 0, red);
  if (threadIdx.x == 0) {
    const int ld = MAX_M + 2;
    const double nrm = sqrt(s + kd->wnorm2_bot);
    kd->sigma[j] = 1.0;
    kd->J = j + 1;
    if (nrm < tol) {
      kd->happy = 1;
    } else {
      kd->H[(j + 1) * ld + j] = nrm;
      kd->sigma[j + 1] = 1.0 / nrm;
      double *bn = kd->bot + (j + 1) * MAX_P;
      for (int k = 0; k < p; ++k) bn[k] /= nrm;
    }
  }
}

struct Ybot {
  double y[MAX_P];
};

// start of a sub-step: v~_0 = x (copied), partial ||x||^2
__global__ __launch_bounds__(BLOCK) void arnoldi_start_kernel(int64_t n3, const double *x, double *v0,
                                                              double *partials) {
  __shared__ double red[BLOCK / 64];
  double acc = 0.0;
  for (int64_t i = (int64_t)blockIdx.x * BLOCK + threadIdx.x; i < n3; i += (int64_t)gridDim.x * BLOCK) {
    const double xv = x[i];
    v0[i] = xv;
    acc += xv * xv;
  }
  const double b = block_sum(acc, red);
  if (threadIdx.x == 0) partials[blockIdx.x * 2] = b;
}

// one block: beta = ||[x; mu y(t)]||, sigma_0 = 1/beta, bottom block mu y(t)/beta,
// Hessenberg cleared
__global__ __launch_bounds__(BLOCK) void arnoldi_start_finalize_kernel(int np, int p, const Ybot yb,
                                                                       const double *partials, KDev *kd) {
  __shared__ double red[BLOCK / 64];
  const double s = reduce_partials(partials, np, 2, 0, red);
  const int ld = MAX_M + 2;
  for (int k = threadIdx.x; k < ld * ld; k += BLOCK) kd->H[k] = 0.0;
  if (threadIdx.x == 0) {
    double s2 = s;
    for (int k = 0; k < p; ++k) s2 += yb.y[k] * yb.y[k];
    const double beta = sqrt(s2);
    kd->beta = beta;
    kd->sigma[0] = 1.0 / beta;
    for (int k = 0; k < p; ++k) kd->bot[k] = yb.y[k] / beta;
    kd->happy = 0;
    kd->J = 0;
  }
}

// accepted sub-step: x = beta * sum_{k<J} v_k E[k][0]
__global__ __launch_bounds__(BLOCK) void arnoldi_combine_kernel(int64_t n3, const double *V, int64_t ldv, const KDev *kd,
                                                                double *x) {
  const int J = kd->J;
  const double beta = kd->beta;
  for (int64_t i = (int64_t)blockIdx.x * BLOCK + threadIdx.x; i < n3; i += (int64_t)gridDim.x * BLOCK) {
    double acc = 0.0;
    for (int k = 0; k < J; ++k) acc += V[k * ldv + i] * kd->E0[k];
    x[i] = beta * acc;
  }
}

// ---------------------------------------------------------------------------
// exp(tau H_aug), H_aug = [[H_J, e_1], [0, 0]] ((J+1) x (J+1)), in one
// workgroup: scaling to ||.||_1 <= 1, Taylor polynomial of degree 18 in
// Paterson-Stockmeyer form (blocks of A^2), then repeated squaring.  The
// truncation error for ||A||_1 <= 1 is below sum_{k>=19} 1/k! < 1e-17.
// C = A B for n x n row-major matrices in LDS with leading dimension ld
// (ld = n rounded up to a multiple of 4, padding rows/columns zero): each
// thread accumulates a 4 x 4 tile in registers, so every LDS value read feeds
// four FMAs.
__device__ void lds_matmul(const double *A, const double *B, double *C, int ld) {
  const int nt = ld / 4;
  for (int tile = threadIdx.x; tile < nt * nt; tile += blockDim.x) {
    const int r0 = (tile / nt) * 4, c0 = (tile % nt) * 4;
    double acc[4][4];
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
      for (int j = 0; j < 4; ++j) acc[i][j] = 0.0;
    for (int k = 0; k < ld; ++k) {
      const double a0 = A[(r0 + 0) * ld + k], a1 = A[(r0 + 1) * ld + k];
      const double a2 = A[(r0 + 2) * ld + k], a3 = A[(r0 + 3) * ld + k];
      const double b0 = B[k * ld + c0 + 0], b1 = B[k * ld + c0 + 1];
      const double b2 = B[k * ld + c0 + 2], b3 = B[k * ld + c0 + 3];
      acc[0][0] += a0 * b0; acc[0][1] += a0 * b1; acc[0][2] += a0 * b2; acc[0][3] += a0 * b3;
      acc[1][0] += a1 * b0; acc[1][1] += a1 * b1; acc[1][2] += a1 * b2; acc[1][3] += a1 * b3;
      acc[2][0] += a2 * b0; acc[2][1] += a2 * b1; acc[2][2] += a2 * b2; acc[2][3] += a2 * b3;
      acc[3][0] += a3 * b0; acc[3][1] += a3 * b1; acc[3][2] += a3 * b2; acc[3][3] += a3 * b3;
    }
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
      for (int j = 0; j < 4; ++j) C[(r0 + i) * ld + c0 + j] = acc[i][j];
  }
}

__global__ __launch_bounds__(BLOCK) void expm_kernel(KDev *kd, double tau, KHost *res) {
  extern __shared__ double lds[];
  __shared__ double red[BLOCK / 64];
  __shared__ double cnorm;
  const int J = kd->J;
  const int n = J + 1;
  const int ld = (n + 3) & ~3;          // padded to whole 4 x 4 tiles (zero padding)
  const int nn = ld * ld;
  double *A = lds, *A2 = lds + nn, *P = lds + 2 * nn, *Q = lds + 3 * nn;
  const int hld = MAX_M + 2;
  for (int idx = threadIdx.x; idx < nn; idx += blockDim.x) {
    const int i = idx / ld, j = idx - i * ld;
    double v = 0.0;
    if (i < J && j < J) v = tau * kd->H[i * hld + j];
    if (i == 0 && j == J) v = tau;
    A[idx] = v;
  }
  __syncthreads();
  // 1-norm (max column sum)
  double cm = 0.0;
  for (int j = threadIdx.x; j < n; j += blockDim.x) {
    double cs = 0.0;
    for (int i = 0; i < n; ++i) cs += fabs(A[i * ld + j]);
    cm = fmax(cm, cs);
  }
  {
    double v = cm;
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o, 64));
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
    __syncthreads();
    if (threadIdx.x == 0) {
      double m = 0.0;
      for (int k = 0; k < (int)(blockDim.x >> 6); ++k) m = fmax(m, red[k]);
      cnorm = m;
    }
    __syncthreads();
  }
  int sq = 0;
  if (cnorm > 1.0) sq = (int)ceil(log2(cnorm));
  if (sq > 0) {
    const double sc = ldexp(1.0, -sq);
    for (int idx = threadIdx.x; idx < nn; idx += blockDim.x) A[idx] *= sc;
    __syncthreads();
  }
  lds_matmul(A, A, A2, ld);
  __syncthreads();
  // c_k = 1/k!, k = 0..19 (c_19 = 0 keeps the degree at 18)
  double c[20];
  c[0] = 1.0;
  for (int k = 1; k < 19; ++k) c[k] = c[k - 1] / k;
  c[19] = 0.0;
  // P = c18 I + c19 A  (padding stays zero: only the leading n x n block is set)
  for (int idx = threadIdx.x; idx < nn; idx += blockDim.x) {
    const int i = idx / ld, j = idx - i * ld;
    P[idx] = ((i == j && i < n) ? c[18] : 0.0) + c[19] * A[idx];
  }
  __syncthreads();
  for (int k = 8; k >= 0; --k) {
    lds_matmul(A2, P, Q, ld);
    __syncthreads();
    for (int idx = threadIdx.x; idx < nn; idx += blockDim.x) {
      const int i = idx / ld, j = idx - i * ld;
      P[idx] = Q[idx] + ((i == j && i < n) ? c[2 * k] : 0.0) + c[2 * k + 1] * A[idx];
    }
    __syncthreads();
  }
  for (int r = 0; r < sq; ++r) {
    lds_matmul(P, P, Q, ld);
    __syncthreads();
    double *t = P;
    P = Q;
    Q = t;
  }
  for (int k = threadIdx.x; k < J; k += blockDim.x) kd->E0[k] = P[k * ld];
  if (threadIdx.x == 0) {
    const double eJ = P[(J - 1) * ld + J];
    const double hl = kd->happy ? 0.0 : kd->H[J * hld + (J - 1)];
    kd->eJ = eJ;
    kd->hlast = hl;
    kd->err = kd->beta * hl * fabs(eJ);
    res->err = kd->err;
    res->beta = kd->beta;
    res->hlast = hl;
    res->eJ = eJ;
    res->J = J;
    res->happy = kd->happy;
  }
}

// ---------------------------------------------------------------------------
// vector helpers
__global__ __launch_bounds__(BLOCK) void axpby_kernel(int64_t n, double a, const double *x, double b, const double *y,
                                                      double *out) {
  for (int64_t i = (int64_t)blockIdx.x * BLOCK + threadIdx.x; i < n; i += (int64_t)gridDim.x * BLOCK) {
    double r = a * x[i];
    if (y) r += b * y[i];
    out[i] = r;
  }
}

__global__ __launch_bounds__(BLOCK) void to_f32_kernel(int64_t n, const double *x, float *y) {
  for (int64_t i = (int64_t)blockIdx.x * BLOCK + threadIdx.x; i < n; i += (int64_t)gridDim.x * BLOCK) y[i] = (float)x[i];
}

__global__ __launch_bounds__(BLOCK) void check_state_kernel(int64_t n, const double *q, int *err) {
  int bad = 0;
  for (int64_t i = (int64_t)blockIdx.x * BLOCK + threadIdx.x; i < 3 * n; i += (int64_t)gridDim.x * BLOCK) {
    const double x = q[i];
    if (!isfinite(x)) bad |= 1;
    if (i < n && !(x > 0.0)) bad |= 2;
  }
  if (bad) atomicOr(err, bad);
}

// ---------------------------------------------------------------------------
// launchers
static inline int grid_for(int64_t n) {
  int64_t b = (n + BLOCK - 1) / BLOCK;
  if (b > 8192) b = 8192;
  if (b < 1) b = 1;
  return (int)b;
}

// elements per block: the largest divisor of ne that fits BLOCK threads
int dfr_epb(const Ctx *c) {
  const int cap = BLOCK / (c->ns * c->ns);
  int e = cap < c->ne ? cap : c->ne;
  while (c->ne % e) --e;
  return e;
}

int64_t dfr_grid_blocks(const Ctx *c) {
  const int64_t nlog = 6LL * c->ne * (c->ne / dfr_epb(c));
  return ((nlog + 7) / 8) * 8;
}

template <int NS, typename T, typename TQ, bool CS>
static void launch_ns(Ctx *c, const TQ *q, const double *v, const double *vscale, double eps, double *out,
                      const ArnoldiArgs &ar) {
  const int epb = dfr_epb(c);
  const int64_t nb = dfr_grid_blocks(c);
  tbegin(c, !CS ? DFR_K_RHS : (ar.on ? DFR_K_JV_ARNOLDI : DFR_K_JV));
  hipLaunchKernelGGL((dfr_kernel<NS, T, TQ, CS>), dim3((unsigned)nb), dim3(BLOCK), 0, c->stream, c->ga, c->ops, epb,
                     q, v, vscale, eps, out, ar);
  tend(c);
  if (ar.on) launch_dots_finalize(c, (int)nb, ar);
}

template <typename T, typename TQ, bool CS>
static int dispatch_ns(Ctx *c, const TQ *q, const double *v, const double *vscale, double eps, double *out,
                       const ArnoldiArgs &ar) {
  switch (c->ns) {
    case 2: launch_ns<2, T, TQ, CS>(c, q, v, vscale, eps, out, ar); break;
    case 3: launch_ns<3, T, TQ, CS>(c, q, v, vscale, eps, out, ar); break;
    case 4: launch_ns<4, T, TQ, CS>(c, q, v, vscale, eps, out, ar); break;
    case 5: launch_ns<5, T, TQ, CS>(c, q, v, vscale, eps, out, ar); break;
    case 6: launch_ns<6, T, TQ, CS>(c, q, v, vscale, eps, out, ar); break;
    case 7: launch_ns<7, T, TQ, CS>(c, q, v, vscale, eps, out, ar); break;
    case 8: launch_ns<8, T, TQ, CS>(c, q, v, vscale, eps, out, ar); break;
    default: set_error("unsupported number of GL points"); return DFR_E_INVAL;
  }
  DFR_HIP(hipGetLastError());
  return DFR_OK;
}

int launch_dfr(Ctx *c, const double *q, const float *q32, const double *v, const double *vscale, double eps,
               bool complex_step, bool fp32, double *out, const ArnoldiArgs *ar) {
  ArnoldiArgs none{};
  const ArnoldiArgs &a = ar ? *ar : none;
  if (!complex_step) return dispatch_ns<double, double, false>(c, q, nullptr, nullptr, 0.0, out, a);
  if (fp32) return dispatch_ns<float, float, true>(c, q32, v, vscale, eps, out, a);
  return dispatch_ns<double, double, true>(c, q, v, vscale, eps, out, a);
}

int launch_arnoldi_first(Ctx *c, const ArnoldiArgs &ar, double *out) {
  const int64_t n3 = 3 * c->n;
  tbegin(c, DFR_K_OTHER);
  hipLaunchKernelGGL(arnoldi_first_kernel, dim3(grid_for(n3)), dim3(BLOCK), 0, c->stream, n3, ar, out);
  tend(c);
  DFR_HIP(hipGetLastError());
  return launch_dots_finalize(c, grid_for(n3), ar);
}

int launch_dots_finalize(Ctx *c, int np, const ArnoldiArgs &ar) {
  tbegin(c, DFR_K_FINALIZE);
  hipLaunchKernelGGL(arnoldi_dots_finalize_kernel, dim3(1), dim3(BLOCK), 0, c->stream, np, ar);
  tend(c);
  DFR_HIP(hipGetLastError());
  return DFR_OK;
}

int launch_update(Ctx *c, int j, double *w, double *vj, const double *vprev, double tol) {
  const int64_t n3 = 3 * c->n;
  tbegin(c, DFR_K_UPDATE);
  hipLaunchKernelGGL(arnoldi_update_kernel, dim3(grid_for(n3)), dim3(BLOCK), 0, c->stream, n3, j, w, vj, vprev,
                     c->d_partials, c->d_kd);
  tend(c);
  DFR_HIP(hipGetLastError());
  tbegin(c, DFR_K_FINALIZE);
  hipLaunchKernelGGL(arnoldi_norm_finalize_kernel, dim3(1), dim3(BLOCK), 0, c->stream, grid_for(n3), j, c->kiops_p,
                     c->d_partials, c->d_kd, tol);
  tend(c);
  DFR_HIP(hipGetLastError());
  return DFR_OK;
}

int launch_start(Ctx *c, const double *x, double *v0, int p, const double *ybot) {
  const int64_t n3 = 3 * c->n;
  Ybot yb{};
  for (int k = 0; k < p; ++k) yb.y[k] = ybot[k];
  tbegin(c, DFR_K_OTHER);
  hipLaunchKernelGGL(arnoldi_start_kernel, dim3(grid_for(n3)), dim3(BLOCK), 0, c->stream, n3, x, v0, c->d_partials);
  tend(c);
  DFR_HIP(hipGetLastError());
  tbegin(c, DFR_K_FINALIZE);
  hipLaunchKernelGGL(arnoldi_start_finalize_kernel, dim3(1), dim3(BLOCK), 0, c->stream, grid_for(n3), p, yb,
                     c->d_partials, c->d_kd);
  tend(c);
  DFR_HIP(hipGetLastError());
  return DFR_OK;
}

int launch_combine(Ctx *c, double *x) {
  const int64_t n3 = 3 * c->n;
  tbegin(c, DFR_K_OTHER);
  hipLaunchKernelGGL(arnoldi_combine_kernel, dim3(grid_for(n3)), dim3(BLOCK), 0, c->stream, n3, c->d_V, n3, c->d_kd, x);
  tend(c);
  DFR_HIP(hipGetLastError());
  return DFR_OK;
}

int launch_expm(Ctx *c, double tau) {
  const int n = ((c->kiops_mmax + 1) + 3) & ~3;
  const size_t lds = (size_t)4 * n * n * sizeof(double);
  tbegin(c, DFR_K_EXPM);
  hipLaunchKernelGGL(expm_kernel, dim3(1), dim3(BLOCK), lds, c->stream, c->d_kd, tau, (KHost *)c->d_expm_scratch);
  tend(c);
  DFR_HIP(hipGetLastError());
  return DFR_OK;
}

int launch_axpby(Ctx *c, int64_t n, double a, const double *x, double b, const double *y, double *out) {
  tbegin(c, DFR_K_OTHER);
  hipLaunchKernelGGL(axpby_kernel, dim3(grid_for(n)), dim3(BLOCK), 0, c->stream, n, a, x, b, y, out);
  tend(c);
  DFR_HIP(hipGetLastError());
  return DFR_OK;
}

int launch_copy_to_f32(Ctx *c, int64_t n, const double *x, float *y) {
  tbegin(c, DFR_K_OTHER);
  hipLaunchKernelGGL(to_f32_kernel, dim3(grid_for(n)), dim3(BLOCK), 0, c->stream, n, x, y);
  tend(c);
  DFR_HIP(hipGetLastError());
  return DFR_OK;
}

int launch_check_state(Ctx *c, const double *q) {
  tbegin(c, DFR_K_OTHER);
  hipLaunchKernelGGL(check_state_kernel, dim3(grid_for(3 * c->n)), dim3(BLOCK), 0, c->stream, c->n, q, c->d_err);
  tend(c);
  DFR_HIP(hipGetLastError());
  return DFR_OK;
}

int set_expm_lds_limit(int n) {
  n = (n + 3) & ~3;
  const size_t lds = (size_t)4 * n * n * sizeof(double);
  DFR_HIP(hipFuncSetAttribute((const void *)expm_kernel, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
  return DFR_OK;
}

}  // namespace dfrsw
