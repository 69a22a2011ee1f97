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

#include <algorithm>
#include <cmath>

namespace dfrsw {

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

// Sum of pin[k*stride + off], k < np, in an order that does not depend on the
// workgroup size: 256 virtual lanes take every 256th value; the first wave
// (always 64 lanes) adds them in a fixed pattern and a fixed butterfly.  Every
// workgroup of every kernel gets the identical value.  red: 256 doubles of
// LDS.  Call from all threads of the workgroup; valid in every thread.
__device__ double reduce_fixed(const double *pin, int np, int stride, int off, double *red) {
  __syncthreads();
  for (int l = threadIdx.x; l < 256; l += blockDim.x) {
    double s = 0.0;
    for (int k = l; k < np; k += 256) s += pin[(int64_t)k * stride + off];
    red[l] = s;
  }
  __syncthreads();
  if (threadIdx.x < 64) {
    const int l = threadIdx.x;
    double v = (red[l] + red[l + 64]) + (red[l + 128] + red[l + 192]);
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    if (l == 0) red[0] = v;
  }
  __syncthreads();
  const double r = red[0];
  __syncthreads();
  return r;
}

// Arnoldi prologue: finalise the norm of the vector v_j (start vector, or the
// vector built by the previous update), giving sigma_j = 1/||.|| for the
// stored top block and the normalised bottom block b_j.  Returns false (in
// every workgroup) on a happy breakdown.  Workgroup 0 records the values.
__device__ bool arnoldi_prologue(const ArnoldiArgs &ar, double *red, double &sig, double bj[MAX_P]) {
  KDev *kd = ar.kd;
  const int j = ar.j, p = ar.p;
  const double s = reduce_fixed(ar.pin, ar.np_in, 1, 0, red);
  const int ld = MAX_M + 2;
  const bool w0 = blockIdx.x == 0;
  if (ar.start) {
    double s2 = s;
    for (int k = 0; k < p; ++k) s2 += ar.ybot[k] * ar.ybot[k];
    const double beta = sqrt(s2);
    sig = 1.0 / beta;
    for (int k = 0; k < p; ++k) bj[k] = ar.ybot[k] / beta;
    if (w0) {
      for (int k = threadIdx.x; k < ld * ld; k += blockDim.x) kd->H[k] = 0.0;
      if (threadIdx.x == 0) {
        kd->beta = beta;
        kd->sigma[0] = sig;
        for (int k = 0; k < p; ++k) kd->bot[k] = bj[k];
        kd->happy = 0;
        kd->J = 0;
      }
    }
    return true;
  }
  const double nrm = sqrt(s + kd->wn2[j]);
  if (nrm < ar.tol) {
    if (w0 && threadIdx.x == 0) {
      kd->happy = 1;
      kd->J = j;
    }
    return false;
  }
  sig = 1.0 / nrm;
  for (int k = 0; k < p; ++k) bj[k] = kd->botu[j * MAX_P + k] / nrm;
  if (w0 && threadIdx.x == 0) {
    kd->H[j * ld + (j - 1)] = nrm;
    kd->sigma[j] = sig;
    for (int k = 0; k < p; ++k) kd->bot[j * MAX_P + k] = bj[k];
    kd->J = j;
  }
  return true;
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
// The fused DFR kernel.  A block takes a tile of TX x TY elements of one panel
// (TX, TY divide ne), one thread per GL node.
//  A  (per node): metric terms from 1-D tangent tables (App. B), nodal fluxes
//     (Eq. 136) and sources (Eq. 2) in complex arithmetic; state and fluxes
//     staged in LDS.
//  B1 (per node): the interior part of the extended-point derivative of
//     Eq. (12) in both directions, kept in registers.
//  B2 (per element, face, field, face point): own traces (Eq. 7 at +-1) from
//     LDS; traces of the neighbours outside the tile from global memory.
//  C  (per face point of the tile, each face once): App. C map of the
//     neighbour's momentum at panel edges, Rusanov common flux.
//  D  (per node): face terms of Eq. (12), sources, division by sqrt(g);
//     output Re (F) or Im/eps (J v), optionally with the Arnoldi epilogue.
// LDS regions are reused across phases: R0 = state (A..B2) then face fluxes
// (C, D); R1 = x^1 fluxes (A, B1) then own traces (B2, C); R2 = x^2 fluxes
// (A, B1) then halo traces (B2, C).
constexpr int DFR_MAX_THREADS = 1024;
constexpr int DFR_MAX_HALO = 128;   // external faces of a tile: 2 (TX + TY)

struct HaloDesc {
  int base;    // first node index of the neighbour element
  int qface;   // the neighbour's face that touches the tile
  int rev;     // along-edge orientation reversed
  int edge;    // 1 on a panel edge (App. C map needed)
};

template <typename T>
__device__ __forceinline__ cx<T> lds_cx(const T *p, int i) {
  return {p[2 * i], p[2 * i + 1]};
}
template <typename T>
__device__ __forceinline__ void lds_cx_store(T *p, int i, cx<T> z) {
  p[2 * i] = z.r;
  p[2 * i + 1] = z.i;
}

template <int NS, typename T, typename TQ, bool CS>
__global__ __launch_bounds__(DFR_MAX_THREADS) void dfr_kernel(const GridArgs g, const Ops1D ops, const int TX,
                                                               const int TY, const int r0_len, const int r1_len,
                                                               const TQ *__restrict__ q, const double *__restrict__ v,
                                                               const double *__restrict__ vscale, double eps,
                                                               double *__restrict__ out, const ArnoldiArgs ar) {
  constexpr int NN = NS * NS;
  extern __shared__ double dyn[];
  __shared__ T sD[NS][NS + 2];
  __shared__ T slm[NS], slp[NS];
  __shared__ HaloDesc hd[DFR_MAX_HALO];
  __shared__ double red[256];
  // complex values are stored as (re, im) pairs of T
  T *R0 = reinterpret_cast<T *>(dyn);
  T *R1 = R0 + 2 * r0_len;
  T *R2 = R1 + 2 * r1_len;

  if (ar.on && ar.kd->happy) return;   // uniform: the sub-step ended in a happy breakdown

  const int tid = threadIdx.x;
  const int ne = g.ne;
  const int N = (int)g.n;
  const int ntx = ne / TX, nty = ne / TY;
  const int nel = TX * TY;
  const int lb = (int)logical_block(6 * ntx * nty);
  if (lb < 0) {                        // uniform: padding block of the XCD mapping
    if (ar.on && tid == 0) {
      ar.pout[blockIdx.x * 2 + 0] = 0.0;
      ar.pout[blockIdx.x * 2 + 1] = 0.0;
    }
    return;
  }
  double vs = 1.0;
  double bj[MAX_P];
  if (ar.on) {
    if (!arnoldi_prologue(ar, red, vs, bj)) return;   // uniform
  } else if (CS && vscale) {
    vs = *vscale;
  }
  const int p = lb / (ntx * nty);
  const int trow = (lb - p * ntx * nty) / ntx;
  const int tcol = lb - p * ntx * nty - trow * ntx;
  const int ej0 = trow * TY, ei0 = tcol * TX;

  for (int k = tid; k < NS * (NS + 2); k += blockDim.x) sD[k / (NS + 2)][k % (NS + 2)] = (T)ops.Dt[k / (NS + 2)][k % (NS + 2)];
  if (tid < NS) {
    slm[tid] = (T)ops.lm[tid];
    slp[tid] = (T)ops.lp[tid];
  }
  // halo descriptors: [0,TY) west, [TY,2TY) east, [2TY,2TY+TX) south, then north
  const int nhalo = 2 * (TX + TY);
  if (tid < nhalo) {
    int face, ei, ej;
    if (tid < TY) { face = 0; ej = ej0 + tid; ei = ei0; }
    else if (tid < 2 * TY) { face = 1; ej = ej0 + tid - TY; ei = ei0 + TX - 1; }
    else if (tid < 2 * TY + TX) { face = 2; ei = ei0 + tid - 2 * TY; ej = ej0; }
    else { face = 3; ei = ei0 + tid - 2 * TY - TX; ej = ej0 + TY - 1; }
    int qp = p, qe = ej, qi = ei, qf, rev = 0, edge = 0;
    if (face == 0) { if (ei > 0) { qi = ei - 1; qf = 1; } else edge = 1; }
    else if (face == 1) { if (ei < ne - 1) { qi = ei + 1; qf = 0; } else edge = 1; }
    else if (face == 2) { if (ej > 0) { qe = ej - 1; qf = 3; } else edge = 1; }
    else { if (ej < ne - 1) { qe = ej + 1; qf = 2; } else edge = 1; }
    if (edge) {
      const int along = (face < 2) ? ej : ei;
      qp = g.nb_q[p][face];
      qf = g.nb_e[p][face];
      rev = g.nb_rev[p][face];
      const int qa = rev ? ne - 1 - along : along;
      if (qf == 0) { qi = 0; qe = qa; }
      else if (qf == 1) { qi = ne - 1; qe = qa; }
      else if (qf == 2) { qe = 0; qi = qa; }
      else { qe = ne - 1; qi = qa; }
    }
    hd[tid] = {((qp * ne + qe) * ne + qi) * NN, qf, rev, edge};
  }

  const int s = tid / NN, node = tid - s * NN, nj = node / NS, ni = node - nj * NS;
  const bool active = s < nel;
  const int sy = s / TX, sx = s - sy * TX;
  const int ei = ei0 + sx, ej = ej0 + sy;
  const int gidx = ((p * ne + ej) * ne + ei) * NN + node;
  const T gred = (T)g.g_red;
  const double eps_vs = eps * vs;

  cx<T> src1 = {T(0), T(0)}, src2 = {T(0), T(0)};
  T rs = T(0);
  double vtrue[3] = {0.0, 0.0, 0.0};

  // ---- A: state, nodal fluxes, sources
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
      lds_cx_store(R0, (s * 3 + f) * NN + node, Qz[f]);
    }
    const cx<T> H = Qz[0], M1 = Qz[1], M2 = Qz[2];
    if (!(H.r > T(0))) atomicOr(g.err_flag, 2);
    const cx<T> rH = crcp1(H);
    const cx<T> u1 = cmul(M1, rH), u2 = cmul(M2, rH);
    const cx<T> H2h = (T(0.5) * gred) * cmul(H, H);
    const cx<T> m11 = cmul(M1, u1), m12 = cmul(M1, u2), m22 = cmul(M2, u2);
    const cx<T> f12 = sg * (m12 + e12 * H2h);
    lds_cx_store(R1, (s * 3 + 0) * NN + node, sg * M1);
    lds_cx_store(R1, (s * 3 + 1) * NN + node, sg * (m11 + e11 * H2h));
    lds_cx_store(R1, (s * 3 + 2) * NN + node, f12);
    lds_cx_store(R2, (s * 3 + 0) * NN + node, sg * M2);
    lds_cx_store(R2, (s * 3 + 1) * NN + node, f12);
    lds_cx_store(R2, (s * 3 + 2) * NN + node, sg * (m22 + e22 * H2h));
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

  // ---- B1: interior part of the derivative, both directions
  cx<T> acc[3];
  if (active) {
#pragma unroll
    for (int f = 0; f < 3; ++f) {
      const int b = (s * 3 + f) * NN;
      cx<T> d = {T(0), T(0)};
#pragma unroll
      for (int k = 0; k < NS; ++k) {
        d = d + sD[ni][k + 1] * lds_cx(R1, b + nj * NS + k);
        d = d + sD[nj][k + 1] * lds_cx(R2, b + k * NS + ni);
      }
      acc[f] = d;
    }
  }
  __syncthreads();

  // ---- B2: own traces (into R1) and halo traces (into R2)
  // own: task = ((s * 4 + face) * 3 + f) * NS + t ; stored at the same index
  for (int task = tid; task < nel * 12 * NS; task += blockDim.x) {
    const int t = task % NS;
    const int r = task / NS;
    const int f = r % 3;
    const int r2 = r / 3;
    const int face = r2 & 3, es = r2 >> 2;
    const T *w = (face == 0 || face == 2) ? slm : slp;
    const int b = (es * 3 + f) * NN + ((face < 2) ? t * NS : t);
    const int st = (face < 2) ? 1 : NS;
    cx<T> a = {T(0), T(0)};
#pragma unroll
    for (int k = 0; k < NS; ++k) a = a + w[k] * lds_cx(R0, b + k * st);
    lds_cx_store(R1, task, a);
  }
  // halo: task = (h * 3 + f) * NS + t
  for (int task = tid; task < nhalo * 3 * NS; task += blockDim.x) {
    const int t = task % NS;
    const int r = task / NS;
    const int f = r % 3, h = r / 3;
    const HaloDesc d = hd[h];
    const int qt = d.rev ? NS - 1 - t : t;
    const T *w = (d.qface == 0 || d.qface == 2) ? slm : slp;
    const int first = f * N + d.base + ((d.qface < 2) ? qt * NS : qt);
    const int st = (d.qface < 2) ? 1 : NS;
    cx<T> a = {T(0), T(0)};
#pragma unroll
    for (int k = 0; k < NS; ++k) {
      const int id = first + k * st;
      T zi = T(0);
      if (CS) zi = (T)(eps_vs * v[id]);
      a = a + w[k] * cx<T>{(T)q[id], zi};
    }
    lds_cx_store(R2, task, a);
  }
  __syncthreads();

  // ---- C: common fluxes, each face of the tile once, into R0
  // vertical faces (x^1 normal): (fx, sy, t), fx = 0..TX ; then horizontal (fy, sx, t)
  const int nvert = (TX + 1) * TY * NS;
  const int nflux = nvert + (TY + 1) * TX * NS;
  for (int task = tid; task < nflux; task += blockDim.x) {
    const bool vert = task < nvert;
    const int tk = vert ? task : task - nvert;
    const int t = tk % NS;
    const int r = tk / NS;
    int n, lo_el, hi_el, lo_h, hi_h, ex, ey, fxy;
    if (vert) {
      n = 0;
      const int fy_ = r % TY;   // element row in the tile
      fxy = r / TY;             // face column 0..TX
      lo_el = (fxy > 0) ? fy_ * TX + fxy - 1 : -1;
      hi_el = (fxy < TX) ? fy_ * TX + fxy : -1;
      lo_h = fy_;               // west halo
      hi_h = TY + fy_;          // east halo
      ex = ei0 + fxy;           // edge index along x^1
      ey = ej0 + fy_;
    } else {
      n = 1;
      const int fx_ = r % TX;
      fxy = r / TX;             // face row 0..TY
      lo_el = (fxy > 0) ? (fxy - 1) * TX + fx_ : -1;
      hi_el = (fxy < TY) ? fxy * TX + fx_ : -1;
      lo_h = 2 * TY + fx_;      // south halo
      hi_h = 2 * TY + TX + fx_; // north halo
      ex = ei0 + fx_;
      ey = ej0 + fxy;
    }
    cx<T> QL[3], QR[3];
    int hq = -1;   // halo side read (for the App. C map)
#pragma unroll
    for (int f = 0; f < 3; ++f) {
      // own traces of the low element on its high face (E or N), of the high
      // element on its low face (W or S)
      if (lo_el >= 0) QL[f] = lds_cx(R1, ((lo_el * 4 + (n == 0 ? 1 : 3)) * 3 + f) * NS + t);
      else { QL[f] = lds_cx(R2, (lo_h * 3 + f) * NS + t); hq = lo_h; }
      if (hi_el >= 0) QR[f] = lds_cx(R1, ((hi_el * 4 + (n == 0 ? 0 : 2)) * 3 + f) * NS + t);
      else { QR[f] = lds_cx(R2, (hi_h * 3 + f) * NS + t); hq = hi_h; }
    }
    if (hq >= 0 && hd[hq].edge) {
      // App. C: neighbour components -> this panel's basis
      const int face = (hq < TY) ? 0 : (hq < 2 * TY) ? 1 : (hq < 2 * TY + TX) ? 2 : 3;
      const int along = (face < 2) ? ey : ex;
      const double *M = g.xform + (((p * 4 + face) * ne + along) * NS + t) * 4;
      const T m00 = (T)M[0], m01 = (T)M[1], m10 = (T)M[2], m11 = (T)M[3];
      cx<T> *Qn = (lo_el < 0) ? QL : QR;
      const cx<T> a1 = m00 * Qn[1] + m01 * Qn[2];
      const cx<T> a2 = m10 * Qn[1] + m11 * Qn[2];
      Qn[1] = a1;
      Qn[2] = a2;
    }
    // metric at the face point
    T X, Y, ax, ay, rax, ray;
    if (n == 0) {
      X = (T)g.tedge[ex]; ax = T(1) + X * X; rax = frcp(ax);
      const Tan3 ty = g.tnode[ey * NS + t];
      Y = (T)ty.x; ay = (T)ty.ax; ray = (T)ty.rax;
    } else {
      const Tan3 tx = g.tnode[ex * NS + t];
      X = (T)tx.x; ax = (T)tx.ax; rax = (T)tx.rax;
      Y = (T)g.tedge[ey]; ay = T(1) + Y * Y; ray = frcp(ay);
    }
    const T d2 = ax + Y * Y;
    const T rd = frsqrt(d2);
    const T sg = ax * ay * rd * rd * rd;
    const T e11 = d2 * rax, e22 = d2 * ray, e12 = X * Y * e11 * ray;
    const T eta1n = n == 0 ? e11 : e12, eta2n = n == 0 ? e12 : e22, etann = n == 0 ? e11 : e22;
    cx<T> fL[3], fR[3], cL, cR;
    side_flux1(QL, n, eta1n, eta2n, etann, gred, fL, cL);
    side_flux1(QR, n, eta1n, eta2n, etann, gred, fR, cR);
    const cx<T> lam = (cL.r >= cR.r) ? cL : cR;
#pragma unroll
    for (int f = 0; f < 3; ++f) {
      const cx<T> F = T(0.5) * (fL[f] + fR[f]) - T(0.5) * cmul(lam, QR[f] - QL[f]);
      lds_cx_store(R0, task * 3 + f, sg * F);
    }
  }
  __syncthreads();

  // ---- D: face terms, sources, output
  double w[3] = {0.0, 0.0, 0.0};
  if (active) {
    const T scale = -(T)g.two_over_delta * rs;
    const T invE = CS ? (T)(1.0 / eps) : T(1);
    const int iW = ((sx * TY + sy) * NS + nj) * 3, iE = (((sx + 1) * TY + sy) * NS + nj) * 3;
    const int iS = nvert * 3 + ((sy * TX + sx) * NS + ni) * 3, iN = nvert * 3 + (((sy + 1) * TX + sx) * NS + ni) * 3;
#pragma unroll
    for (int f = 0; f < 3; ++f) {
      cx<T> d = acc[f];
      d = d + sD[ni][0] * lds_cx(R0, iW + f) + sD[ni][NS + 1] * lds_cx(R0, iE + f);
      d = d + sD[nj][0] * lds_cx(R0, iS + f) + sD[nj][NS + 1] * lds_cx(R0, iN + f);
      cx<T> r = scale * d;
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
#pragma unroll
    for (int f = 0; f < 3; ++f) {
      const int id = f * N + gidx;
      double a = w[f];
      for (int k = 0; k < ar.p; ++k) a += ar.W[k][id] * bj[k];
      out[id] = a;
      d0 += a * vtrue[f];
      if (ar.vprev) d1 += a * ar.vprev[id];
    }
  }
  const double b0 = block_sum(d0, red);
  const double b1 = block_sum(d1, red);
  if (tid == 0) {
    ar.pout[blockIdx.x * 2 + 0] = b0;
    ar.pout[blockIdx.x * 2 + 1] = b1;
  }
}

// first Arnoldi step of a sub-step whose top block is identically zero:
// w = W b_0 (no J v); both partial inner products vanish
__global__ __launch_bounds__(BLOCK) void arnoldi_first_kernel(int64_t n3, const ArnoldiArgs ar, double *out) {
  __shared__ double red[256];
  if (ar.kd->happy) return;
  double sig, bj[MAX_P];
  if (!arnoldi_prologue(ar, red, sig, bj)) return;
  for (int64_t i = (int64_t)blockIdx.x * BLOCK + threadIdx.x; i < n3; i += (int64_t)gridDim.x * BLOCK) {
    double acc = 0.0;
    for (int k = 0; k < ar.p; ++k) acc += ar.W[k][i] * bj[k];
    out[i] = acc;
  }
  if (threadIdx.x == 0) {
    ar.pout[blockIdx.x * 2 + 0] = 0.0;
    ar.pout[blockIdx.x * 2 + 1] = 0.0;
  }
}

// Gram-Schmidt step.  Prologue: the inner products h_{j,j}, h_{j-1,j} (top
// partials of the J v kernel plus the bottom blocks; classical Gram-Schmidt
// over the last two vectors) and the new bottom block, recorded by workgroup
// 0.  Body: w <- w - h_jj sigma_j v~_j - h_{j-1,j} v_{j-1}; v_j <- sigma_j v~_j
// (stored normalised); partial ||w||^2 per workgroup.
__global__ __launch_bounds__(BLOCK) void arnoldi_update_kernel(int64_t n3, int j, int p, double *w, double *vj,
                                                               const double *vprev, const double *pin, int np_in,
                                                               double *pout, KDev *kd) {
  __shared__ double red[256];
  if (kd->happy) return;
  const double d0 = reduce_fixed(pin, np_in, 2, 0, red);
  const double d1 = reduce_fixed(pin, np_in, 2, 1, red);
  const int ld = MAX_M + 2;
  const bool two = (j >= 1) && (vprev != nullptr);
  const double *bj = kd->bot + j * MAX_P;
  const double *bp = kd->bot + (j - (j >= 1 ? 1 : 0)) * MAX_P;
  double wb[MAX_P];
  for (int k = 0; k < p; ++k) wb[k] = (k + 1 < p) ? bj[k + 1] : 0.0;   // K b_j (upper shift)
  double hjj = d0, hpj = d1;
  for (int k = 0; k < p; ++k) hjj += bj[k] * wb[k];
  if (two) {
    for (int k = 0; k < p; ++k) hpj += bp[k] * wb[k];
  } else {
    hpj = 0.0;
  }
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    kd->H[j * ld + j] = hjj;
    if (two) kd->H[(j - 1) * ld + j] = hpj;
    double nb2 = 0.0;
    for (int k = 0; k < p; ++k) {
      double v = wb[k] - hjj * bj[k];
      if (two) v -= hpj * bp[k];
      kd->botu[(j + 1) * MAX_P + k] = v;
      nb2 += v * v;
    }
    kd->wn2[j + 1] = nb2;
  }
  const double sj = kd->sigma[j];
  double acc = 0.0;
  for (int64_t i = (int64_t)blockIdx.x * BLOCK + threadIdx.x; i < n3; i += (int64_t)gridDim.x * BLOCK) {
    const double vv = sj * vj[i];
    double x = w[i] - hjj * vv;
    if (two) x -= hpj * vprev[i];
    w[i] = x;
    vj[i] = vv;
    acc += x * x;
  }
  const double b = block_sum(acc, red);
  if (threadIdx.x == 0) pout[blockIdx.x] = b;
}

// start of a sub-step: v~_0 = x (copied), partial ||x||^2 per workgroup
__global__ __launch_bounds__(BLOCK) void arnoldi_start_kernel(int64_t n3, const double *x, double *v0, double *pout) {
  __shared__ double red[BLOCK / 64];
  double acc = 0.0;
  for (int64_t i = (int64_t)blockIdx.x * BLOCK + threadIdx.x; i < n3; i += (int64_t)gridDim.x * BLOCK) {
    const double xv = x[i];
    v0[i] = xv;
    acc += xv * xv;
  }
  const double b = block_sum(acc, red);
  if (threadIdx.x == 0) pout[blockIdx.x] = b;
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
// four FMAs; the k loop is unrolled for independent loads in flight.
__device__ void lds_matmul(const double *A, const double *B, double *C, int ld) {
  const int nt = ld / 4;
  for (int tile = threadIdx.x; tile < nt * nt; tile += blockDim.x) {
    const int r0 = (tile / nt) * 4, c0 = (tile % nt) * 4;
    double acc[4][4];
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
      for (int j = 0; j < 4; ++j) acc[i][j] = 0.0;
    const double *a0p = A + r0 * ld, *a1p = a0p + ld, *a2p = a1p + ld, *a3p = a2p + ld;
#pragma unroll 4
    for (int k = 0; k < ld; ++k) {
      const double a0 = a0p[k], a1 = a1p[k], a2 = a2p[k], a3 = a3p[k];
      const double *bp = B + k * ld + c0;
      const double b0 = bp[0], b1 = bp[1], b2 = bp[2], b3 = bp[3];
      acc[0][0] = fma(a0, b0, acc[0][0]); acc[0][1] = fma(a0, b1, acc[0][1]);
      acc[0][2] = fma(a0, b2, acc[0][2]); acc[0][3] = fma(a0, b3, acc[0][3]);
      acc[1][0] = fma(a1, b0, acc[1][0]); acc[1][1] = fma(a1, b1, acc[1][1]);
      acc[1][2] = fma(a1, b2, acc[1][2]); acc[1][3] = fma(a1, b3, acc[1][3]);
      acc[2][0] = fma(a2, b0, acc[2][0]); acc[2][1] = fma(a2, b1, acc[2][1]);
      acc[2][2] = fma(a2, b2, acc[2][2]); acc[2][3] = fma(a2, b3, acc[2][3]);
      acc[3][0] = fma(a3, b0, acc[3][0]); acc[3][1] = fma(a3, b1, acc[3][1]);
      acc[3][2] = fma(a3, b2, acc[3][2]); acc[3][3] = fma(a3, b3, acc[3][3]);
    }
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
      for (int j = 0; j < 4; ++j) C[(r0 + i) * ld + c0 + j] = acc[i][j];
  }
}

// Taylor coefficients 1/k!, k = 0..18, and a zero for k = 19 (degree 18)
__constant__ double kInvFact[20] = {
    1.0, 1.0, 0.5, 1.0 / 6.0, 1.0 / 24.0, 1.0 / 120.0, 1.0 / 720.0, 1.0 / 5040.0, 1.0 / 40320.0,
    1.0 / 362880.0, 1.0 / 3628800.0, 1.0 / 39916800.0, 1.0 / 479001600.0, 1.0 / 6227020800.0,
    1.0 / 87178291200.0, 1.0 / 1307674368000.0, 1.0 / 20922789888000.0, 1.0 / 355687428096000.0,
    1.0 / 6402373705728000.0, 0.0};

__global__ __launch_bounds__(EXPM_BLOCK) void expm_kernel(KDev *kd, double tau, KHost *res, int jfin, const double *pin,
                                                     int np_in, double tol) {
  extern __shared__ double lds[];
  __shared__ double red[256];
  __shared__ double cnorm;
  // finalise the norm of the last vector built (unless a happy breakdown
  // already ended the sweep): h_{jfin, jfin-1}, or a happy breakdown
  if (!kd->happy) {
    const double s = reduce_fixed(pin, np_in, 1, 0, red);
    if (threadIdx.x == 0) {
      const double nrm = sqrt(s + kd->wn2[jfin]);
      if (nrm < tol) kd->happy = 1;
      else kd->H[jfin * (MAX_M + 2) + (jfin - 1)] = nrm;
      kd->J = jfin;
    }
    __syncthreads();
  }
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
  // 1-norm (max column sum): the column sums of H_aug are those of tau*H_J
  // plus tau in column J; four threads per column
  double cm = 0.0;
  for (int idx = threadIdx.x; idx < 4 * n; idx += blockDim.x) {
    const int j = idx >> 2, part = idx & 3;
    double cs = 0.0;
    for (int i = part; i < n; i += 4) cs += fabs(A[i * ld + j]);
    cs += __shfl_xor(cs, 1, 64);
    cs += __shfl_xor(cs, 2, 64);
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
  // P = c18 I + c19 A  (padding stays zero: only the leading n x n block is set)
  for (int idx = threadIdx.x; idx < nn; idx += blockDim.x) {
    const int i = idx / ld, j = idx - i * ld;
    P[idx] = ((i == j && i < n) ? kInvFact[18] : 0.0) + kInvFact[19] * A[idx];
  }
  __syncthreads();
  for (int k = 8; k >= 0; --k) {
    lds_matmul(A2, P, Q, ld);
    __syncthreads();
    for (int idx = threadIdx.x; idx < nn; idx += blockDim.x) {
      const int i = idx / ld, j = idx - i * ld;
      P[idx] = Q[idx] + ((i == j && i < n) ? kInvFact[2 * k] : 0.0) + kInvFact[2 * k + 1] * A[idx];
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

// a positive smooth state (H = 1 + 0.1 sin, small momenta) and a direction,
// used only to time kernels
__global__ __launch_bounds__(BLOCK) void fill_kernel(int64_t n, double *q, double *v) {
  for (int64_t i = (int64_t)blockIdx.x * BLOCK + threadIdx.x; i < 3 * n; i += (int64_t)gridDim.x * BLOCK) {
    const double x = (double)(i % n) * 1e-3;
    q[i] = (i < n) ? 1.0 + 0.1 * sin(x) : 0.05 * cos(x + (double)(i / n));
    v[i] = 1e-3 * sin(3.0 * x + 1.0);
  }
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

// LDS regions of the tiled kernel, in complex values: R0, R1, R2
static void dfr_regions(int ns, int tx, int ty, int &r0, int &r1, int &r2) {
  const int nn = ns * ns, nel = tx * ty, nhalo = 2 * (tx + ty);
  const int nflux = ((tx + 1) * ty + (ty + 1) * tx) * ns;
  r0 = std::max(nel * 3 * nn, nflux * 3);
  r1 = std::max(nel * 3 * nn, nel * 12 * ns);
  r2 = std::max(nel * 3 * nn, nhalo * 3 * ns);
}

size_t dfr_lds_bytes(int ns, int tx, int ty, bool fp32) {
  int r0, r1, r2;
  dfr_regions(ns, tx, ty, r0, r1, r2);
  return (size_t)(r0 + r1 + r2) * 2 * (fp32 ? sizeof(float) : sizeof(double));
}

int64_t dfr_grid_blocks(const Ctx *c) {
  const int64_t nlog = 6LL * (c->ne / c->tile_tx) * (c->ne / c->tile_ty);
  return ((nlog + 7) / 8) * 8;
}

template <int NS, typename T, typename TQ, bool CS>
static void launch_ns(Ctx *c, const TQ *q, const double *v, const double *vscale, double eps, double *out,
                      const ArnoldiArgs &ar) {
  const int tx = c->tile_tx, ty = c->tile_ty;
  int r0, r1, r2;
  dfr_regions(NS, tx, ty, r0, r1, r2);
  const size_t lds = (size_t)(r0 + r1 + r2) * 2 * sizeof(T);
  const int threads = ((tx * ty * NS * NS + 63) / 64) * 64;
  const int64_t nb = dfr_grid_blocks(c);
  tbegin(c, !CS ? DFR_K_RHS : (ar.on ? DFR_K_JV_ARNOLDI : DFR_K_JV));
  hipLaunchKernelGGL((dfr_kernel<NS, T, TQ, CS>), dim3((unsigned)nb), dim3(threads), lds, c->stream, c->ga, c->ops,
                     tx, ty, r0, r1, q, v, vscale, eps, out, ar);
  tend(c);
}

template <int NS>
static int set_lds_attr(size_t bytes) {
  DFR_HIP(hipFuncSetAttribute((const void *)dfr_kernel<NS, double, double, false>,
                              hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes));
  DFR_HIP(hipFuncSetAttribute((const void *)dfr_kernel<NS, double, double, true>,
                              hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes));
  DFR_HIP(hipFuncSetAttribute((const void *)dfr_kernel<NS, float, float, true>,
                              hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes));
  return DFR_OK;
}

// allow the dynamic LDS of every tile the context may use
int dfr_set_lds_limits(Ctx *c, size_t bytes) {
  switch (c->ns) {
    case 2: return set_lds_attr<2>(bytes);
    case 3: return set_lds_attr<3>(bytes);
    case 4: return set_lds_attr<4>(bytes);
    case 5: return set_lds_attr<5>(bytes);
    case 6: return set_lds_attr<6>(bytes);
    case 7: return set_lds_attr<7>(bytes);
    case 8: return set_lds_attr<8>(bytes);
    default: set_error("unsupported number of GL points"); return DFR_E_INVAL;
  }
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

static inline int grid_reduce(int64_t n) {
  // vector kernels whose partial sums are consumed by the next kernel use at
  // most 1024 workgroups (grid-stride loops)
  const int g = grid_for(n);
  return g < 1024 ? g : 1024;
}

int launch_arnoldi_first(Ctx *c, const ArnoldiArgs &ar, double *out, int *np_out) {
  const int64_t n3 = 3 * c->n;
  const int nb = grid_reduce(n3);
  tbegin(c, DFR_K_OTHER);
  hipLaunchKernelGGL(arnoldi_first_kernel, dim3(nb), dim3(BLOCK), 0, c->stream, n3, ar, out);
  tend(c);
  DFR_HIP(hipGetLastError());
  *np_out = nb;
  return DFR_OK;
}

int launch_update(Ctx *c, int j, double *w, double *vj, const double *vprev, const double *pin, int np_in,
                  double *pout, int *np_out) {
  const int64_t n3 = 3 * c->n;
  const int nb = grid_reduce(n3);
  tbegin(c, DFR_K_UPDATE);
  hipLaunchKernelGGL(arnoldi_update_kernel, dim3(nb), dim3(BLOCK), 0, c->stream, n3, j, c->kiops_p, w, vj, vprev, pin,
                     np_in, pout, c->d_kd);
  tend(c);
  DFR_HIP(hipGetLastError());
  *np_out = nb;
  return DFR_OK;
}

int launch_start(Ctx *c, const double *x, double *v0, double *pout, int *np_out) {
  const int64_t n3 = 3 * c->n;
  const int nb = grid_reduce(n3);
  tbegin(c, DFR_K_OTHER);
  hipLaunchKernelGGL(arnoldi_start_kernel, dim3(nb), dim3(BLOCK), 0, c->stream, n3, x, v0, pout);
  tend(c);
  DFR_HIP(hipGetLastError());
  *np_out = nb;
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

int launch_expm(Ctx *c, double tau, int jfin, const double *pin, int np_in, double tol) {
  const int n = ((c->kiops_mmax + 1) + 3) & ~3;
  const size_t lds = (size_t)4 * n * n * sizeof(double);
  tbegin(c, DFR_K_EXPM);
  hipLaunchKernelGGL(expm_kernel, dim3(1), dim3(EXPM_BLOCK), lds, c->stream, c->d_kd, tau, (KHost *)c->d_expm_scratch, jfin,
                     pin, np_in, tol);
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

int launch_fill(Ctx *c, double *q, double *v) {
  hipLaunchKernelGGL(fill_kernel, dim3(grid_for(3 * c->n)), dim3(BLOCK), 0, c->stream, c->n, q, v);
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
