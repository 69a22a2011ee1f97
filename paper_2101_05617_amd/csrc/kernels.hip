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
#include <type_traits>
#include <cmath>
#include <cstring>

namespace dfrsw {

// ---------------------------------------------------------------------------
// complex arithmetic on (re, im) pairs: the complex step evaluates F on
// z = q + i eps v, whose imaginary parts are O(eps |v|)
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
// product without the Im*Im term: it is below half an ulp of Re*Re whenever
// both imaginary parts are below 2^-27 (FP64) / 2^-12 (FP32) of the real
// parts, so the result equals that of exact complex arithmetic in floating
// point (the same condition as crcp1 / csqrt1 below)
template <typename T>
__device__ __forceinline__ cx<T> cmul1(cx<T> a, cx<T> b) {
  return {a.r * b.r, fma(a.r, b.i, a.i * b.r)};
}
// lane exchange within rows of 16 lanes by DPP (register moves, no LDS):
// CTRL 0xB1 swaps neighbours, 0x4E swaps pairs within a quad, 0x141 mirrors
// each half-row, 0x140 mirrors each row
template <int CTRL>
__device__ __forceinline__ double dpp_mov(double v) {
  const int lo = __builtin_amdgcn_update_dpp(0, __double2loint(v), CTRL, 0xf, 0xf, false);
  const int hi = __builtin_amdgcn_update_dpp(0, __double2hiint(v), CTRL, 0xf, 0xf, false);
  return __hiloint2double(hi, lo);
}
__device__ __forceinline__ double read_lane(double v, int lane) {
  return __hiloint2double(__builtin_amdgcn_readlane(__double2hiint(v), lane),
                          __builtin_amdgcn_readlane(__double2loint(v), lane));
}

// sum over the 64 lanes of a wave (every lane active), in a fixed order, the
// same value in every lane: pairs, quads, half-rows and rows by DPP, then
// the four row sums
__device__ __forceinline__ double wave_sum(double v) {
  v += dpp_mov<0xB1>(v);
  v += dpp_mov<0x4E>(v);
  v += dpp_mov<0x141>(v);
  v += dpp_mov<0x140>(v);
  return (read_lane(v, 0) + read_lane(v, 16)) + (read_lane(v, 32) + read_lane(v, 48));
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

// block-wide sums of two values in a fixed order; valid in thread 0
__device__ __forceinline__ void block_sum2(double &a, double &b, double *red) {
  a = wave_sum(a);
  b = wave_sum(b);
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  __syncthreads();
  if (lane == 0) {
    red[2 * wv] = a;
    red[2 * wv + 1] = b;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    double sa = 0.0, sb = 0.0;
    for (int k = 0; k < (int)(blockDim.x >> 6); ++k) {
      sa += red[2 * k];
      sb += red[2 * k + 1];
    }
    a = sa;
    b = sb;
  }
}

// XCD-aware logical block: consecutive logical blocks land on the same XCD
// (the dispatcher places block b on XCD b % 8), so neighbouring elements
// share an L2.  The stride per XCD follows the logical count, not the grid,
// so a grid larger than 8 ceil(nlogical / 8) (sized for counts known only
// on the device) still spreads the work over all eight XCDs; the blocks
// beyond it idle.
__device__ __forceinline__ int64_t logical_block(int64_t nlogical) {
  const int64_t b = blockIdx.x, per = (nlogical + 7) / 8;
  if (b >= 8 * per) return -1;
  const int64_t lb = (b % 8) * per + b / 8;
  return lb < nlogical ? lb : -1;
}

// Sum of pin[k*stride + off], k < np, in an order that does not depend on the
// workgroup size: 256 virtual lanes take every 256th value; the first wave
// (always 64 lanes) adds them in a fixed pattern and a fixed butterfly.  Every
// workgroup of every kernel gets the identical value.  red: 256 doubles of
// LDS.  Call from all threads of the workgroup; valid in every thread.
// One virtual lane l's share: the values k = l, l + 256, ... added in
// increasing k (a missing value adds 0.0, which leaves the sum unchanged);
// the loads of each group of four are issued together.
__device__ __forceinline__ double lane_sum(const double *pin, int np, int stride, int off, int l) {
  double s = 0.0;
  for (int k0 = l; k0 < np; k0 += 1024) {
    double x[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int k = k0 + 256 * u;
      x[u] = k < np ? pin[(int64_t)k * stride + off] : 0.0;
    }
#pragma unroll
    for (int u = 0; u < 4; ++u) s += x[u];
  }
  return s;
}

__device__ double reduce_fixed(const double *pin, int np, int stride, int off, double *red) {
  __syncthreads();
  for (int l = threadIdx.x; l < 256; l += blockDim.x) red[l] = lane_sum(pin, np, stride, off, l);
  __syncthreads();
  if (threadIdx.x < 64) {
    const int l = threadIdx.x;
    const double v = wave_sum((red[l] + red[l + 64]) + (red[l + 128] + red[l + 192]));
    if (l == 0) red[0] = v;
  }
  __syncthreads();
  const double r = red[0];
  __syncthreads();
  return r;
}

// The end of a fixed-order reduction of two interleaved sets pin[2k],
// pin[2k+1] (the order of reduce_fixed, hence the same values), once each
// virtual lane l < 256 has left its shares in red[l] and red[256 + l]; red:
// 512 doubles of LDS.  Valid in every thread.
__device__ void reduce_fixed2_finish(double *red, double &s0, double &s1) {
  __syncthreads();
  if (threadIdx.x < 64) {
    const int l = threadIdx.x;
    const double x = wave_sum((red[l] + red[l + 64]) + (red[l + 128] + red[l + 192]));
    const double y = wave_sum((red[256 + l] + red[256 + l + 64]) + (red[256 + l + 128] + red[256 + l + 192]));
    if (l == 0) {
      red[0] = x;
      red[256] = y;
    }
  }
  __syncthreads();
  s0 = red[0];
  s1 = red[256];
  __syncthreads();
}

// Arnoldi prologue, given the finished sum s of the partial squared norms:
// the norm of the vector v_j (start vector, or the vector built by the
// previous update), sigma_j = 1/||.|| for the stored top block and the
// normalised bottom block b_j.  Returns false on a happy breakdown.  In
// the writer workgroup (w0) the threads lane < nthr record the values (lane 0
// the scalars).
__device__ bool arnoldi_finish(const ArnoldiArgs &ar, double s, int lane, int nthr, bool w0, double &sig,
                               double bj[MAX_P]) {
  KDev *kd = ar.kd;
  const int j = ar.j, p = ar.p;
  const int ld = MAX_M + 2;
  if (ar.start) {
    double s2 = s;
    for (int k = 0; k < p; ++k) s2 += ar.ybot[k] * ar.ybot[k];
    const double beta = sqrt(s2);
    sig = 1.0 / beta;
    for (int k = 0; k < p; ++k) bj[k] = ar.ybot[k] / beta;
    if (w0) {
      for (int k = lane; k < ld * ld; k += nthr) kd->H[k] = 0.0;
      if (lane == 0) {
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
    if (w0 && lane == 0) {
      kd->happy = 1;
      kd->J = j;
    }
    return false;
  }
  sig = 1.0 / nrm;
  for (int k = 0; k < p; ++k) bj[k] = kd->botu[j * MAX_P + k] / nrm;
  if (w0 && lane == 0) {
    kd->H[j * ld + (j - 1)] = nrm;
    kd->sigma[j] = sig;
    for (int k = 0; k < p; ++k) kd->bot[j * MAX_P + k] = bj[k];
    kd->J = j;
  }
  return true;
}

// the prologue with its reduction, all threads of the workgroup taking part
__device__ bool arnoldi_prologue(const ArnoldiArgs &ar, double *red, bool w0, double &sig, double bj[MAX_P]) {
  const double s = reduce_fixed(ar.pin, ar.np_in, 1, 0, red);
  return arnoldi_finish(ar, s, threadIdx.x, blockDim.x, w0, sig, bj);
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

// ---------------------------------------------------------------------------
// Raw buffer access: a resource (base, size in bytes) in scalar registers and
// 32-bit byte offsets per lane, so that an indexed load or store costs one
// address instruction instead of 64-bit address arithmetic; offsets beyond
// the size read 0 and write nothing.  Every stream the kernels index is
// below 2 GiB (3N doubles at N = 4.2 M is 102 MB).
typedef __amdgpu_buffer_rsrc_t rsrc_t;
// base and size are the same in every lane of the wave (workgroup-uniform
// arguments); taking them from the first lane keeps the resource in scalar
// registers, where the buffer instructions need it
__device__ __forceinline__ rsrc_t make_rsrc(const void *base, uint32_t bytes) {
  const uint64_t a = reinterpret_cast<uint64_t>(base);
  const uint32_t lo = (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)a);
  const uint32_t hi = (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)(a >> 32));
  const int nb = __builtin_amdgcn_readfirstlane((int)bytes);
  void *u = reinterpret_cast<void *>(((uint64_t)hi << 32) | lo);
  // word 3 of a raw buffer resource on gfx9-family devices: 32-bit data format
  return __builtin_amdgcn_make_buffer_rsrc(u, (short)0, nb, 0x00020000);
}
template <typename T>
__device__ __forceinline__ T bload(rsrc_t r, uint32_t index);
template <>
__device__ __forceinline__ double bload<double>(rsrc_t r, uint32_t index) {
  return __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(r, index * 8u, 0, 0));
}
template <>
__device__ __forceinline__ float bload<float>(rsrc_t r, uint32_t index) {
  return __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(r, index * 4u, 0, 0));
}
template <typename T>
__device__ __forceinline__ void bstore(rsrc_t r, uint32_t index, T v);
template <>
__device__ __forceinline__ void bstore<double>(rsrc_t r, uint32_t index, double v) {
  typedef unsigned int u2 __attribute__((ext_vector_type(2)));
  __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(u2, v), r, index * 8u, 0, 0);
}
template <>
__device__ __forceinline__ void bstore<float>(rsrc_t r, uint32_t index, float v) {
  __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(unsigned int, v), r, index * 4u, 0, 0);
}
// a device-memory pointer as a global-address-space one: loads through it
// are global loads (scalar base, 32-bit lane offsets) rather than flat ones,
// also where the pointer itself was read from memory (the batched calls)
template <typename T>
__device__ __forceinline__ const __attribute__((address_space(1))) T *gmem(const T *p) {
  return (const __attribute__((address_space(1))) T *)p;
}

// four consecutive floats (16 bytes) at float4 index `index`
// three FP32 values at index (12-byte records)
__device__ __forceinline__ float4 bload3f(rsrc_t r, uint32_t index) {
  typedef unsigned int u3 __attribute__((ext_vector_type(3)));
  const u3 w = __builtin_bit_cast(u3, __builtin_amdgcn_raw_buffer_load_b96(r, index * 12u, 0, 0));
  return make_float4(__uint_as_float(w.x), __uint_as_float(w.y), __uint_as_float(w.z), 0.0f);
}
__device__ __forceinline__ float4 bload4f(rsrc_t r, uint32_t index) {
  typedef unsigned int u4 __attribute__((ext_vector_type(4)));
  const u4 w = __builtin_bit_cast(u4, __builtin_amdgcn_raw_buffer_load_b128(r, index * 16u, 0, 0));
  return make_float4(__uint_as_float(w.x), __uint_as_float(w.y), __uint_as_float(w.z), __uint_as_float(w.w));
}

// tangent record i of a device table, as global loads
__device__ __forceinline__ Tan3 ld_tan3(const Tan3 *tab, int i) {
  const auto r = gmem(tab) + i;
  Tan3 t;
  t.x = r->x;
  t.ax = r->ax;
  t.rax = r->rax;
  t.pad = 0.0;
  return t;
}

// two consecutive doubles (16 bytes) at double index `index`
__device__ __forceinline__ double2 bload2(rsrc_t r, uint32_t index) {
  typedef unsigned int u4 __attribute__((ext_vector_type(4)));
  const u4 w = __builtin_bit_cast(u4, __builtin_amdgcn_raw_buffer_load_b128(r, index * 8u, 0, 0));
  double2 d;
  d.x = __hiloint2double((int)w.y, (int)w.x);
  d.y = __hiloint2double((int)w.w, (int)w.z);
  return d;
}

// physical flux through an x^n = const face per unit sqrt(g)/a^2, and the
// Rusanov wave speed |u^n| + sqrt(h^nn g H), for Q = (H, H u^1, H u^2); the
// state is taken by value and the normal momentum Mn = H u^n passed in (no
// indexed arrays: they would live in scratch memory)
template <typename T>
__device__ __forceinline__ void side_flux1(cx<T> H, cx<T> M1, cx<T> M2, cx<T> Mn, T eta_1n, T eta_2n, T eta_nn,
                                           T gred, cx<T> &f0, cx<T> &f1, cx<T> &f2, cx<T> &c) {
  const cx<T> rH = crcp1(H);
  const cx<T> un = cmul1(Mn, rH);
  const cx<T> H2h = (T(0.5) * gred) * cmul1(H, H);
  f0 = Mn;
  f1 = cmul1(M1, un) + eta_1n * H2h;
  f2 = cmul1(M2, un) + eta_2n * H2h;
  // |u^n| with the branch of the real evaluation: sign(Re H u^n), H > 0
  const cx<T> au = (Mn.r >= T(0)) ? un : -un;
  c = au + csqrt1((eta_nn * gred) * H);
}

// AUSM common flux with double Froude-number splitting (App. D, Eqs.
// 137-143) per unit sqrt(g)/a^2: sqrt(g) T^{mu n} = M^n A^{mu n} + P^{mu n}
// with A^{mu n} = q^mu a^n, a^n = sqrt(h^nn g H) (App. E), P^{0n} = 0 and
// P^{in} = g h^{in} H^2 / 2 (per unit sqrt(g)).  The split functions are the
// original AUSM's (Liou and Steffen 1993): for |M| <= 1, M+- = +-(M +- 1)^2/4
// and pressure weights (M +- 1)^2 (2 -+ M)/4; beyond, the upwind values.
// "+" parts come from the low side L, "-" parts from the high side R; every
// branch follows the real parts, and a split Froude number of exactly zero
// takes the advective part from L.
template <typename T>
__device__ __forceinline__ void ausm_flux(cx<T> HL, cx<T> L1, cx<T> L2, cx<T> HR, cx<T> R1, cx<T> R2, int n,
                                          T eta1n, T eta2n, T etann, T gred, cx<T> &F0, cx<T> &F1, cx<T> &F2) {
  const cx<T> one{T(1), T(0)};
  // low side: Froude number, wave speed, "+" splits
  const cx<T> aL = csqrt1((etann * gred) * HL);
  const cx<T> ML = cmul1(cmul1(n == 0 ? L1 : L2, crcp1(HL)), crcp1(aL));
  cx<T> Mp, Wp;
  if (ML.r > T(1)) { Mp = ML; Wp = one; }
  else if (ML.r < T(-1)) { Mp = cx<T>{T(0), T(0)}; Wp = cx<T>{T(0), T(0)}; }
  else {
    const cx<T> s = ML + one;
    Mp = T(0.25) * cmul1(s, s);
    Wp = cmul1(Mp, T(2) * one - ML);
  }
  // high side: "-" splits
  const cx<T> aR = csqrt1((etann * gred) * HR);
  const cx<T> MR = cmul1(cmul1(n == 0 ? R1 : R2, crcp1(HR)), crcp1(aR));
  cx<T> Mm, Wm;
  if (MR.r < T(-1)) { Mm = MR; Wm = one; }
  else if (MR.r > T(1)) { Mm = cx<T>{T(0), T(0)}; Wm = cx<T>{T(0), T(0)}; }
  else {
    const cx<T> s = MR - one;
    Mm = T(-0.25) * cmul1(s, s);
    Wm = cmul1(-Mm, T(2) * one + MR);
  }
  const cx<T> m = Mp + Mm;   // Eq. (138) across the face
  // Eqs. (140)-(143): max[0, m] A^+ + min[0, m] A^- + P^+ + P^-
  const bool low = m.r >= T(0);
  const cx<T> a = low ? aL : aR;
  const cx<T> ma = cmul1(m, a);
  const cx<T> PL = (T(0.5) * gred) * cmul1(HL, HL), PR = (T(0.5) * gred) * cmul1(HR, HR);
  const cx<T> wP = cmul1(Wp, PL), wQ = cmul1(Wm, PR);
  F0 = cmul1(ma, low ? HL : HR);
  F1 = cmul1(ma, low ? L1 : R1) + eta1n * (wP + wQ);
  F2 = cmul1(ma, low ? L2 : R2) + eta2n * (wP + wQ);
}

// ---------------------------------------------------------------------------
// The fused DFR kernel.  A block takes a tile of TX x TY elements of one panel
// (TX, TY divide ne), one thread per GL node.
//
// The discrete operator is linear in the fluxes once they are formed: the
// derivative of Eq. (12), the extrapolation of Eq. (7) and the face terms.  Of
// the complex evaluation only one part is kept through these stages, the
// "linear lane": Im for the complex-step product (its result is Im F / eps),
// Re for F itself.  The states extrapolated to the faces keep both parts,
// since the Rusanov flux is nonlinear in them.
//  A  (per node): metric terms from 1-D tangent tables (App. B), nodal fluxes
//     (Eq. 136, linear lane) and sources (Eq. 2, linear lane); the state (both
//     parts) to LDS.  Then, per face point of the tile's neighbours, the
//     neighbour's state extrapolated to the shared face, from global memory.
//  B  (per node): interior part of the extended-point derivative of Eq. (12)
//     in both directions, in registers; (per element row / column) the own
//     states extrapolated to both faces of the row / column.
//  C  (per face point of the tile, each face once): App. C map of the
//     neighbour's momentum at panel edges, Rusanov common flux.
//  D  (per node): face terms of Eq. (12), sources, division by sqrt(g);
//     output, optionally with the Arnoldi epilogue.
constexpr int DFR_MAX_THREADS = 1024;

// one face of the tile, set up once per workgroup
struct FaceDesc {
  int lo, hi;   // trace slots of the two sides: own el*4+face, or 4*nel + halo
  int xf;       // App. C table offset ((panel*4 + halo face)*ne + along)*NS, or -1
  int info;     // bit 0: normal direction (0: x^1, 1: x^2); bit 1: map the lo side, bit 2: the hi side
  int eedge;    // face line index in the edge-tangent table
  int enode;    // element index along the face in the node-tangent table
};

// one neighbour element line of the tile's halo, set up once per workgroup:
// the neighbour's node index (in one field) of the line through face point
// 0, the index steps to the next face point and along the line, and which
// end of the line the shared face is
struct HaloDesc {
  int base, tstep, kstep, lo;
};

// LDS layout of the tiled kernel, in values of the compute type T:
// state [nel][3][NN][L], fluxes [nel][5][NN] (reused for the common fluxes
// [nface*NS][3]), traces [4 nel + nhalo][3][NS][L], face table, halo table.
struct DfrLds {
  int state, flux, trace, faces, halo, total;
};
__host__ __device__ inline DfrLds dfr_lds_layout(int ns, int tx, int ty, int lanes, int tsize) {
  const int nn = ns * ns, nel = tx * ty, nhalo = 2 * (tx + ty);
  const int nface = (tx + 1) * ty + (ty + 1) * tx;
  DfrLds l;
  l.state = 0;
  l.flux = nel * 3 * nn * lanes;
  const int nflux = std::max(nel * 5 * nn, nface * ns * 3);
  l.trace = l.flux + nflux;
  l.faces = l.trace + (4 * nel + nhalo) * 3 * ns * lanes;
  const int fvals = (nface * (int)sizeof(FaceDesc) + tsize - 1) / tsize;
  l.halo = l.faces + fvals;
  const int hvals = (nhalo * (int)sizeof(HaloDesc) + tsize - 1) / tsize;
  l.total = l.halo + hvals;
  return l;
}

template <typename T, bool CS>
__device__ __forceinline__ T lin(cx<T> z) {
  if constexpr (CS) return z.i;
  else return z.r;
}

// The kernel body: tile `lb` (0 <= lb < 6 (ne/TX)(ne/TY)) of the grid
// described by g.  Its partial inner products (Krylov form) go to
// ar.pout[2 lb], ar.pout[2 lb + 1]; tile 0 records the prologue's values.
template <int NS, typename T, typename TQ, bool CS, bool AR, int RS, typename TV>
__device__ __forceinline__ void dfr_body(const GridArgs &g, const Ops1D &ops, const int TX, const int TY, const int lb,
                                         const TQ *__restrict__ q, const TV *__restrict__ v,
                                         const double *__restrict__ vscale, double eps, TV *__restrict__ out,
                                         const ArnoldiArgs &ar) {
  constexpr int NN = NS * NS;
  constexpr int L = CS ? 2 : 1;   // parts kept of a state value
  extern __shared__ double dyn[];
  __shared__ T sD[NS][NS + 2];
  __shared__ T slm[NS], slp[NS];
  __shared__ double red[256];

  const int tid = threadIdx.x;
  const int ne = g.ne;
  const int N = (int)g.n;
  const int ntx = ne / TX, nty = ne / TY;
  const int nel = TX * TY;
  const int nhalo = 2 * (TX + TY);
  const int nvf = (TX + 1) * TY;
  const int nface = nvf + (TY + 1) * TX;
  const DfrLds lay = dfr_lds_layout(NS, TX, TY, L, (int)sizeof(T));
  T *S = reinterpret_cast<T *>(dyn) + lay.state;
  T *Fl = reinterpret_cast<T *>(dyn) + lay.flux;
  T *TR = reinterpret_cast<T *>(dyn) + lay.trace;
  FaceDesc *FD = reinterpret_cast<FaceDesc *>(reinterpret_cast<T *>(dyn) + lay.faces);
  HaloDesc *HD = reinterpret_cast<HaloDesc *>(reinterpret_cast<T *>(dyn) + lay.halo);
  // the state and direction streams (3N values each) and the output
  const uint32_t n3 = 3u * (uint32_t)N;
  const rsrc_t rq = make_rsrc(q, n3 * (uint32_t)sizeof(TQ));
  const rsrc_t rv = make_rsrc(CS ? (const void *)v : (const void *)q, n3 * (uint32_t)sizeof(TV));
  const rsrc_t ro = make_rsrc(out, n3 * (uint32_t)sizeof(TV));
  // the complex step in the compute type: z = q + i epsT v, and the result
  // Im F / epsT (epsT = eps in FP64; the FP32 value nearest eps in FP32)
  const T epsT = (T)eps;
  const double invE = CS ? 1.0 / (double)epsT : 1.0;

  // The direction enters unscaled: J (sigma v) = sigma J v, the scale sigma
  // (vscale, or the Arnoldi sigma_j) multiplies the result.  In Arnoldi mode
  // the loads of the previous kernel's partial sums are issued here and the
  // reduction finished after phase A, off the critical path (blockDim >= 256,
  // np_in <= 1024: one virtual lane of reduce_fixed per thread tid < 256,
  // summed in the same order).
  __shared__ double ssig;         // sigma_j
  __shared__ int shappy;          // happy breakdown found by this kernel's prologue
  int happy0 = 0;
  double pv[4] = {0.0, 0.0, 0.0, 0.0};
  if constexpr (AR) {
    happy0 = gmem(ar.kd)->happy;
    if (tid < 256) {
#pragma unroll
      for (int k = 0; k < 4; ++k)
        if (tid + 256 * k < ar.np_in) pv[k] = gmem(ar.pin)[tid + 256 * k];
    }
  }
  const double vs_in = (!AR && CS && vscale) ? *vscale : 1.0;
  const int p = lb / (ntx * nty);
  const int trow = (lb - p * ntx * nty) / ntx;
  const int tcol = lb - p * ntx * nty - trow * ntx;
  const int ej0 = trow * TY, ei0 = tcol * TX;

  {
    // the 1-D operators to LDS: each thread's first entry and its lm / lp
    // entries loaded together (one round trip), then any further entries
    constexpr int ND = NS * (NS + 2);
    const int k0 = min(tid, ND - 1), t0 = min(tid, NS - 1);
    const double d0 = ops.Dt[k0 / (NS + 2)][k0 % (NS + 2)], m0 = ops.lm[t0], p0 = ops.lp[t0];
    if (tid < ND) sD[k0 / (NS + 2)][k0 % (NS + 2)] = (T)d0;
    if (tid < NS) {
      slm[tid] = (T)m0;
      slp[tid] = (T)p0;
    }
    for (int k = tid + (int)blockDim.x; k < ND; k += blockDim.x) sD[k / (NS + 2)][k % (NS + 2)] = (T)ops.Dt[k / (NS + 2)][k % (NS + 2)];
  }
  // face table: vertical faces (x^1 normal) id = fx*TY + row, fx = 0..TX;
  // then horizontal faces id = nvf + fy*TX + col, fy = 0..TY.  Halo slots:
  // [0,TY) west, [TY,2TY) east, [2TY,2TY+TX) south, then north.
  for (int id = tid; id < nface; id += blockDim.x) {
    FaceDesc d;
    const int h0 = 4 * nel;
    if (id < nvf) {
      const int fx = id / TY, row = id - fx * TY;
      d.lo = fx > 0 ? (row * TX + fx - 1) * 4 + 1 : h0 + row;
      d.hi = fx < TX ? (row * TX + fx) * 4 + 0 : h0 + TY + row;
      d.eedge = ei0 + fx;
      d.enode = ej0 + row;
      d.info = 0;
      d.xf = -1;
      if (fx == 0 && ei0 == 0) { d.info |= 2; d.xf = ((p * 4 + 0) * ne + ej0 + row) * NS; }
      if (fx == TX && ei0 + TX == ne) { d.info |= 4; d.xf = ((p * 4 + 1) * ne + ej0 + row) * NS; }
    } else {
      const int k = id - nvf;
      const int fy = k / TX, col = k - fy * TX;
      d.lo = fy > 0 ? ((fy - 1) * TX + col) * 4 + 3 : h0 + 2 * TY + col;
      d.hi = fy < TY ? (fy * TX + col) * 4 + 2 : h0 + 2 * TY + TX + col;
      d.eedge = ej0 + fy;
      d.enode = ei0 + col;
      d.info = 1;
      d.xf = -1;
      if (fy == 0 && ej0 == 0) { d.info |= 2; d.xf = ((p * 4 + 2) * ne + ei0 + col) * NS; }
      if (fy == TY && ej0 + TY == ne) { d.info |= 4; d.xf = ((p * 4 + 3) * ne + ei0 + col) * NS; }
    }
    FD[id] = d;
  }
  // halo table: slots [0,TY) west, [TY,2TY) east, [2TY,2TY+TX) south, then
  // north; across a panel edge the neighbour's face, element and line order
  // come from the connectivity of App. C
  for (int h = tid; h < nhalo; h += blockDim.x) {
    int face, ai;
    if (h < TY) { face = 0; ai = h; }
    else if (h < 2 * TY) { face = 1; ai = h - TY; }
    else if (h < 2 * TY + TX) { face = 2; ai = h - 2 * TY; }
    else { face = 3; ai = h - 2 * TY - TX; }
    int qp = p, qe, qi, qf, rev = 0;
    if (face == 0) { qe = ej0 + ai; qi = ei0 - 1; qf = 1; }
    else if (face == 1) { qe = ej0 + ai; qi = ei0 + TX; qf = 0; }
    else if (face == 2) { qi = ei0 + ai; qe = ej0 - 1; qf = 3; }
    else { qi = ei0 + ai; qe = ej0 + TY; qf = 2; }
    if (qi < 0 || qi >= ne || qe < 0 || qe >= ne) {   // across a panel edge
      const int along = (face < 2) ? ej0 + ai : ei0 + ai;
      qp = g.nb_q[p][face];
      qf = g.nb_e[p][face];
      rev = g.nb_rev[p][face];
      const int qa = rev ? ne - 1 - along : along;
      if (qf == 0) { qi = 0; qe = qa; }
      else if (qf == 1) { qi = ne - 1; qe = qa; }
      else if (qf == 2) { qe = 0; qi = qa; }
      else { qe = ne - 1; qi = qa; }
    }
    // face point t of the shared face is the neighbour's line qt = t (or
    // NS-1-t when the orders oppose): a node row (x^1 faces) or column
    const int t0 = rev ? NS - 1 : 0;
    HaloDesc hd;
    hd.base = ((qp * ne + qe) * ne + qi) * NN + ((qf < 2) ? t0 * NS : t0);
    hd.tstep = (rev ? -1 : 1) * ((qf < 2) ? NS : 1);
    hd.kstep = (qf < 2) ? 1 : NS;
    hd.lo = (qf == 0 || qf == 2) ? 1 : 0;
    HD[h] = hd;
  }

  const int s = tid / NN, node = tid - s * NN, nj = node / NS, ni = node - nj * NS;
  const bool active = s < nel;
  const int sy = s / TX, sx = s - sy * TX;
  const int ei = ei0 + sx, ej = ej0 + sy;
  const int gidx = ((p * ne + ej) * ne + ei) * NN + node;
  const T gred = (T)g.g_red;

  T src1 = T(0), src2 = T(0);
  T rs = T(0);
  double vtrue[3] = {0.0, 0.0, 0.0};
  // Arnoldi: the b-column combination of the augmented operator and the
  // previous basis vector are read here, in flight during the computation.
  // With the unnormalised bottom block u_j (the start vector's mu y, or the
  // one left by the previous update), w_j = sigma_j (J v~_j + W u_j).
  double wb[3] = {0.0, 0.0, 0.0}, vp[3] = {0.0, 0.0, 0.0};
  if (AR && active) {
    const auto ub = gmem(ar.kd->botu) + ar.j * MAX_P;
    const double sp = ar.vprev ? gmem(ar.kd->sigma)[ar.j - 1] : 0.0;   // v_{j-1} = sigma_{j-1} v~_{j-1}
    double uw[4];   // the bottom entries paired with the interleaved columns (0 beyond p)
#pragma unroll
    for (int k = 0; k < 4; ++k) uw[k] = k < ar.p ? (ar.start ? ar.ybot[k] : ub[k]) : 0.0;
    if (ar.wil) {
      // four interleaved columns: every load of the three fields first (one
      // memory round trip), then the sums.  Without a previous vector the
      // direction v is read for a zero term.
      const rsrc_t rp = make_rsrc(ar.vprev ? ar.vprev : (const void *)v, n3 * (uint32_t)sizeof(TV));
      double pv[3];
      if constexpr (std::is_same<TV, float>::value) {
        // FP32 basis: the columns are kept in FP32 too (what they feed is
        // rounded to FP32 when stored), one 16-byte load per value
        // (three per value when p <= 3, one 12-byte load; else four)
        const bool w3 = ar.wil == 3;
        const rsrc_t rw = make_rsrc(ar.W[0], n3 * (w3 ? 12u : 16u));
        float4 x[3];
#pragma unroll
        for (int f = 0; f < 3; ++f) {
          const uint32_t id = (uint32_t)(f * N + gidx);
          x[f] = w3 ? bload3f(rw, id) : bload4f(rw, id);
          pv[f] = (double)bload<TV>(rp, id);
        }
#pragma unroll
        for (int f = 0; f < 3; ++f) {
          wb[f] = (((double)x[f].x * uw[0] + (double)x[f].y * uw[1]) + (double)x[f].z * uw[2]) +
                  (double)x[f].w * uw[3];
          vp[f] = sp * pv[f];
        }
      } else {
        // FP64: two 16-byte loads per value
        const rsrc_t rw = make_rsrc(ar.W[0], n3 * 32u);
        double2 x0[3], x1[3];
#pragma unroll
        for (int f = 0; f < 3; ++f) {
          const uint32_t id = (uint32_t)(f * N + gidx);
          x0[f] = bload2(rw, 4u * id);
          x1[f] = bload2(rw, 4u * id + 2u);
          pv[f] = (double)bload<TV>(rp, id);
        }
#pragma unroll
        for (int f = 0; f < 3; ++f) {
          wb[f] = ((x0[f].x * uw[0] + x0[f].y * uw[1]) + x1[f].x * uw[2]) + x1[f].y * uw[3];
          vp[f] = sp * pv[f];
        }
      }
    } else {
#pragma unroll
      for (int f = 0; f < 3; ++f) {
        const int id = f * N + gidx;
        double a = 0.0;
        for (int k = 0; k < ar.p; ++k) a += gmem(ar.W[k])[id] * (ar.start ? ar.ybot[k] : ub[k]);
        wb[f] = a;
        if (ar.vprev) vp[f] = sp * (double)static_cast<const TV *>(ar.vprev)[id];
      }
    }
  }

  // ---- A: state, nodal fluxes, sources
  if (active) {
    const Tan3 tx = ld_tan3(g.tnode, ei * NS + ni), ty = ld_tan3(g.tnode, ej * NS + nj);
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
      const T qr = (T)bload<TQ>(rq, (uint32_t)(f * N + gidx));
      T qi = T(0);
      if constexpr (CS) {
        const TV vv = bload<TV>(rv, (uint32_t)(f * N + gidx));
        vtrue[f] = (double)vv;
        qi = epsT * (T)vv;
      }
      Qz[f] = {qr, qi};
      T *sp = S + ((s * 3 + f) * NN + node) * L;
      sp[0] = qr;
      if constexpr (CS) sp[1] = qi;
    }
    const cx<T> H = Qz[0], M1 = Qz[1], M2 = Qz[2];
    if (!(H.r > T(0))) atomicOr(g.err_flag, 2);
    const cx<T> rH = crcp1(H);
    const cx<T> u1 = cmul1(M1, rH), u2 = cmul1(M2, rH);
    const T H2h = lin<T, CS>((T(0.5) * gred) * cmul1(H, H));
    const T m11 = lin<T, CS>(cmul1(M1, u1)), m12 = lin<T, CS>(cmul1(M1, u2)), m22 = lin<T, CS>(cmul1(M2, u2));
    const T l1 = lin<T, CS>(M1), l2 = lin<T, CS>(M2), lH = lin<T, CS>(H);
    T *fp = Fl + s * 5 * NN + node;
    fp[0 * NN] = sg * l1;                      // x^1 flux of H
    fp[1 * NN] = sg * (m11 + e11 * H2h);       // x^1 flux of H u^1
    fp[2 * NN] = sg * (m12 + e12 * H2h);       // x^1 flux of H u^2 = x^2 flux of H u^1
    fp[3 * NN] = sg * l2;                      // x^2 flux of H
    fp[4 * NN] = sg * (m22 + e22 * H2h);       // x^2 flux of H u^2
    // sources per unit sqrt(g): Coriolis -2 Gamma^i_0j H u^j, metric -Gamma^i_jk H u^j u^k
    // (the h^jk Gamma^i_jk term vanishes identically on the cubed sphere, App. B)
    src1 = -(T(2) * (G101 * l1 + G102 * l2) + (G111 * m11 + (T(2) * G112) * m12));
    src2 = -(T(2) * (G201 * l1 + G202 * l2) + ((T(2) * G212) * m12 + G222 * m22));
    if (g.orog) {
      src1 -= (T)gmem(g.orog)[gidx] * lH;
      src2 -= (T)gmem(g.orog)[N + gidx] * lH;
    }
  }
  if constexpr (AR) {
    if (happy0) return;   // uniform: the sub-step ended in a happy breakdown
    if (tid < 256) red[tid] = ((pv[0] + pv[1]) + pv[2]) + pv[3];
  }
  __syncthreads();
  if (AR && tid < 64) {
    // finish the reduction (the fixed butterfly of reduce_fixed) and the
    // prologue in the first wave; the results are read after two barriers
    const double x = wave_sum((red[tid] + red[tid + 64]) + (red[tid + 128] + red[tid + 192]));
    double sg_, bj[MAX_P];
    const bool ok = arnoldi_finish(ar, x, tid, 64, lb == 0, sg_, bj);
    if (tid == 0) {
      shappy = ok ? 0 : 1;
      ssig = sg_;
    }
  }

  // ---- B: the neighbours' states extrapolated to the faces they share with
  // the tile (Eq. 7), task = (h * 3 + f) * NS + t: the loads of this thread's
  // first task go out first and are used after the interior derivative and
  // the own traces, which read only LDS
  const int nhtask = nhalo * 3 * NS;
  T hz[NS], hzi[NS];
  int hdst = -1, hlo = 1;
  if (tid < nhtask) {
    const int t = tid % NS, r = tid / NS;
    const int f = r % 3, h = r / 3;
    const HaloDesc hd = HD[h];
    const uint32_t id0 = (uint32_t)(f * N + hd.base + t * hd.tstep);
#pragma unroll
    for (int k = 0; k < NS; ++k) {
      hz[k] = (T)bload<TQ>(rq, id0 + (uint32_t)(k * hd.kstep));
      if constexpr (CS) hzi[k] = (T)bload<TV>(rv, id0 + (uint32_t)(k * hd.kstep));
    }
    hlo = hd.lo;
    hdst = (((4 * nel + h) * 3 + f) * NS + t) * L;
  }

  // ---- B: interior part of the derivative (linear lane), both directions
  T acc[3] = {T(0), T(0), T(0)};
  if (active) {
    const T *fp = Fl + s * 5 * NN;
    T d0 = T(0), d1 = T(0), d2 = T(0);
#pragma unroll
    for (int k = 0; k < NS; ++k) {
      const T cxk = sD[ni][k + 1], cyk = sD[nj][k + 1];
      const int ix = nj * NS + k, iy = k * NS + ni;
      d0 += cxk * fp[0 * NN + ix] + cyk * fp[3 * NN + iy];
      d1 += cxk * fp[1 * NN + ix] + cyk * fp[2 * NN + iy];
      d2 += cxk * fp[2 * NN + ix] + cyk * fp[4 * NN + iy];
    }
    acc[0] = d0;
    acc[1] = d1;
    acc[2] = d2;
  }
  // own states extrapolated to both faces of each row (dir 0: W, E) and
  // column (dir 1: S, N): task = ((es * 2 + dir) * 3 + f) * NS + t
  for (int task = tid; task < nel * 6 * NS; task += blockDim.x) {
    const int t = task % NS;
    const int r = task / NS;
    const int f = r % 3;
    const int r2 = r / 3;
    const int dir = r2 & 1, es = r2 >> 1;
    const T *sp = S + ((es * 3 + f) * NN + (dir == 0 ? t * NS : t)) * L;
    const int st = (dir == 0 ? 1 : NS) * L;
    T lr = T(0), li = T(0), hr = T(0), hi = T(0);
#pragma unroll
    for (int k = 0; k < NS; ++k) {
      const T zr = sp[k * st];
      lr += slm[k] * zr;
      hr += slp[k] * zr;
      if constexpr (CS) {
        const T zi = sp[k * st + 1];
        li += slm[k] * zi;
        hi += slp[k] * zi;
      }
    }
    T *lo = TR + (((es * 4 + 2 * dir) * 3 + f) * NS + t) * L;
    T *up = TR + (((es * 4 + 2 * dir + 1) * 3 + f) * NS + t) * L;
    lo[0] = lr;
    up[0] = hr;
    if constexpr (CS) {
      lo[1] = li;
      up[1] = hi;
    }
  }
  // the halo extrapolation: the first task from the loads above, any
  // further ones (large tiles) in turn; eps multiplies each sum once
  if (hdst >= 0) {
    T a = T(0), b = T(0);
#pragma unroll
    for (int k = 0; k < NS; ++k) {
      const T wk = hlo ? slm[k] : slp[k];
      a += wk * hz[k];
      if constexpr (CS) b += wk * hzi[k];
    }
    TR[hdst] = a;
    if constexpr (CS) TR[hdst + 1] = epsT * b;
  }
  for (int task = tid + (int)blockDim.x; task < nhtask; task += blockDim.x) {
    const int t = task % NS, r = task / NS;
    const int f = r % 3, h = r / 3;
    const HaloDesc hd = HD[h];
    const uint32_t id0 = (uint32_t)(f * N + hd.base + t * hd.tstep);
    T a = T(0), b = T(0);
#pragma unroll
    for (int k = 0; k < NS; ++k) {
      const T wk = hd.lo ? slm[k] : slp[k];
      a += wk * (T)bload<TQ>(rq, id0 + (uint32_t)(k * hd.kstep));
      if constexpr (CS) b += wk * (T)bload<TV>(rv, id0 + (uint32_t)(k * hd.kstep));
    }
    T *tp = TR + (((4 * nel + h) * 3 + f) * NS + t) * L;
    tp[0] = a;
    if constexpr (CS) tp[1] = epsT * b;
  }
  __syncthreads();

  if (AR && shappy) return;   // uniform: happy breakdown found above

  // ---- C: common fluxes, each face point of the tile once (linear lane) ->
  // Fl[(face * NS + t) * 3 + f]
  for (int task = tid; task < nface * NS; task += blockDim.x) {
    const int fid = task / NS, t = task - fid * NS;
    const FaceDesc d = FD[fid];
    const int n = d.info & 1;
    auto ld_tr = [&](int slot, int f) -> cx<T> {
      const T *a = TR + ((slot * 3 + f) * NS + t) * L;
      return {a[0], CS ? a[L - 1] : T(0)};
    };
    const cx<T> HL = ld_tr(d.lo, 0), HR = ld_tr(d.hi, 0);
    cx<T> L1 = ld_tr(d.lo, 1), L2 = ld_tr(d.lo, 2), R1 = ld_tr(d.hi, 1), R2 = ld_tr(d.hi, 2);
    if (d.xf >= 0) {
      // App. C: the neighbour's components -> this panel's basis
      const auto M = gmem(g.xform) + (int64_t)(d.xf + t) * 4;
      const T m00 = (T)M[0], m01 = (T)M[1], m10 = (T)M[2], m11 = (T)M[3];
      if (d.info & 2) {
        const cx<T> a1 = m00 * L1 + m01 * L2, a2 = m10 * L1 + m11 * L2;
        L1 = a1;
        L2 = a2;
      } else {
        const cx<T> a1 = m00 * R1 + m01 * R2, a2 = m10 * R1 + m11 * R2;
        R1 = a1;
        R2 = a2;
      }
    }
    // metric at the face point
    T X, Y, ax, ay, rax, ray;
    if (n == 0) {
      X = (T)gmem(g.tedge)[d.eedge]; ax = T(1) + X * X; rax = frcp(ax);
      const Tan3 ty = ld_tan3(g.tnode, d.enode * NS + t);
      Y = (T)ty.x; ay = (T)ty.ax; ray = (T)ty.rax;
    } else {
      const Tan3 tx = ld_tan3(g.tnode, d.enode * NS + t);
      X = (T)tx.x; ax = (T)tx.ax; rax = (T)tx.rax;
      Y = (T)gmem(g.tedge)[d.eedge]; ay = T(1) + Y * Y; ray = frcp(ay);
    }
    const T d2 = ax + Y * Y;
    const T rd = frsqrt(d2);
    const T sg = ax * ay * rd * rd * rd;
    const T e11 = d2 * rax, e22 = d2 * ray, e12 = X * Y * e11 * ray;
    const T eta1n = n == 0 ? e11 : e12, eta2n = n == 0 ? e12 : e22, etann = n == 0 ? e11 : e22;
    T *cf = Fl + task * 3;
    if constexpr (RS == 1) {   // AUSM
      cx<T> F0, F1, F2;
      ausm_flux(HL, L1, L2, HR, R1, R2, n, eta1n, eta2n, etann, gred, F0, F1, F2);
      cf[0] = sg * lin<T, CS>(F0);
      cf[1] = sg * lin<T, CS>(F1);
      cf[2] = sg * lin<T, CS>(F2);
    } else {
      cx<T> fL0, fL1, fL2, fR0, fR1, fR2, cL, cR;
      side_flux1(HL, L1, L2, n == 0 ? L1 : L2, eta1n, eta2n, etann, gred, fL0, fL1, fL2, cL);
      side_flux1(HR, R1, R2, n == 0 ? R1 : R2, eta1n, eta2n, etann, gred, fR0, fR1, fR2, cR);
      const cx<T> lam = (cL.r >= cR.r) ? cL : cR;
      const T hs = T(0.5) * sg;
      cf[0] = hs * lin<T, CS>((fL0 + fR0) - cmul1(lam, HR - HL));
      cf[1] = hs * lin<T, CS>((fL1 + fR1) - cmul1(lam, R1 - L1));
      cf[2] = hs * lin<T, CS>((fL2 + fR2) - cmul1(lam, R2 - L2));
    }
  }
  __syncthreads();

  // ---- D: face terms, sources, output
  double w[3] = {0.0, 0.0, 0.0};
  double wr[3] = {0.0, 0.0, 0.0};   // Im F / (eps sigma) in FP64, Arnoldi form
  const double vs = AR ? ssig : vs_in;
  if (active) {
    const T scale = -(T)g.two_over_delta * rs;
    const int iW = ((sx * TY + sy) * NS + nj) * 3, iE = (((sx + 1) * TY + sy) * NS + nj) * 3;
    const int iS = ((nvf + sy * TX + sx) * NS + ni) * 3, iN = ((nvf + (sy + 1) * TX + sx) * NS + ni) * 3;
    const T cw = sD[ni][0], ce = sD[ni][NS + 1], cs = sD[nj][0], cn = sD[nj][NS + 1];
#pragma unroll
    for (int f = 0; f < 3; ++f) {
      T d = acc[f] + cw * Fl[iW + f] + ce * Fl[iE + f] + cs * Fl[iS + f] + cn * Fl[iN + f];
      T r = scale * d;
      if (f == 1) r += src1;
      if (f == 2) r += src2;
      w[f] = CS ? ((double)r * invE) * vs : (double)r;
      wr[f] = (double)r;
    }
    if constexpr (!AR) {
#pragma unroll
      for (int f = 0; f < 3; ++f) bstore<TV>(ro, (uint32_t)(f * N + gidx), (TV)w[f]);
    }
  }
  if constexpr (!AR) return;

  // ---- Arnoldi epilogue: w = sigma_j (J v~_j + W u_j); partial <v_j, w>, <v_{j-1}, w>
  double d0 = 0.0, d1 = 0.0;
  if (active) {
#pragma unroll
    for (int f = 0; f < 3; ++f) {
      // the inner products use the value as stored (rounded to the basis type)
      const TV a = (TV)(vs * (wr[f] * invE + wb[f]));
      bstore<TV>(ro, (uint32_t)(f * N + gidx), a);
      d0 += (double)a * (vs * vtrue[f]);
      d1 += (double)a * vp[f];
    }
  }
  block_sum2(d0, d1, red);
  if (tid == 0) {
    ar.pout[lb * 2 + 0] = d0;
    ar.pout[lb * 2 + 1] = d1;
  }
}

// Waves per SIMD asked of the product kernels: the complex-FP32 forms with up
// to seven GL points fit the registers of six waves without spilling (80
// VGPRs, against 77-90 left to themselves at five or six), which shortened
// the ensemble's batched products by 12% and sped up EPI6 at ne 120 with
// FP32 products and basis by 17%; the FP64 forms and eight points would
// spill there (a five-wave bound slowed the plain FP64 J*v by 11%) and keep
// the compiler's choice (1: no bound).
template <int NS, typename T>
constexpr int product_waves_per_eu() {
  return (std::is_same<T, float>::value && NS <= 7) ? 6 : 1;
}

// one grid: the logical blocks are its tiles (XCD-aware order), the grid
// rounded up to whole groups of eight workgroups; RS: the common flux
// (0 Rusanov, 1 AUSM), a template argument so that each kernel keeps the
// registers of its own flux
template <int NS, typename T, typename TQ, bool CS, bool AR, int RS, typename TV>
__global__ __launch_bounds__(DFR_MAX_THREADS) __attribute__((amdgpu_waves_per_eu(product_waves_per_eu<NS, T>())))
void dfr_kernel(const GridArgs g, const Ops1D ops, const int TX,
                                                               const int TY, const TQ *__restrict__ q,
                                                               const TV *__restrict__ v,
                                                               const double *__restrict__ vscale, double eps,
                                                               TV *__restrict__ out, const ArnoldiArgs ar) {
  const int lb = (int)logical_block(6 * (g.ne / TX) * (g.ne / TY));
  if (lb < 0) return;   // uniform: padding workgroup of the XCD mapping
  dfr_body<NS, T, TQ, CS, AR, RS, TV>(g, ops, TX, TY, lb, q, v, vscale, eps, out, ar);
}

// several grids (ensemble members) in one launch: member m owns the logical
// blocks [b0, b0 + ntiles); Rusanov fluxes; TV: the basis type.  dc: NULL,
// or the number of calls and of logical blocks in device memory (written by
// the round planner; the grid is sized for every member)
template <int NS, typename T, typename TQ, bool CS, bool AR, typename TV>
__global__ __launch_bounds__(DFR_MAX_THREADS) __attribute__((amdgpu_waves_per_eu(product_waves_per_eu<NS, T>())))
void dfr_kernel_batch(const DfrCall *__restrict__ calls, int ncalls,
                                                                     int nlogical, const int *__restrict__ dc) {
  __shared__ int s_m;
  if (dc) {
    ncalls = dc[0];
    nlogical = dc[1];
  }
  const int lbg = (int)logical_block(nlogical);
  if (lbg < 0) return;   // uniform
  for (int t = threadIdx.x; t < ncalls; t += blockDim.x) {
    const int b0 = calls[t].b0;
    if (lbg >= b0 && lbg < b0 + calls[t].ntiles) s_m = t;
  }
  __syncthreads();
  // the member's call, at a workgroup-uniform index (scalar loads)
  const DfrCall &c = calls[__builtin_amdgcn_readfirstlane(s_m)];
  dfr_body<NS, T, TQ, CS, AR, 0, TV>(*c.g, *c.ops, c.TX, c.TY, lbg - c.b0, reinterpret_cast<const TQ *>(c.q),
                                     static_cast<const TV *>(c.v), c.vscale, c.eps, static_cast<TV *>(c.out), c.ar);
}

// ---------------------------------------------------------------------------
// Vector kernels of the Krylov iteration.  Each is a body run by workgroup
// `blk` of `nblk` (grid-stride over its vector), with two entry points: one
// vector (blk = blockIdx.x), or a batch of members' vectors in one launch
// (member m owns the workgroups [b0, b0 + nblk); find_call locates it).

template <typename C>
__device__ __forceinline__ int find_call_at(const C *__restrict__ calls, int ncalls, int b) {
  __shared__ int s_m;
  for (int t = threadIdx.x; t < ncalls; t += blockDim.x) {
    const int b0 = calls[t].b0;
    if (b >= b0 && b < b0 + calls[t].nblk) s_m = t;
  }
  __syncthreads();
  return __builtin_amdgcn_readfirstlane(s_m);
}
template <typename C>
__device__ __forceinline__ int find_call(const C *__restrict__ calls, int ncalls) {
  return find_call_at(calls, ncalls, (int)blockIdx.x);
}

// first Arnoldi step of a sub-step whose top block is identically zero:
// w = W b_0 (no J v); both partial inner products vanish
template <typename TV>
__device__ __forceinline__ void arnoldi_first_body(int blk, int nblk, int64_t n3, const ArnoldiArgs &ar, TV *out) {
  __shared__ double red[256];
  if (ar.kd->happy) return;
  double sig, bj[MAX_P];
  if (!arnoldi_prologue(ar, red, blk == 0, sig, bj)) return;
  for (int64_t i = (int64_t)blk * BLOCK + threadIdx.x; i < n3; i += (int64_t)nblk * BLOCK) {
    double acc = 0.0;
    if (ar.wil) {
      if constexpr (std::is_same<TV, float>::value) {   // FP32 columns with an FP32 basis
        const float *w = reinterpret_cast<const float *>(ar.W[0]) + (ar.wil == 3 ? 3 : 4) * i;
        for (int k = 0; k < ar.p; ++k) acc += (double)w[k] * bj[k];
      } else {
        const double *w = ar.W[0] + 4 * i;
        for (int k = 0; k < ar.p; ++k) acc += w[k] * bj[k];
      }
    } else {
      for (int k = 0; k < ar.p; ++k) acc += ar.W[k][i] * bj[k];
    }
    out[i] = (TV)acc;
  }
  if (threadIdx.x == 0) {
    ar.pout[blk * 2 + 0] = 0.0;
    ar.pout[blk * 2 + 1] = 0.0;
  }
}
template <typename TV>
__global__ __launch_bounds__(BLOCK) void arnoldi_first_kernel(int64_t n3, const ArnoldiArgs ar, TV *out) {
  arnoldi_first_body(blockIdx.x, gridDim.x, n3, ar, out);
}
// dc: NULL (one workgroup per block of the calls), or the number of calls
// and blocks in device memory; then each workgroup takes the blocks
// blockIdx.x, blockIdx.x + gridDim.x, ... (a grid of fixed size for any count)
template <typename TV>
__global__ __launch_bounds__(BLOCK) void arnoldi_first_batch(const FirstCall *__restrict__ calls, int ncalls,
                                                  const int *__restrict__ dc) {
  const int total = dc ? dc[1] : (int)gridDim.x;
  if (dc) ncalls = dc[0];
  for (int lb = blockIdx.x; lb < total; lb += gridDim.x) {
    __syncthreads();   // the previous block's use of shared memory
    const FirstCall &c = calls[find_call_at(calls, ncalls, lb)];
    arnoldi_first_body(lb - c.b0, c.nblk, c.n3, c.ar, static_cast<TV *>(c.out));
  }
}

// Gram-Schmidt step.  Prologue: the inner products h_{j,j}, h_{j-1,j} (top
// partials of the J v kernel plus the bottom blocks; classical Gram-Schmidt
// over the last two vectors) and the new bottom block, recorded by workgroup
// 0.  Body: w <- w - h_jj sigma_j v~_j - h_{j-1,j} sigma_{j-1} v~_{j-1};
// partial ||w||^2 per workgroup.  Basis vectors stay as built (v~_k), their
// scales sigma_k kept in KDev.  The first UNROLL elements of each thread are
// read before the prologue, in flight during its reductions.  With !two the
// third stream rereads v~_j, multiplied by a zero coefficient.
template <typename TV, int UNROLL, int MP = MAX_P>
__device__ __forceinline__ void arnoldi_update_body(int blk, int nblk, int64_t n3, int j, int p, TV *w,
                                                    const TV *vj, const TV *vprev, const double *pin,
                                                    int np_in, double *pout, KDev *kd) {
  // UNROLL grid strides per chunk: a chunk's loads are issued together (one
  // memory round trip per chunk); the first chunk before the reduction.  A
  // single grid takes up to 1024 workgroups and needs few strides (4); a
  // member of a batch, at most 256 workgroups, more (8).  MP: the largest p
  // of the calls (the bottom-block loops are unrolled to it: MAX_P, or 4
  // for a batch whose calls all have p <= 4, which needs fewer registers)
  static_assert(MP >= 1 && MP <= MAX_P, "bottom blocks of at most MAX_P entries");
  static_assert(BLOCK == 256, "one virtual lane of the fixed-order reduction per thread");
  __shared__ double red[512];
  const bool two = (j >= 1) && (vprev != nullptr);
  const int64_t gs = (int64_t)nblk * BLOCK;
  const int64_t i0 = (int64_t)blk * BLOCK + threadIdx.x;
  // This thread's first four partial pairs (virtual lane threadIdx.x of the
  // fixed-order reduction), issued before the data: waiting for them then
  // does not wait for the data.  All loads here are unconditional, at
  // clamped indices (np_in >= 1, n3 >= 1), so that the wait is exact.
  const int l = threadIdx.x;
  double pa[4], pb[4];
#pragma unroll
  for (int u = 0; u < 4; ++u) {
    const int k = min(l + 256 * u, np_in - 1);
    pa[u] = pin[2 * (int64_t)k];
    pb[u] = pin[2 * (int64_t)k + 1];
  }
  __builtin_amdgcn_sched_barrier(0);
  const TV *vp2 = two ? vprev : vj;
  TV xw[UNROLL], xv[UNROLL], xp[UNROLL];
#pragma unroll
  for (int u = 0; u < UNROLL; ++u) {
    const int64_t i = i0 + u * gs < n3 ? i0 + u * gs : n3 - 1;
    xw[u] = w[i];
    xv[u] = vj[i];
    xp[u] = vp2[i];
  }
  // the bottom blocks b_j, b_{j-1} and the scales, read ahead of the
  // reduction's barriers (the first MP values of each row: no branch on p)
  const double *bj = kd->bot + j * MAX_P;
  const double *bp = kd->bot + (j - (j >= 1 ? 1 : 0)) * MAX_P;
  double bjv[MP], bpv[MP];
#pragma unroll
  for (int k = 0; k < MP; ++k) {
    bjv[k] = bj[k];
    bpv[k] = bp[k];
  }
  const double sgj = kd->sigma[j], sgp = kd->sigma[j - (j >= 1 ? 1 : 0)];
  // After a happy breakdown (uniform) nothing is written; the reductions
  // still run, so that no branch ahead of them holds back the loads above.
  const bool happy = kd->happy != 0;
  double d0, d1;
  {
    double a = 0.0, b = 0.0;
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const bool in = l + 256 * u < np_in;
      a += in ? pa[u] : 0.0;
      b += in ? pb[u] : 0.0;
    }
    for (int k = l + 1024; k < np_in; k += 256) {
      a += pin[2 * (int64_t)k];
      b += pin[2 * (int64_t)k + 1];
    }
    red[l] = a;
    red[256 + l] = b;
    reduce_fixed2_finish(red, d0, d1);
  }
  const int ld = MAX_M + 2;
  // (loops over all MP slots, unrolled, with k < p selecting: no run-time
  // index into the register arrays)
  double wb[MP];
#pragma unroll
  for (int k = 0; k < MP; ++k) wb[k] = (k + 1 < MP && k + 1 < p) ? bjv[k + 1 < MP ? k + 1 : 0] : 0.0;   // K b_j
  double hjj = d0, hpj = d1;
#pragma unroll
  for (int k = 0; k < MP; ++k)
    if (k < p) hjj += bjv[k] * wb[k];
  if (two) {
#pragma unroll
    for (int k = 0; k < MP; ++k)
      if (k < p) hpj += bpv[k] * wb[k];
  } else {
    hpj = 0.0;
  }
  if (!happy && blk == 0 && threadIdx.x == 0) {
    kd->H[j * ld + j] = hjj;
    if (two) kd->H[(j - 1) * ld + j] = hpj;
    double nb2 = 0.0;
#pragma unroll
    for (int k = 0; k < MP; ++k) {
      if (k < p) {
        double v = wb[k] - hjj * bjv[k];
        if (two) v -= hpj * bpv[k];
        kd->botu[(j + 1) * MAX_P + k] = v;
        nb2 += v * v;
      }
    }
    kd->wn2[j + 1] = nb2;
  }
  const double ca = hjj * sgj;
  const double cb = two ? hpj * sgp : 0.0;
  // the values in increasing i, chunk by chunk (the order of acc's sum is
  // that of a plain grid-stride loop)
  double acc = 0.0;
  for (int64_t base = i0;;) {
#pragma unroll
    for (int u = 0; u < UNROLL; ++u) {
      const int64_t i = base + u * gs;
      if (i < n3) {
        // the norm is that of the vector as stored (rounded to the basis type)
        const TV x = (TV)(((double)xw[u] - ca * (double)xv[u]) - cb * (double)xp[u]);
        if (!happy) w[i] = x;
        acc += (double)x * (double)x;
      }
    }
    base += UNROLL * gs;
    if (happy || base >= n3) break;
#pragma unroll
    for (int u = 0; u < UNROLL; ++u) {
      const int64_t i = base + u * gs < n3 ? base + u * gs : n3 - 1;
      xw[u] = w[i];
      xv[u] = vj[i];
      xp[u] = vp2[i];
    }
  }
  const double b = block_sum(acc, red);
  if (!happy && threadIdx.x == 0) pout[blk] = b;
}
template <typename TV>
__global__ __launch_bounds__(BLOCK) void arnoldi_update_kernel(int64_t n3, int j, int p, TV *w, const TV *vj,
                                                               const TV *vprev, const double *pin, int np_in,
                                                               double *pout, KDev *kd) {
  arnoldi_update_body<TV, 4>(blockIdx.x, gridDim.x, n3, j, p, w, vj, vprev, pin, np_in, pout, kd);
}
// Waves per SIMD asked of the batched update: with an FP32 basis and p <= 4
// it fits the registers of eight waves without spilling (64 VGPRs, against
// 75 and six waves); more waves keep more of the streaming loads in flight.
template <typename TV, int MP>
constexpr int update_waves_per_eu() {
  return (std::is_same<TV, float>::value && MP <= 4) ? 8 : 1;
}
template <typename TV, int MP>
__global__ __launch_bounds__(BLOCK) __attribute__((amdgpu_waves_per_eu(update_waves_per_eu<TV, MP>()))) void arnoldi_update_batch(const UpdateCall *__restrict__ calls, int ncalls,
                                                  const int *__restrict__ dc) {
  if (dc) {   // counts in device memory: calls, workgroups
    ncalls = dc[0];
    if ((int)blockIdx.x >= dc[1]) return;
  }
  const UpdateCall &c = calls[find_call(calls, ncalls)];
  arnoldi_update_body<TV, 8, MP>(blockIdx.x - c.b0, c.nblk, c.n3, c.j, c.p, static_cast<TV *>(c.w), static_cast<const TV *>(c.vj),
                      static_cast<const TV *>(c.vprev), c.pin, c.np_in, c.pout, c.kd);
}

// start of a sub-step: v~_0 = x (copied), partial ||x||^2 per workgroup.
// Workgroup 0 also clears the happy-breakdown flag of the previous sub-step
// (or of an earlier call on the context): every later kernel of the sweep
// reads it in stream order, and the Krylov-form products return at once
// while it is set.
template <typename TV>
__device__ __forceinline__ void arnoldi_start_body(int blk, int nblk, int64_t n3, const double *x, TV *v0,
                                                   double *pout, KDev *kd) {
  __shared__ double red[BLOCK / 64];
  if (blk == 0 && threadIdx.x == 0) kd->happy = 0;
  double acc = 0.0;
  for (int64_t i = (int64_t)blk * BLOCK + threadIdx.x; i < n3; i += (int64_t)nblk * BLOCK) {
    const TV xv = (TV)x[i];
    v0[i] = xv;
    acc += (double)xv * (double)xv;
  }
  const double b = block_sum(acc, red);
  if (threadIdx.x == 0) pout[blk] = b;
}
template <typename TV>
__global__ __launch_bounds__(BLOCK) void arnoldi_start_kernel(int64_t n3, const double *x, TV *v0, double *pout,
                                                              KDev *kd) {
  arnoldi_start_body(blockIdx.x, gridDim.x, n3, x, v0, pout, kd);
}
template <typename TV>
__global__ __launch_bounds__(BLOCK) void arnoldi_start_batch(const StartCall *__restrict__ calls, int ncalls) {
  const StartCall &c = calls[find_call(calls, ncalls)];
  arnoldi_start_body(blockIdx.x - c.b0, c.nblk, c.n3, c.x, static_cast<TV *>(c.v0), c.pout, c.kd);
}

// accepted sub-step: x = beta * sum_{k<J} sigma_k v~_k E[k][0]; the
// coefficients are staged in LDS
template <typename TV>
__device__ __forceinline__ void arnoldi_combine_body(int blk, int nblk, int64_t n3, const TV *V, int64_t ldv,
                                                     const KDev *kd, double *x) {
  __shared__ double cf[MAX_M + 1];
  const int J = kd->J;
  const double beta = kd->beta;
  for (int k = threadIdx.x; k < J; k += blockDim.x) cf[k] = kd->sigma[k] * kd->E0[k];
  __syncthreads();
  for (int64_t i = (int64_t)blk * BLOCK + threadIdx.x; i < n3; i += (int64_t)nblk * BLOCK) {
    // added in k order; the loads of each group of 16 vectors are issued
    // together (one memory round trip per group, not per few vectors)
    double acc = 0.0;
    int k = 0;
    for (; k + 16 <= J; k += 16) {
      TV xv[16];
#pragma unroll
      for (int u = 0; u < 16; ++u) xv[u] = V[(int64_t)(k + u) * ldv + i];
#pragma unroll
      for (int u = 0; u < 16; ++u) acc += (double)xv[u] * cf[k + u];
    }
    for (; k < J; ++k) acc += (double)V[(int64_t)k * ldv + i] * cf[k];
    x[i] = beta * acc;
  }
}
template <typename TV>
__global__ __launch_bounds__(BLOCK) void arnoldi_combine_kernel(int64_t n3, const TV *V, int64_t ldv, const KDev *kd,
                                                                double *x) {
  arnoldi_combine_body(blockIdx.x, gridDim.x, n3, V, ldv, kd, x);
}
template <typename TV>
__global__ __launch_bounds__(BLOCK) void arnoldi_combine_batch(const CombineCall *__restrict__ calls, int ncalls) {
  const CombineCall &c = calls[find_call(calls, ncalls)];
  arnoldi_combine_body(blockIdx.x - c.b0, c.nblk, c.n3, static_cast<const TV *>(c.V), c.n3, c.kd, c.x);
}

// The device-controlled rounds' combination and start in one launch: per
// member the accepted sub-step's combination (x = beta V E[:, 0]), the next
// sub-step's start vector from x, or both.  The two share the element
// mapping (block blk of nblk, grid-stride), so each thread reads back only
// the x values it wrote, and reads its entries of basis slot 0 before the
// start overwrites them: the results are those of the two kernels in turn.
// Counts in device memory (dc: calls, blocks); fixed grid, blocks in turn.
template <typename TV>
__global__ __launch_bounds__(BLOCK) void arnoldi_pre_batch(const PreCall *__restrict__ calls, const int *__restrict__ dc) {
  const int ncalls = dc[0], total = dc[1];
  for (int lb = blockIdx.x; lb < total; lb += gridDim.x) {
    __syncthreads();   // the previous block's use of shared memory
    const PreCall &c = calls[find_call_at(calls, ncalls, lb)];
    const int blk = lb - c.b0;
    if (c.comb) arnoldi_combine_body(blk, c.nblk, c.n3, static_cast<const TV *>(c.V), c.n3, c.kd, c.x);
    if (c.start) arnoldi_start_body(blk, c.nblk, c.n3, c.x, static_cast<TV *>(c.V), c.pout, c.kd);
  }
}

// ---------------------------------------------------------------------------
// The small exponential of the Krylov step: E = exp(tau H_aug) with
// H_aug = [[H_J, e_1], [0, 0]] ((J+1) x (J+1)); only E[:J, 0] (the sub-step
// result) and E[J-1, J] (the error estimate) are needed.  With A = tau H_J
// and c = tau e_1, every polynomial in tau H_aug has the form
// [[p(A), q(A) c], [0, p(0)]]: the J x J block is carried as a matrix (on the
// matrix cores, FP64 MFMA 16x16x4) and the last column as a vector.
// Method: scaling and squaring with the degree-18 Taylor polynomial,
// 1-norm of the scaled matrix <= 1, Paterson-Stockmeyer in A^2.

typedef double dbl4 __attribute__((ext_vector_type(4)));

// Taylor coefficients 1/k!, k = 0..18, and a zero for k = 19 (degree 18)
__constant__ double kInvFact[20] = {
    1.0, 1.0, 0.5, 1.0 / 6.0, 1.0 / 24.0, 1.0 / 120.0, 1.0 / 720.0, 1.0 / 5040.0, 1.0 / 40320.0,
    1.0 / 362880.0, 1.0 / 3628800.0, 1.0 / 39916800.0, 1.0 / 479001600.0, 1.0 / 6227020800.0,
    1.0 / 87178291200.0, 1.0 / 1307674368000.0, 1.0 / 20922789888000.0, 1.0 / 355687428096000.0,
    1.0 / 6402373705728000.0, 0.0};

// C = X Y for P x P matrices (P = 16 nt) in LDS with leading dimension ld,
// then C[r][c] = epi(r, c, value).  FP64 MFMA 16x16x4: lane l supplies
// X[i][k] and Y[k][j] with i = j = l % 16, k = l / 16, and receives
// D[4 q + l / 16][l % 16] in its q-th accumulator.  Wave w takes the 16x16
// output tiles w, w + nwaves, ...; two accumulators per tile split the k sum.
template <typename Epi>
__device__ void mfma_matmul(const double *X, const double *Y, double *C, int nt, int ld, Epi epi) {
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6, nw = blockDim.x >> 6;
  const int li = lane & 15, lk = lane >> 4;
  const int P = 16 * nt;
  for (int tile = wv; tile < nt * nt; tile += nw) {
    const int ti = tile / nt, tj = tile - ti * nt;
    dbl4 acc0 = {0.0, 0.0, 0.0, 0.0}, acc1 = {0.0, 0.0, 0.0, 0.0};
    const double *xa = X + (ti * 16 + li) * ld + lk;
    const double *yb = Y + lk * ld + tj * 16 + li;
    for (int k0 = 0; k0 < P; k0 += 8) {
      acc0 = __builtin_amdgcn_mfma_f64_16x16x4f64(xa[k0], yb[k0 * ld], acc0, 0, 0, 0);
      acc1 = __builtin_amdgcn_mfma_f64_16x16x4f64(xa[k0 + 4], yb[(k0 + 4) * ld], acc1, 0, 0, 0);
    }
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int row = ti * 16 + 4 * q + lk, col = tj * 16 + li;
      C[row * ld + col] = epi(row, col, acc0[q] + acc1[q]);
    }
  }
}

// y[i * ys] = epi(i, sum_k X[i][k] x[k * xs]), i < P: eight lanes per row
template <typename Epi>
__device__ void lds_matvec(const double *X, int ld, const double *x, int xs, double *y, int ys, int P, Epi epi) {
  for (int t = threadIdx.x; t < 8 * P; t += blockDim.x) {
    const int i = t >> 3, part = t & 7;
    double s = 0.0;
    for (int k = part; k < P; k += 8) s = fma(X[i * ld + k], x[k * xs], s);
    // the eight lanes of a row (whole waves take part: 8P is a multiple of
    // 64): pairs, quads, then the two quads of the half-row, by DPP
    s += dpp_mov<0xB1>(s);
    s += dpp_mov<0x4E>(s);
    s += dpp_mov<0x141>(s);
    if (part == 0) y[i * ys] = epi(i, s);
  }
}

__host__ __device__ inline int expm_pad(int m) { return 16 * ((m + 15) / 16); }
size_t expm_lds_bytes(int m) {
  const int P = expm_pad(m);
  return (size_t)4 * P * (P + 1) * sizeof(double);
}

__device__ __forceinline__ void expm_body(KDev *kd, double tau, KHost *res, int jfin, const double *pin, int np_in,
                                          double tol, unsigned *seq_out, unsigned seq) {
  extern __shared__ double lds[];
  __shared__ double red[256];
  __shared__ double cnorm;
  __shared__ double vec[5][MAX_M];   // pc (two buffers), A c, scratch column
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
  const int tid = threadIdx.x;
  const int J = kd->J;
  const int nt = (J + 15) / 16, P = 16 * nt, ld = P + 1;   // odd stride: LDS banks
  const int nn = P * ld;
  double *A = lds, *A2 = lds + nn, *Pm = lds + 2 * nn, *Qm = lds + 3 * nn;
  const int hld = MAX_M + 2;
  // A = tau H (zero-padded to P x P): each thread's loads of a group of four
  // entries issued together (every index i, j < P <= MAX_M is inside H)
  for (int base = 0; base < P * P; base += 4 * (int)blockDim.x) {
    double hv[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int idx = min(base + u * (int)blockDim.x + tid, P * P - 1);
      const int i = idx / P, j = idx - i * P;
      hv[u] = kd->H[i * hld + j];
    }
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int idx = base + u * (int)blockDim.x + tid;
      if (idx < P * P) {
        const int i = idx / P, j = idx - i * P;
        A[i * ld + j] = (i < J && j < J) ? tau * hv[u] : 0.0;
      }
    }
  }
  __syncthreads();
  // 1-norm of tau H_aug: the column sums of A, and |tau| for the last column
  double cm = (tid == 0) ? fabs(tau) : 0.0;
  for (int idx = tid; idx < 4 * P; idx += blockDim.x) {
    const int j = idx >> 2, part = idx & 3;
    double cs = 0.0;
    for (int i = part; i < P; i += 4) cs += fabs(A[i * ld + j]);
    cs += dpp_mov<0xB1>(cs);   // the four lanes of a column (4P: whole waves)
    cs += dpp_mov<0x4E>(cs);
    cm = fmax(cm, cs);
  }
  {
    double v = cm;
    v = fmax(v, dpp_mov<0xB1>(v));
    v = fmax(v, dpp_mov<0x4E>(v));
    v = fmax(v, dpp_mov<0x141>(v));
    v = fmax(v, dpp_mov<0x140>(v));
    v = fmax(fmax(read_lane(v, 0), read_lane(v, 16)), fmax(read_lane(v, 32), read_lane(v, 48)));
    if ((tid & 63) == 0) red[tid >> 6] = v;
    __syncthreads();
    if (tid == 0) {
      double m = 0.0;
      for (int k = 0; k < (int)(blockDim.x >> 6); ++k) m = fmax(m, red[k]);
      cnorm = m;
    }
    __syncthreads();
  }
  int sq = 0;
  if (cnorm > 1.0) sq = (int)ceil(log2(cnorm));
  const double sc = ldexp(1.0, -sq);
  const double c0 = tau * sc;   // the scaled last column is c0 e_1
  if (sq > 0) {
    for (int idx = tid; idx < P * P; idx += blockDim.x) {
      const int i = idx / P, j = idx - i * P;
      A[i * ld + j] *= sc;
    }
    __syncthreads();
  }
  double *pc = vec[0], *pcn = vec[1], *Ac = vec[2];
  mfma_matmul(A, A, A2, nt, ld, [](int, int, double v) { return v; });
  if (tid < P) Ac[tid] = c0 * A[tid * ld];
  __syncthreads();
  // Paterson-Stockmeyer in A^2, from the top: P = c18 I + c19 A gives, after
  // one step, P = c18 A^2 + c16 I + c17 A; the last column of the running
  // polynomial (q(A) c) and its corner entry pz run alongside
  for (int idx = tid; idx < P * P; idx += blockDim.x) {
    const int i = idx / P, j = idx - i * P;
    Pm[i * ld + j] = kInvFact[18] * A2[i * ld + j] + ((i == j && i < J) ? kInvFact[16] : 0.0) +
                     kInvFact[17] * A[i * ld + j];
  }
  if (tid < P) pc[tid] = kInvFact[18] * Ac[tid] + ((tid == 0) ? kInvFact[17] * c0 : 0.0);
  double pz = kInvFact[16];
  __syncthreads();
  for (int k = 7; k >= 0; --k) {
    const double ca = kInvFact[2 * k], cb = kInvFact[2 * k + 1];
    // last column: q_new(A) c = A^2 (q(A) c) + pz A c + cb c
    const double pzo = pz;
    lds_matvec(A2, ld, pc, 1, pcn, 1, P, [&](int i, double v) { return v + pzo * Ac[i] + ((i == 0) ? cb * c0 : 0.0); });
    if (k > 0 || sq > 0) {
      mfma_matmul(A2, Pm, Qm, nt, ld, [&](int r, int c, double v) {
        return v + ((r == c && r < J) ? ca : 0.0) + cb * A[r * ld + c];
      });
    } else {
      // no squaring follows: only the first column is needed
      lds_matvec(A2, ld, Pm, ld, Qm, ld, P, [&](int i, double v) { return v + ((i == 0) ? ca : 0.0) + cb * A[i * ld]; });
    }
    pz = ca;
    __syncthreads();
    double *t = Pm; Pm = Qm; Qm = t;
    t = pc; pc = pcn; pcn = t;
  }
  // squarings: [[P, pc], [0, pz]]^2 = [[P^2, P pc + pz pc], [0, pz^2]]
  for (int r = 1; r <= sq; ++r) {
    const double pzo = pz;
    const double *pco = pc;
    lds_matvec(Pm, ld, pc, 1, pcn, 1, P, [&](int i, double v) { return v + pzo * pco[i]; });
    if (r < sq) mfma_matmul(Pm, Pm, Qm, nt, ld, [](int, int, double v) { return v; });
    else lds_matvec(Pm, ld, Pm, ld, Qm, ld, P, [](int, double v) { return v; });
    pz = pzo * pzo;
    __syncthreads();
    double *t = Pm; Pm = Qm; Qm = t;
    t = pc; pc = pcn; pcn = t;
  }
  for (int k = tid; k < J; k += blockDim.x) kd->E0[k] = Pm[k * ld];
  if (tid == 0) {
    const double eJ = pc[J - 1];
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
    if (seq_out) {   // a host-memory result: the sequence number last
      __threadfence_system();
      *(volatile unsigned *)seq_out = seq;
    }
  }
}
__global__ __launch_bounds__(EXPM_BLOCK) void expm_kernel(KDev *kd, double tau, KHost *res, int jfin, const double *pin,
                                                          int np_in, double tol, unsigned *seq_out, unsigned seq) {
  expm_body(kd, tau, res, jfin, pin, np_in, tol, seq_out, seq);
}
// one workgroup per member; dc: NULL, or the number of calls in device memory
__global__ __launch_bounds__(EXPM_BLOCK) void expm_batch(const ExpmCall *__restrict__ calls, const int *__restrict__ dc) {
  if (dc && (int)blockIdx.x >= dc[0]) return;
  const ExpmCall &c = calls[blockIdx.x];
  expm_body(c.kd, c.tau, c.res, c.jfin, c.pin, c.np_in, c.tol, nullptr, 0u);
}

// ---------------------------------------------------------------------------
// vector helpers
// out = a x + b y; x or y may be NULL (no term)
__device__ __forceinline__ void axpby_body(int blk, int nblk, int64_t n, double a, const double *x, double b,
                                           const double *y, double *out) {
  for (int64_t i = (int64_t)blk * BLOCK + threadIdx.x; i < n; i += (int64_t)nblk * BLOCK) {
    double r = x ? a * x[i] : 0.0;
    if (y) r += b * y[i];
    out[i] = r;
  }
}
__global__ __launch_bounds__(BLOCK) void axpby_kernel(int64_t n, double a, const double *x, double b, const double *y,
                                                      double *out) {
  axpby_body(blockIdx.x, gridDim.x, n, a, x, b, y, out);
}
__global__ __launch_bounds__(BLOCK) void axpby_batch(const AxpbyCall *__restrict__ calls, int ncalls) {
  const AxpbyCall &c = calls[find_call(calls, ncalls)];
  axpby_body(blockIdx.x - c.b0, c.nblk, c.n, c.a, c.x, c.b, c.y, c.out);
}

__global__ __launch_bounds__(BLOCK) void to_f32_kernel(int64_t n, const double *x, float *y) {
  for (int64_t i = (int64_t)blockIdx.x * BLOCK + threadIdx.x; i < n; i += (int64_t)gridDim.x * BLOCK) y[i] = (float)x[i];
}
__global__ __launch_bounds__(BLOCK) void to_f32_batch(const AxpbyCall *__restrict__ calls, int ncalls) {
  const AxpbyCall &c = calls[find_call(calls, ncalls)];
  float *y = reinterpret_cast<float *>(c.out);
  for (int64_t i = (int64_t)(blockIdx.x - c.b0) * BLOCK + threadIdx.x; i < c.n; i += (int64_t)c.nblk * BLOCK)
    y[i] = (float)c.x[i];
}

// ||x||_2^2: per-workgroup partial sums, then one workgroup sums them in a
// fixed order
__device__ __forceinline__ void norm2_body(int blk, int nblk, int64_t n, const double *x, double *partials) {
  __shared__ double red[BLOCK / 64];
  double acc = 0.0;
  for (int64_t i = (int64_t)blk * BLOCK + threadIdx.x; i < n; i += (int64_t)nblk * BLOCK) acc += x[i] * x[i];
  const double s = block_sum(acc, red);
  if (threadIdx.x == 0) partials[blk] = s;
}
__global__ __launch_bounds__(BLOCK) void norm2_kernel(int64_t n, const double *x, double *partials) {
  norm2_body(blockIdx.x, gridDim.x, n, x, partials);
}
__global__ __launch_bounds__(BLOCK) void norm2_batch(const AxpbyCall *__restrict__ calls, int ncalls) {
  const AxpbyCall &c = calls[find_call(calls, ncalls)];
  norm2_body(blockIdx.x - c.b0, c.nblk, c.n, c.x, c.out);
}
__device__ __forceinline__ void sum_body(int np, const double *partials, double *out) {
  __shared__ double red[BLOCK / 64];
  double acc = 0.0;
  for (int k = threadIdx.x; k < np; k += BLOCK) acc += partials[k];
  const double s = block_sum(acc, red);
  if (threadIdx.x == 0) *out = s;
}
__global__ __launch_bounds__(BLOCK) void sum_kernel(int np, const double *partials, double *out) {
  sum_body(np, partials, out);
}
// one workgroup per call: out = sum of the call's nblk partials in x
__global__ __launch_bounds__(BLOCK) void sum_batch(const AxpbyCall *__restrict__ calls) {
  const AxpbyCall &c = calls[blockIdx.x];
  sum_body(c.nblk, c.x, c.out);
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

// every value finite, the first ndepth (the depths H) positive
__device__ __forceinline__ void check_state_body(int blk, int nblk, int64_t nall, int64_t ndepth, const double *q,
                                                 int *err) {
  int bad = 0;
  for (int64_t i = (int64_t)blk * BLOCK + threadIdx.x; i < nall; i += (int64_t)nblk * BLOCK) {
    const double x = q[i];
    if (!isfinite(x)) bad |= 1;
    if (i < ndepth && !(x > 0.0)) bad |= 2;
  }
  if (bad) atomicOr(err, bad);
}
__global__ __launch_bounds__(BLOCK) void check_state_kernel(int64_t nall, int64_t ndepth, const double *q, int *err) {
  check_state_body(blockIdx.x, gridDim.x, nall, ndepth, q, err);
}
// n = nodes (the vector holds 3n values); out = the member's error flag
__global__ __launch_bounds__(BLOCK) void check_state_batch(const AxpbyCall *__restrict__ calls, int ncalls) {
  const AxpbyCall &c = calls[find_call(calls, ncalls)];
  check_state_body(blockIdx.x - c.b0, c.nblk, 3 * c.n, c.n, c.x, reinterpret_cast<int *>(c.out));
}

// ---------------------------------------------------------------------------
// Diagnostics of Sec. 5.4.  A workgroup holds EPB = 256 / NN whole elements,
// one thread per node.  Per node: the covariant velocity v_j = g_jk u^k
// (Eqs. 64-66), the relative vorticity zeta = (d_1 v_2 - d_2 v_1)/sqrt(g)
// (Eq. 43, element-local collocation derivatives), the Coriolis parameter
// f (Eq. 46); per workgroup the GL-quadrature sums (area element sqrt(g)
// dx^1 dx^2) of H, of the total energy (1/2)[H g_ij u^i u^j + g_r((H +
// h_B)^2 - h_B^2)] and of the potential enstrophy (zeta + f)^2/(2H), in a
// fixed order; diag_sum_kernel adds the partial sums.
template <int NS>
__global__ __launch_bounds__(256) void diag_kernel(const GridArgs g, const DiagOps d, double a2, double gr,
                                                   const double *__restrict__ q, const double *__restrict__ hB,
                                                   double *__restrict__ zeta, double *__restrict__ fcor,
                                                   double *__restrict__ part) {
  constexpr int NN = NS * NS;
  constexpr int EPB = 256 / NN;
  __shared__ double sv[2][EPB * NN];
  __shared__ double red[3 * 4];
  const int tid = threadIdx.x;
  const int le = tid / NN, node = tid - le * NN;
  const int64_t e = (int64_t)blockIdx.x * EPB + le;
  const bool active = le < EPB && e < g.nelem;
  const int64_t N = g.n;
  const int ne = g.ne;
  const int ni = node % NS, nj = node / NS;
  double sm = 0.0, se = 0.0, sz = 0.0;
  double H = 1.0, u1 = 0.0, u2 = 0.0, v1 = 0.0, v2 = 0.0, X = 0.0, Y = 0.0, ax = 1.0, ay = 1.0;
  int64_t gidx = 0;
  int p = 0;
  if (active) {
    const int ei = (int)(e % ne), ej = (int)((e / ne) % ne);
    p = (int)(e / ((int64_t)ne * ne));
    gidx = e * NN + node;
    const Tan3 tx = g.tnode[ei * NS + ni], ty = g.tnode[ej * NS + nj];
    X = tx.x;
    ax = tx.ax;
    Y = ty.x;
    ay = ty.ax;
    const double d2 = ax + Y * Y, rd4 = 1.0 / (d2 * d2);
    const double g11 = a2 * ax * ax * ay * rd4, g12 = -a2 * X * Y * ax * ay * rd4, g22 = a2 * ax * ay * ay * rd4;
    H = q[gidx];
    u1 = q[N + gidx] / H;
    u2 = q[2 * N + gidx] / H;
    v1 = g11 * u1 + g12 * u2;
    v2 = g12 * u1 + g22 * u2;
    sv[0][le * NN + node] = v1;
    sv[1][le * NN + node] = v2;
  }
  __syncthreads();
  if (active) {
    const double *w1 = sv[0] + le * NN, *w2 = sv[1] + le * NN;
    double d1v2 = 0.0, d2v1 = 0.0;
#pragma unroll
    for (int k = 0; k < NS; ++k) {
      d1v2 += d.Dg[ni][k] * w2[nj * NS + k];
      d2v1 += d.Dg[nj][k] * w1[k * NS + ni];
    }
    const double d2 = ax + Y * Y, sd = sqrt(d2);
    const double sg = a2 * ax * ay / (d2 * sd);                                   // Eq. (70)
    const double z = g.two_over_delta * (d1v2 - d2v1) / sg;                      // Eq. (43)
    const double f = 2.0 * g.omega / sd * (g.cA[p] + X * g.cB[p] + Y * g.cC[p]);   // Eq. (46)
    const double hb = hB ? hB[gidx] : 0.0;
    const double en = 0.5 * (H * (u1 * v1 + u2 * v2) + gr * ((H + hb) * (H + hb) - hb * hb));
    const double zs = (z + f) * (z + f) / (2.0 * H);
    const double wgt = d.w[ni] * d.w[nj] * sg / (g.two_over_delta * g.two_over_delta);
    sm = wgt * H;
    se = wgt * en;
    sz = wgt * zs;
    if (zeta) zeta[gidx] = z;
    if (fcor) fcor[gidx] = f;
  }
  sm = wave_sum(sm);
  se = wave_sum(se);
  sz = wave_sum(sz);
  const int lane = tid & 63, wv = tid >> 6;
  if (lane == 0) {
    red[3 * wv + 0] = sm;
    red[3 * wv + 1] = se;
    red[3 * wv + 2] = sz;
  }
  __syncthreads();
  if (tid < 3) {
    double s = 0.0;
    for (int k = 0; k < (int)(blockDim.x >> 6); ++k) s += red[3 * k + tid];
    part[(int64_t)blockIdx.x * 3 + tid] = s;
  }
}

// the three totals from the partial sums of nb workgroups, in a fixed order
__global__ __launch_bounds__(BLOCK) void diag_sum_kernel(int64_t nb, const double *__restrict__ part,
                                                         double *__restrict__ out) {
  __shared__ double red[BLOCK / 64];
  for (int k = 0; k < 3; ++k) {
    double acc = 0.0;
    for (int64_t b = threadIdx.x; b < nb; b += BLOCK) acc += part[b * 3 + k];
    const double s = block_sum(acc, red);
    if (threadIdx.x == 0) out[k] = s;
    __syncthreads();
  }
}

// ---------------------------------------------------------------------------
// The stiff test problems of Sec. 5.1 on the same Krylov machinery.  They are
// small (at most a few thousand unknowns), so one workgroup of 1024 threads
// evaluates F(u) or the exact J(u) v and, in the Krylov form, the Arnoldi
// prologue and epilogue of the DFR kernel: w = sigma_j (J v~_j + W u_j) and
// the two inner products, reduced in a fixed order (one partial pair).
constexpr int ODE_THREADS = 1024;

// fixed-order sum over the workgroup (ODE_THREADS threads)
__device__ double ode_block_sum(double v, double *red) {
  v = wave_sum(v);
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  __syncthreads();
  if (lane == 0) red[wv] = v;
  __syncthreads();
  double s = 0.0;
  for (int k = 0; k < ODE_THREADS / 64; ++k) s += red[k];
  __syncthreads();
  return s;
}

// (J v)_i or F(u)_i of problem `o` at unknown i; usum / vsum: the sums of the
// first n values of u / v (semilinear integral term)
template <bool JVP>
__device__ __forceinline__ double ode_value(const OdeArgs &o, const double *u, const double *v, int64_t i, double vsum) {
  const double h = o.h;
  if (o.kind == 1) {   // advection-diffusion-reaction, Neumann by reflection
    const int N = o.n;
    const int ii = (int)(i % N), jj = (int)(i / N);
    const int64_t e = ii + 1 < N ? i + 1 : i - 1, w = ii > 0 ? i - 1 : i + 1;
    const int64_t nn = jj + 1 < N ? i + N : i - N, s = jj > 0 ? i - N : i + N;
    const double *x = JVP ? v : u;
    const double lin = o.eps * (x[e] + x[w] + x[nn] + x[s] - 4.0 * x[i]) / (h * h) -
                       o.alpha * ((x[e] - x[w]) / (2.0 * h) + (x[nn] - x[s]) / (2.0 * h));
    const double ui = u[i];
    if (JVP) return lin + o.gamma * (-3.0 * ui * ui + 3.0 * ui - 0.5) * v[i];
    return lin + o.gamma * ui * (ui - 0.5) * (1.0 - ui);
  }
  if (o.kind == 2) {   // Burgers, zero ends
    const int n = o.n;
    const double *x = JVP ? v : u;
    const double xp = i + 1 < n ? x[i + 1] : 0.0, xm = i > 0 ? x[i - 1] : 0.0;
    const double lap = (xp - 2.0 * x[i] + xm) / (h * h);
    const double up = i + 1 < n ? u[i + 1] : 0.0, um = i > 0 ? u[i - 1] : 0.0;
    if (JVP) return -(up * xp - um * xm) / (2.0 * h) + o.eps * lap;
    return -(up * up - um * um) / (4.0 * h) + o.eps * lap;
  }
  // semilinear parabolic, zero ends, time as unknown n
  const int n = o.n;
  if (i == n) return JVP ? 0.0 : 1.0;
  const double *x = JVP ? v : u;
  const double xp = i + 1 < n ? x[i + 1] : 0.0, xm = i > 0 ? x[i - 1] : 0.0;
  const double xi = (double)(i + 1) * h;
  const double src = xi * (1.0 - xi) + 2.0 - o.isum;
  const double lap = (xp - 2.0 * x[i] + xm) / (h * h);
  const double et = exp(u[n]);
  return lap + h * vsum + (JVP ? v[n] : 1.0) * et * src;
}

template <bool JVP, bool AR>
__global__ __launch_bounds__(ODE_THREADS) void ode_kernel(const OdeArgs o, const double *__restrict__ u,
                                                          const double *__restrict__ v,
                                                          const double *__restrict__ vscale,
                                                          double *__restrict__ out, const ArnoldiArgs ar) {
  __shared__ double red[256];
  const int64_t len = o.len;
  double sig = 1.0, bj[MAX_P];
  if constexpr (AR) {
    if (ar.kd->happy) return;
    if (!arnoldi_prologue(ar, red, true, sig, bj)) return;
  }
  // the integral term of the semilinear problem: sum of the first n values
  double xsum = 0.0;
  if (o.kind == 3) {
    const double *x = JVP ? v : u;
    double a = 0.0;
    for (int64_t i = threadIdx.x; i < o.n; i += ODE_THREADS) a += x[i];
    xsum = ode_block_sum(a, red);
  }
  const double vs = AR ? sig : ((JVP && vscale) ? *vscale : 1.0);
  double d0 = 0.0, d1 = 0.0;
  const double *ub = AR ? ar.kd->botu + ar.j * MAX_P : nullptr;
  const double sp = (AR && ar.vprev) ? ar.kd->sigma[ar.j - 1] : 0.0;
  for (int64_t i = threadIdx.x; i < len; i += ODE_THREADS) {
    const double r = ode_value<JVP>(o, u, v, i, xsum);
    if constexpr (AR) {
      double wb = 0.0;
      for (int k = 0; k < ar.p; ++k) wb += ar.W[k][i] * (ar.start ? ar.ybot[k] : ub[k]);
      const double a = vs * (r + wb);
      out[i] = a;
      d0 += a * (vs * v[i]);
      if (ar.vprev) d1 += a * (sp * static_cast<const double *>(ar.vprev)[i]);
    } else {
      out[i] = JVP ? r * vs : r;
    }
  }
  if constexpr (AR) {
    d0 = ode_block_sum(d0, red);
    d1 = ode_block_sum(d1, red);
    if (threadIdx.x == 0) {
      ar.pout[0] = d0;
      ar.pout[1] = d1;
    }
  }
}

// ---------------------------------------------------------------------------
// launchers
static inline int grid_for(int64_t n) {
  int64_t b = (n + BLOCK - 1) / BLOCK;
  if (b > 8192) b = 8192;
  if (b < 1) b = 1;
  return (int)b;
}

// dynamic LDS of the tiled kernel (complex-step form, the largest)
size_t dfr_lds_bytes(int ns, int tx, int ty, bool fp32) {
  const int ts = fp32 ? (int)sizeof(float) : (int)sizeof(double);
  return (size_t)dfr_lds_layout(ns, tx, ty, 2, ts).total * ts;
}

int64_t dfr_num_tiles(const Ctx *c, bool arnoldi) {
  if (c->ode_kind) return 1;   // one workgroup
  const int tx = arnoldi ? c->ar_tx : c->tile_tx, ty = arnoldi ? c->ar_ty : c->tile_ty;
  return 6LL * (c->ne / tx) * (c->ne / ty);
}

int launch_norm2(Ctx *c, int64_t n, const double *x, double *partials, int nblk) {
  dfr_launch(c, DFR_K_OTHER, norm2_kernel, dim3((unsigned)nblk), dim3(BLOCK), 0, n, x, partials);
  DFR_HIP(hipGetLastError());
  return DFR_OK;
}

int launch_sum(Ctx *c, int np, const double *partials, double *out) {
  dfr_launch(c, DFR_K_FINALIZE, sum_kernel, dim3(1), dim3(BLOCK), 0, np, partials, out);
  DFR_HIP(hipGetLastError());
  return DFR_OK;
}

int64_t dfr_grid_blocks(const Ctx *c, bool arnoldi) {
  const int tx = arnoldi ? c->ar_tx : c->tile_tx, ty = arnoldi ? c->ar_ty : c->tile_ty;
  const int64_t nlog = 6LL * (c->ne / tx) * (c->ne / ty);
  return ((nlog + 7) / 8) * 8;
}

template <int NS, typename T, typename TQ, bool CS, bool AR>
static void launch_ns(Ctx *c, const TQ *q, const void *v, const double *vscale, double eps, void *out,
                      const ArnoldiArgs &ar) {
  const int tx = ar.on ? c->ar_tx : c->tile_tx, ty = ar.on ? c->ar_ty : c->tile_ty;
  const size_t lds = (size_t)dfr_lds_layout(NS, tx, ty, CS ? 2 : 1, (int)sizeof(T)).total * sizeof(T);
  const int threads = std::max(256, ((tx * ty * NS * NS + 63) / 64) * 64);
  const int64_t nb = dfr_grid_blocks(c, ar.on != 0);
  const int kind = !CS ? DFR_K_RHS : (ar.on ? DFR_K_JV_ARNOLDI : DFR_K_JV);
  const dim3 grid((unsigned)nb), block(threads);
  if constexpr (AR && std::is_same<T, float>::value) {
    if (c->basis32) {   // the FP32 form with an FP32 basis
      const float *vf = static_cast<const float *>(v);
      float *of = static_cast<float *>(out);
      if (c->ga.riemann == DFR_AUSM)
        dfr_launch(c, kind, (dfr_kernel<NS, T, TQ, CS, AR, 1, float>), grid, block, lds, c->ga, c->ops, tx, ty, q, vf, vscale, eps, of, ar);
      else
        dfr_launch(c, kind, (dfr_kernel<NS, T, TQ, CS, AR, 0, float>), grid, block, lds, c->ga, c->ops, tx, ty, q, vf, vscale, eps, of, ar);
      return;
    }
  }
  const double *vd = static_cast<const double *>(v);
  double *od = static_cast<double *>(out);
  if (c->ga.riemann == DFR_AUSM)
    dfr_launch(c, kind, (dfr_kernel<NS, T, TQ, CS, AR, 1, double>), grid, block, lds, c->ga, c->ops, tx, ty, q, vd, vscale, eps, od, ar);
  else
    dfr_launch(c, kind, (dfr_kernel<NS, T, TQ, CS, AR, 0, double>), grid, block, lds, c->ga, c->ops, tx, ty, q, vd, vscale, eps, od, ar);
}

template <int NS>
static int set_lds_attr(size_t bytes) {
  const void *fns[] = {(const void *)dfr_kernel<NS, double, double, false, false, 0, double>,
                       (const void *)dfr_kernel<NS, double, double, true, false, 0, double>,
                       (const void *)dfr_kernel<NS, float, float, true, false, 0, double>,
                       (const void *)dfr_kernel<NS, double, double, true, true, 0, double>,
                       (const void *)dfr_kernel<NS, float, float, true, true, 0, double>,
                       (const void *)dfr_kernel<NS, float, float, true, true, 0, float>,
                       (const void *)dfr_kernel<NS, double, double, false, false, 1, double>,
                       (const void *)dfr_kernel<NS, double, double, true, false, 1, double>,
                       (const void *)dfr_kernel<NS, float, float, true, false, 1, double>,
                       (const void *)dfr_kernel<NS, double, double, true, true, 1, double>,
                       (const void *)dfr_kernel<NS, float, float, true, true, 1, double>,
                       (const void *)dfr_kernel<NS, float, float, true, true, 1, float>,
                       (const void *)dfr_kernel_batch<NS, double, double, false, false, double>,
                       (const void *)dfr_kernel_batch<NS, double, double, true, false, double>,
                       (const void *)dfr_kernel_batch<NS, float, float, true, false, double>,
                       (const void *)dfr_kernel_batch<NS, double, double, true, true, double>,
                       (const void *)dfr_kernel_batch<NS, float, float, true, true, double>,
                       (const void *)dfr_kernel_batch<NS, float, float, true, true, float>};
  for (const void *f : fns) DFR_HIP(hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes));
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
static int dispatch_ns(Ctx *c, const TQ *q, const void *v, const double *vscale, double eps, void *out,
                       const ArnoldiArgs &ar) {
  switch (c->ns) {
    case 2: ar.on ? launch_ns<2, T, TQ, CS, CS>(c, q, v, vscale, eps, out, ar)
            : launch_ns<2, T, TQ, CS, false>(c, q, v, vscale, eps, out, ar); break;
    case 3: ar.on ? launch_ns<3, T, TQ, CS, CS>(c, q, v, vscale, eps, out, ar)
            : launch_ns<3, T, TQ, CS, false>(c, q, v, vscale, eps, out, ar); break;
    case 4: ar.on ? launch_ns<4, T, TQ, CS, CS>(c, q, v, vscale, eps, out, ar)
            : launch_ns<4, T, TQ, CS, false>(c, q, v, vscale, eps, out, ar); break;
    case 5: ar.on ? launch_ns<5, T, TQ, CS, CS>(c, q, v, vscale, eps, out, ar)
            : launch_ns<5, T, TQ, CS, false>(c, q, v, vscale, eps, out, ar); break;
    case 6: ar.on ? launch_ns<6, T, TQ, CS, CS>(c, q, v, vscale, eps, out, ar)
            : launch_ns<6, T, TQ, CS, false>(c, q, v, vscale, eps, out, ar); break;
    case 7: ar.on ? launch_ns<7, T, TQ, CS, CS>(c, q, v, vscale, eps, out, ar)
            : launch_ns<7, T, TQ, CS, false>(c, q, v, vscale, eps, out, ar); break;
    case 8: ar.on ? launch_ns<8, T, TQ, CS, CS>(c, q, v, vscale, eps, out, ar)
            : launch_ns<8, T, TQ, CS, false>(c, q, v, vscale, eps, out, ar); break;
    default: set_error("unsupported number of GL points"); return DFR_E_INVAL;
  }
  DFR_HIP(hipGetLastError());
  return DFR_OK;
}

int launch_dfr(Ctx *c, const double *q, const float *q32, const void *v, const double *vscale, double eps,
               bool complex_step, bool fp32, void *out, const ArnoldiArgs *ar) {
  if (c->ode_kind)
    return launch_ode(c, q, static_cast<const double *>(v), vscale, complex_step, static_cast<double *>(out), ar);
  ArnoldiArgs none{};
  const ArnoldiArgs &a = ar ? *ar : none;
  if (!complex_step) return dispatch_ns<double, double, false>(c, q, nullptr, nullptr, 0.0, out, a);
  if (fp32) return dispatch_ns<float, float, true>(c, q32, v, vscale, eps, out, a);
  return dispatch_ns<double, double, true>(c, q, v, vscale, eps, out, a);
}

// workgroups of the vector kernels whose partial sums the next kernel
// reduces (in every one of its workgroups): at most DFR_REDUCE_BLOCKS
#ifndef DFR_REDUCE_BLOCKS
#define DFR_REDUCE_BLOCKS 1024
#endif
static_assert(DFR_REDUCE_BLOCKS <= 1024, "the prologue reductions take at most 1024 partial sums");
static inline int grid_reduce(int64_t n) {
  const int g = grid_for(n);
  return g < DFR_REDUCE_BLOCKS ? g : DFR_REDUCE_BLOCKS;
}

int launch_arnoldi_first(Ctx *c, const ArnoldiArgs &ar, void *out, int *np_out) {
  const int64_t n3 = c->n3;
  const int nb = grid_reduce(n3);
  if (c->basis32)
    dfr_launch(c, DFR_K_OTHER, arnoldi_first_kernel<float>, dim3(nb), dim3(BLOCK), 0, n3, ar, static_cast<float *>(out));
  else
    dfr_launch(c, DFR_K_OTHER, arnoldi_first_kernel<double>, dim3(nb), dim3(BLOCK), 0, n3, ar, static_cast<double *>(out));
  DFR_HIP(hipGetLastError());
  *np_out = nb;
  return DFR_OK;
}

int launch_update(Ctx *c, int j, void *w, const void *vj, const void *vprev, const double *pin, int np_in,
                  double *pout, int *np_out) {
  const int64_t n3 = c->n3;
  const int nb = grid_reduce(n3);
  if (c->basis32)
    dfr_launch(c, DFR_K_UPDATE, arnoldi_update_kernel<float>, dim3(nb), dim3(BLOCK), 0, n3, j, c->kiops_p,
               static_cast<float *>(w), static_cast<const float *>(vj), static_cast<const float *>(vprev), pin, np_in,
               pout, c->d_kd);
  else
    dfr_launch(c, DFR_K_UPDATE, arnoldi_update_kernel<double>, dim3(nb), dim3(BLOCK), 0, n3, j, c->kiops_p,
               static_cast<double *>(w), static_cast<const double *>(vj), static_cast<const double *>(vprev), pin,
               np_in, pout, c->d_kd);
  DFR_HIP(hipGetLastError());
  *np_out = nb;
  return DFR_OK;
}

int launch_start(Ctx *c, const double *x, void *v0, double *pout, int *np_out) {
  const int64_t n3 = c->n3;
  const int nb = grid_reduce(n3);
  if (c->basis32)
    dfr_launch(c, DFR_K_OTHER, arnoldi_start_kernel<float>, dim3(nb), dim3(BLOCK), 0, n3, x, static_cast<float *>(v0), pout,
               c->d_kd);
  else
    dfr_launch(c, DFR_K_OTHER, arnoldi_start_kernel<double>, dim3(nb), dim3(BLOCK), 0, n3, x, static_cast<double *>(v0), pout,
               c->d_kd);
  DFR_HIP(hipGetLastError());
  *np_out = nb;
  return DFR_OK;
}

int launch_combine(Ctx *c, double *x) {
  const int64_t n3 = c->n3;
  if (c->basis32)
    dfr_launch(c, DFR_K_OTHER, arnoldi_combine_kernel<float>, dim3(grid_for(n3)), dim3(BLOCK), 0, n3,
               reinterpret_cast<const float *>(c->d_V), n3, (const KDev *)c->d_kd, x);
  else
    dfr_launch(c, DFR_K_OTHER, arnoldi_combine_kernel<double>, dim3(grid_for(n3)), dim3(BLOCK), 0, n3,
               (const double *)c->d_V, n3, (const KDev *)c->d_kd, x);
  DFR_HIP(hipGetLastError());
  return DFR_OK;
}

int launch_expm(Ctx *c, double tau, int jfin, const double *pin, int np_in, double tol, unsigned seq) {
  const size_t lds = expm_lds_bytes(c->kiops_mmax);
  dfr_launch(c, DFR_K_EXPM, expm_kernel, dim3(1), dim3(EXPM_BLOCK), lds, c->d_kd, tau, &c->d_mail->kh, jfin, pin, np_in,
             tol, &c->d_mail->seq, seq);
  DFR_HIP(hipGetLastError());
  return DFR_OK;
}

int launch_axpby(Ctx *c, int64_t n, double a, const double *x, double b, const double *y, double *out) {
  dfr_launch(c, DFR_K_OTHER, axpby_kernel, dim3(grid_for(n)), dim3(BLOCK), 0, n, a, x, b, y, out);
  DFR_HIP(hipGetLastError());
  return DFR_OK;
}

int launch_copy_to_f32(Ctx *c, int64_t n, const double *x, float *y) {
  dfr_launch(c, DFR_K_OTHER, to_f32_kernel, dim3(grid_for(n)), dim3(BLOCK), 0, n, x, y);
  DFR_HIP(hipGetLastError());
  return DFR_OK;
}

int launch_fill(Ctx *c, double *q, double *v) {
  hipLaunchKernelGGL(fill_kernel, dim3(grid_for(3 * c->n)), dim3(BLOCK), 0, c->stream, c->n, q, v);
  DFR_HIP(hipGetLastError());
  return DFR_OK;
}

int launch_check_state(Ctx *c, const double *q) {
  dfr_launch(c, DFR_K_OTHER, check_state_kernel, dim3(grid_for(c->n3)), dim3(BLOCK), 0, c->n3,
             c->ode_kind ? (int64_t)0 : c->n, q, c->d_err);
  DFR_HIP(hipGetLastError());
  return DFR_OK;
}

int set_expm_lds_limit(int m) {
  const size_t lds = expm_lds_bytes(m);
  DFR_HIP(hipFuncSetAttribute((const void *)expm_batch, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
  DFR_HIP(hipFuncSetAttribute((const void *)expm_kernel, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
  return DFR_OK;
}

// ---------------------------------------------------------------------------
// batched launchers

int stage_put(Stage &st, hipStream_t s, const void *src, size_t bytes, void **dev) {
  const size_t off = (st.used + 255) & ~(size_t)255;
  if (off + bytes > st.cap) {
    if (bytes > st.cap) {
      set_error("a batched call table exceeds the staging arena");
      return DFR_E_INVAL;
    }
    // the arena is full: copy and issue what is deferred, wait for the
    // copies in flight, then start over
    if (st.defer) {
      int rc = stage_flush(st, s);
      if (rc) return rc;
      st.defer = true;
    }
    DFR_HIP(hipStreamSynchronize(s));
    st.used = 0;
    st.pend0 = 0;
    return stage_put(st, s, src, bytes, dev);
  }
  std::memcpy(st.h + off, src, bytes);
  if (!st.defer) DFR_HIP(hipMemcpyAsync(st.d + off, st.h + off, bytes, hipMemcpyHostToDevice, s));
  st.used = off + bytes;
  *dev = st.d + off;
  return DFR_OK;
}

int stage_launch(Stage &st, std::function<int()> launch) {
  if (!st.defer) return launch();
  st.pending.push_back(std::move(launch));
  return DFR_OK;
}

int stage_flush(Stage &st, hipStream_t s) {
  st.defer = false;
  int rc = DFR_OK;
  if (st.used > st.pend0) {
    const hipError_t e = hipMemcpyAsync(st.d + st.pend0, st.h + st.pend0, st.used - st.pend0,
                                        hipMemcpyHostToDevice, s);
    if (e != hipSuccess) {
      set_error(std::string("HIP error: ") + hipGetErrorString(e));
      rc = DFR_E_HIP;
    }
  }
  st.pend0 = st.used;
  for (auto &f : st.pending)
    if (!rc) rc = f();
  st.pending.clear();
  return rc;
}

int vec_blocks(int64_t n) { return grid_reduce(n); }

template <typename C>
static int set_b0(std::vector<C> &calls) {
  int b = 0;
  for (auto &c : calls) {
    c.b0 = b;
    b += c.nblk;
  }
  return b;
}

template <int NS, typename T, typename TQ, bool CS, bool AR, typename TV>
static int launch_dfr_batch_ns(hipStream_t s, Stage &st, std::vector<DfrCall> &calls) {
  int nlog = 0, threads = 256;
  size_t lds = 0;
  double nodes = 0.0;
  for (auto &c : calls) {
    c.b0 = nlog;
    c.ntiles = 6 * (c.g_ne / c.TX) * (c.g_ne / c.TY);
    nlog += c.ntiles;
    nodes += (double)c.ntiles * c.TX * c.TY * NS * NS;
    threads = std::max(threads, ((c.TX * c.TY * NS * NS + 63) / 64) * 64);
    lds = std::max(lds, (size_t)dfr_lds_layout(NS, c.TX, c.TY, CS ? 2 : 1, (int)sizeof(T)).total * sizeof(T));
  }
  void *d = nullptr;
  int rc = stage_put(st, s, calls.data(), sizeof(DfrCall) * calls.size(), &d);
  if (rc) return rc;
  const int grid = ((nlog + 7) / 8) * 8;
  const int n = (int)calls.size();
  const int kind = AR ? DFR_K_JV_ARNOLDI : (CS ? DFR_K_JV : DFR_K_RHS);
  KTimer *tm = st.timer;
  return stage_launch(st, [=]() -> int {
    timed_launch(tm, kind, nodes, s, dfr_kernel_batch<NS, T, TQ, CS, AR, TV>, dim3(grid), dim3(threads), lds,
                 (const DfrCall *)d, n, nlog, (const int *)nullptr);
    DFR_HIP(hipGetLastError());
    return DFR_OK;
  });
}

template <int NS>
static int launch_dfr_batch_form(hipStream_t s, Stage &st, bool cs, bool fp32, bool ar, bool b32,
                                 std::vector<DfrCall> &calls) {
  if (!cs) return launch_dfr_batch_ns<NS, double, double, false, false, double>(s, st, calls);
  if (fp32) {
    if (ar && b32) return launch_dfr_batch_ns<NS, float, float, true, true, float>(s, st, calls);
    return ar ? launch_dfr_batch_ns<NS, float, float, true, true, double>(s, st, calls)
              : launch_dfr_batch_ns<NS, float, float, true, false, double>(s, st, calls);
  }
  return ar ? launch_dfr_batch_ns<NS, double, double, true, true, double>(s, st, calls)
            : launch_dfr_batch_ns<NS, double, double, true, false, double>(s, st, calls);
}

int launch_dfr_batch(hipStream_t s, Stage &st, int ns, bool complex_step, bool fp32, bool arnoldi, bool basis32,
                     std::vector<DfrCall> &calls) {
  if (calls.empty()) return DFR_OK;
  if (basis32 && !(complex_step && fp32 && arnoldi)) {
    set_error("an FP32 basis goes with the complex-FP32 Krylov-form product only");
    return DFR_E_INVAL;
  }
  switch (ns) {
    case 2: return launch_dfr_batch_form<2>(s, st, complex_step, fp32, arnoldi, basis32, calls);
    case 3: return launch_dfr_batch_form<3>(s, st, complex_step, fp32, arnoldi, basis32, calls);
    case 4: return launch_dfr_batch_form<4>(s, st, complex_step, fp32, arnoldi, basis32, calls);
    case 5: return launch_dfr_batch_form<5>(s, st, complex_step, fp32, arnoldi, basis32, calls);
    case 6: return launch_dfr_batch_form<6>(s, st, complex_step, fp32, arnoldi, basis32, calls);
    case 7: return launch_dfr_batch_form<7>(s, st, complex_step, fp32, arnoldi, basis32, calls);
    case 8: return launch_dfr_batch_form<8>(s, st, complex_step, fp32, arnoldi, basis32, calls);
    default: set_error("unsupported number of GL points"); return DFR_E_INVAL;
  }
}

template <typename C, typename K>
static int launch_calls(hipStream_t s, Stage &st, std::vector<C> &calls, K kernel, int kind = DFR_K_OTHER) {
  if (calls.empty()) return DFR_OK;
  const int nb = set_b0(calls);
  void *d = nullptr;
  int rc = stage_put(st, s, calls.data(), sizeof(C) * calls.size(), &d);
  if (rc) return rc;
  const int n = (int)calls.size();
  KTimer *tm = st.timer;
  return stage_launch(st, [=]() -> int {
    timed_launch(tm, kind, 0.0, s, kernel, dim3(nb), dim3(BLOCK), 0, (const C *)d, n);
    DFR_HIP(hipGetLastError());
    return DFR_OK;
  });
}

// the same for the Krylov kernels, which also take device-side counts (NULL here)
template <typename C, typename K>
static int launch_calls_k(hipStream_t s, Stage &st, std::vector<C> &calls, K kernel, int kind = DFR_K_OTHER) {
  if (calls.empty()) return DFR_OK;
  const int nb = set_b0(calls);
  void *d = nullptr;
  int rc = stage_put(st, s, calls.data(), sizeof(C) * calls.size(), &d);
  if (rc) return rc;
  const int n = (int)calls.size();
  KTimer *tm = st.timer;
  return stage_launch(st, [=]() -> int {
    timed_launch(tm, kind, 0.0, s, kernel, dim3(nb), dim3(BLOCK), 0, (const C *)d, n, (const int *)nullptr);
    DFR_HIP(hipGetLastError());
    return DFR_OK;
  });
}

int launch_first_batch(hipStream_t s, Stage &st, bool basis32, std::vector<FirstCall> &calls) {
  return basis32 ? launch_calls_k(s, st, calls, arnoldi_first_batch<float>)
                 : launch_calls_k(s, st, calls, arnoldi_first_batch<double>);
}
int launch_update_batch(hipStream_t s, Stage &st, bool basis32, std::vector<UpdateCall> &calls) {
  int pmax = 0;
  for (const UpdateCall &c : calls) pmax = std::max(pmax, c.p);
  if (pmax <= 4)
    return basis32 ? launch_calls_k(s, st, calls, arnoldi_update_batch<float, 4>, DFR_K_UPDATE)
                   : launch_calls_k(s, st, calls, arnoldi_update_batch<double, 4>, DFR_K_UPDATE);
  return basis32 ? launch_calls_k(s, st, calls, arnoldi_update_batch<float, MAX_P>, DFR_K_UPDATE)
                 : launch_calls_k(s, st, calls, arnoldi_update_batch<double, MAX_P>, DFR_K_UPDATE);
}
int launch_start_batch(hipStream_t s, Stage &st, bool basis32, std::vector<StartCall> &calls) {
  return basis32 ? launch_calls(s, st, calls, arnoldi_start_batch<float>)
                 : launch_calls(s, st, calls, arnoldi_start_batch<double>);
}
int launch_combine_batch(hipStream_t s, Stage &st, bool basis32, std::vector<CombineCall> &calls) {
  return basis32 ? launch_calls(s, st, calls, arnoldi_combine_batch<float>)
                 : launch_calls(s, st, calls, arnoldi_combine_batch<double>);
}

int launch_expm_batch(hipStream_t s, Stage &st, std::vector<ExpmCall> &calls, size_t lds) {
  if (calls.empty()) return DFR_OK;
  void *d = nullptr;
  int rc = stage_put(st, s, calls.data(), sizeof(ExpmCall) * calls.size(), &d);
  if (rc) return rc;
  const unsigned n = (unsigned)calls.size();
  KTimer *tm = st.timer;
  return stage_launch(st, [=]() -> int {
    timed_launch(tm, DFR_K_EXPM, 0.0, s, expm_batch, dim3(n), dim3(EXPM_BLOCK), lds, (const ExpmCall *)d,
                 (const int *)nullptr);
    DFR_HIP(hipGetLastError());
    return DFR_OK;
  });
}

// The device-controlled round's launches: tables and counts in device
// memory (dc), grids sized by the caller for every member active.  tm: NULL
// (the launches may be captured into a graph), or a timer to bracket each
// launch with events (units 0: the caller adds the nodes afterwards).
template <int NS>
static void launch_dfr_dev_ns(hipStream_t s, bool fp32, bool basis32, const DfrCall *calls, const int *dc, int grid,
                              int threads, size_t lds, KTimer *tm) {
  const int k = DFR_K_JV_ARNOLDI;
  if (fp32 && basis32)
    timed_launch(tm, k, 0.0, s, dfr_kernel_batch<NS, float, float, true, true, float>, dim3(grid), dim3(threads), lds,
                 calls, 0, 0, dc);
  else if (fp32)
    timed_launch(tm, k, 0.0, s, dfr_kernel_batch<NS, float, float, true, true, double>, dim3(grid), dim3(threads),
                 lds, calls, 0, 0, dc);
  else
    timed_launch(tm, k, 0.0, s, dfr_kernel_batch<NS, double, double, true, true, double>, dim3(grid), dim3(threads),
                 lds, calls, 0, 0, dc);
}

int launch_dfr_batch_dev(hipStream_t s, int ns, bool fp32, bool basis32, const DfrCall *calls, const int *dc,
                         int grid, int threads, size_t lds, KTimer *tm) {
  if (basis32 && !fp32) {
    set_error("an FP32 basis goes with the complex-FP32 Krylov-form product only");
    return DFR_E_INVAL;
  }
  switch (ns) {
    case 2: launch_dfr_dev_ns<2>(s, fp32, basis32, calls, dc, grid, threads, lds, tm); break;
    case 3: launch_dfr_dev_ns<3>(s, fp32, basis32, calls, dc, grid, threads, lds, tm); break;
    case 4: launch_dfr_dev_ns<4>(s, fp32, basis32, calls, dc, grid, threads, lds, tm); break;
    case 5: launch_dfr_dev_ns<5>(s, fp32, basis32, calls, dc, grid, threads, lds, tm); break;
    case 6: launch_dfr_dev_ns<6>(s, fp32, basis32, calls, dc, grid, threads, lds, tm); break;
    case 7: launch_dfr_dev_ns<7>(s, fp32, basis32, calls, dc, grid, threads, lds, tm); break;
    case 8: launch_dfr_dev_ns<8>(s, fp32, basis32, calls, dc, grid, threads, lds, tm); break;
    default: set_error("unsupported number of GL points"); return DFR_E_INVAL;
  }
  DFR_HIP(hipGetLastError());
  return DFR_OK;
}

template <typename TV>
static void launch_krylov_dev_t(hipStream_t s, int kind, const void *calls, const int *dc, int grid, int pmax,
                                KTimer *tm) {
  switch (kind) {
    case KD_PRE:
      timed_launch(tm, DFR_K_OTHER, 0.0, s, arnoldi_pre_batch<TV>, dim3(grid), dim3(BLOCK), 0,
                   (const PreCall *)calls, dc);
      break;
    case KD_FIRST:
      timed_launch(tm, DFR_K_OTHER, 0.0, s, arnoldi_first_batch<TV>, dim3(grid), dim3(BLOCK), 0,
                   (const FirstCall *)calls, 0, dc);
      break;
    case KD_UPDATE:
      if (pmax <= 4)
        timed_launch(tm, DFR_K_UPDATE, 0.0, s, arnoldi_update_batch<TV, 4>, dim3(grid), dim3(BLOCK), 0,
                     (const UpdateCall *)calls, 0, dc);
      else
        timed_launch(tm, DFR_K_UPDATE, 0.0, s, arnoldi_update_batch<TV, MAX_P>, dim3(grid), dim3(BLOCK), 0,
                     (const UpdateCall *)calls, 0, dc);
      break;
    default: break;
  }
}

int launch_krylov_dev(hipStream_t s, int kind, bool basis32, const void *calls, const int *dc, int grid, int pmax,
                      KTimer *tm) {
  if (basis32) launch_krylov_dev_t<float>(s, kind, calls, dc, grid, pmax, tm);
  else launch_krylov_dev_t<double>(s, kind, calls, dc, grid, pmax, tm);
  DFR_HIP(hipGetLastError());
  return DFR_OK;
}

int launch_expm_dev(hipStream_t s, const ExpmCall *calls, const int *dc, int grid, size_t lds, KTimer *tm) {
  timed_launch(tm, DFR_K_EXPM, 0.0, s, expm_batch, dim3(grid), dim3(EXPM_BLOCK), lds, calls, dc);
  DFR_HIP(hipGetLastError());
  return DFR_OK;
}

int launch_vec_batch(hipStream_t s, Stage &st, int kind, std::vector<AxpbyCall> &calls) {
  switch (kind) {
    case VB_AXPBY: return launch_calls(s, st, calls, axpby_batch);
    case VB_TO_F32: return launch_calls(s, st, calls, to_f32_batch);
    case VB_NORM2: return launch_calls(s, st, calls, norm2_batch);
    case VB_CHECK: return launch_calls(s, st, calls, check_state_batch);
    case VB_SUM: {
      if (calls.empty()) return DFR_OK;
      void *d = nullptr;
      int rc = stage_put(st, s, calls.data(), sizeof(AxpbyCall) * calls.size(), &d);
      if (rc) return rc;
      const unsigned n = (unsigned)calls.size();
      KTimer *tm = st.timer;
      return stage_launch(st, [=]() -> int {
        timed_launch(tm, DFR_K_FINALIZE, 0.0, s, sum_batch, dim3(n), dim3(BLOCK), 0, (const AxpbyCall *)d);
        DFR_HIP(hipGetLastError());
        return DFR_OK;
      });
    }
    default: set_error("unknown batched vector kernel"); return DFR_E_INVAL;
  }
}

int64_t diag_blocks(const Ctx *c) {
  const int epb = 256 / (c->ns * c->ns);
  return (c->nelem + epb - 1) / epb;
}

int launch_diagnostics(Ctx *c, const double *q, double *zeta, double *fcor) {
  const int64_t nb = diag_blocks(c);
  const double a2 = c->radius * c->radius;
  double *part = c->d_diag;
  const int threads = ((256 / (c->ns * c->ns)) * c->ns * c->ns + 63) / 64 * 64;
#define DIAG_CASE(K)                                                                                              \
  case K:                                                                                                       \
    dfr_launch(c, DFR_K_OTHER, diag_kernel<K>, dim3((unsigned)nb), dim3(threads), 0, c->ga, c->dops, a2, c->gravity, \
               q, (const double *)c->d_hB, zeta, fcor, part);                                                    \
    break;
  switch (c->ns) {
    DIAG_CASE(2)
    DIAG_CASE(3)
    DIAG_CASE(4)
    DIAG_CASE(5)
    DIAG_CASE(6)
    DIAG_CASE(7)
    DIAG_CASE(8)
    default: set_error("unsupported number of GL points"); return DFR_E_INVAL;
  }
#undef DIAG_CASE
  DFR_HIP(hipGetLastError());
  dfr_launch(c, DFR_K_FINALIZE, diag_sum_kernel, dim3(1), dim3(BLOCK), 0, nb, (const double *)part, part + 3 * nb);
  DFR_HIP(hipGetLastError());
  return DFR_OK;
}

int launch_ode(Ctx *c, const double *q, const double *v, const double *vscale, bool jvp, double *out,
               const ArnoldiArgs *ar) {
  ArnoldiArgs none{};
  const ArnoldiArgs &a = ar ? *ar : none;
  const int kind = !jvp ? DFR_K_RHS : (a.on ? DFR_K_JV_ARNOLDI : DFR_K_JV);
  if (!jvp)
    dfr_launch(c, kind, ode_kernel<false, false>, dim3(1), dim3(ODE_THREADS), 0, c->ode, q, v, vscale, out, a);
  else if (a.on)
    dfr_launch(c, kind, ode_kernel<true, true>, dim3(1), dim3(ODE_THREADS), 0, c->ode, q, v, vscale, out, a);
  else
    dfr_launch(c, kind, ode_kernel<true, false>, dim3(1), dim3(ODE_THREADS), 0, c->ode, q, v, vscale, out, a);
  DFR_HIP(hipGetLastError());
  return DFR_OK;
}

__device__ __forceinline__ void w_interleave_body(int blk, int nblk, int64_t n, int p, double nu, const double *c0,
                                                  const double *c1, const double *c2, const double *c3, double *out,
                                                  int f32) {
  for (int64_t i = (int64_t)blk * BLOCK + threadIdx.x; i < n; i += (int64_t)nblk * BLOCK) {
    const double a0 = (p > 0 && c0) ? nu * c0[i] : 0.0;
    const double a1 = (p > 1 && c1) ? nu * c1[i] : 0.0;
    const double a2 = (p > 2 && c2) ? nu * c2[i] : 0.0;
    const double a3 = (p > 3 && c3) ? nu * c3[i] : 0.0;
    if (f32 && p <= 3) {   // FP32 columns, three per value (wil_code)
      float *o = reinterpret_cast<float *>(out) + 3 * i;
      o[0] = (float)a0;
      o[1] = (float)a1;
      o[2] = (float)a2;
    } else if (f32) {      // the columns of a call with an FP32 Krylov basis
      reinterpret_cast<float4 *>(out)[i] = make_float4((float)a0, (float)a1, (float)a2, (float)a3);
    } else {
      double2 *o = reinterpret_cast<double2 *>(out) + 2 * i;
      o[0] = make_double2(a0, a1);
      o[1] = make_double2(a2, a3);
    }
  }
}
__global__ __launch_bounds__(BLOCK) void w_interleave_kernel(int64_t n, int p, double nu, const double *c0,
                                                             const double *c1, const double *c2, const double *c3,
                                                             double *out, int f32) {
  w_interleave_body(blockIdx.x, gridDim.x, n, p, nu, c0, c1, c2, c3, out, f32);
}
__global__ __launch_bounds__(BLOCK) void w_interleave_batch(const WilCall *__restrict__ calls, int ncalls) {
  const WilCall &c = calls[find_call(calls, ncalls)];
  w_interleave_body(blockIdx.x - c.b0, c.nblk, c.n, c.p, c.nu, c.cols[0], c.cols[1], c.cols[2], c.cols[3], c.out,
                    c.f32);
}

int launch_w_interleave(Ctx *c, int64_t n, int p, double nu, const double *const *cols, double *out, bool f32) {
  if (p > 4) {
    set_error("interleaved W holds at most four columns");
    return DFR_E_INVAL;
  }
  const double *k[4] = {nullptr, nullptr, nullptr, nullptr};
  for (int i = 0; i < p; ++i) k[i] = cols[i];
  dfr_launch(c, DFR_K_OTHER, w_interleave_kernel, dim3(grid_for(n)), dim3(BLOCK), 0, n, p, nu, k[0], k[1], k[2], k[3],
             out, f32 ? 1 : 0);
  DFR_HIP(hipGetLastError());
  return DFR_OK;
}

int launch_wil_batch(hipStream_t s, Stage &st, std::vector<WilCall> &calls) {
  for (auto &c : calls)
    if (c.p > 4) {
      set_error("interleaved W holds at most four columns");
      return DFR_E_INVAL;
    }
  return launch_calls(s, st, calls, w_interleave_batch);
}


// ||x_i||_2^2 of several vectors: per-workgroup partial sums in
// partials[i * gridDim.x + blk], then one workgroup adds each set in a
// fixed order
struct VecSet {
  const double *x[MAX_P + 1];
};
__global__ __launch_bounds__(BLOCK) void multi_norm2_kernel(int64_t n, int k, const VecSet vs, double *partials) {
  __shared__ double red[BLOCK / 64];
  for (int i = 0; i < k; ++i) {
    const double *x = vs.x[i];
    double acc = 0.0;
    if (x)
      for (int64_t j = (int64_t)blockIdx.x * BLOCK + threadIdx.x; j < n; j += (int64_t)gridDim.x * BLOCK)
        acc += x[j] * x[j];
    const double s = block_sum(acc, red);
    if (threadIdx.x == 0) partials[(int64_t)i * gridDim.x + blockIdx.x] = s;
  }
}
__global__ __launch_bounds__(BLOCK) void multi_sum_kernel(int nb, int k, const double *partials, double *out,
                                                          unsigned *seq_out, unsigned seq) {
  __shared__ double red[BLOCK / 64];
  for (int i = 0; i < k; ++i) {
    double acc = 0.0;
    for (int b = threadIdx.x; b < nb; b += BLOCK) acc += partials[(int64_t)i * nb + b];
    const double s = block_sum(acc, red);
    if (threadIdx.x == 0) out[i] = s;
  }
  if (threadIdx.x == 0) {   // host-memory results: the sequence number last
    __threadfence_system();
    *(volatile unsigned *)seq_out = seq;
  }
}

// the latched error flags handed to the host and cleared, in stream order
__global__ void err_mail_kernel(int *err, int *out, unsigned *seq_out, unsigned seq) {
  if (threadIdx.x == 0) {
    *(volatile int *)out = atomicExch(err, 0);
    __threadfence_system();
    *(volatile unsigned *)seq_out = seq;
  }
}

int launch_err_mail(Ctx *c, unsigned seq) {
  hipLaunchKernelGGL(err_mail_kernel, dim3(1), dim3(64), 0, c->stream, c->d_err, &c->d_mail->err, &c->d_mail->seq, seq);
  DFR_HIP(hipGetLastError());
  return DFR_OK;
}

int launch_norms2(Ctx *c, int64_t n, int k, const double *const *x, double *partials, unsigned seq) {
  if (k < 1 || k > MAX_P + 1) {
    set_error("launch_norms2: too many vectors");
    return DFR_E_INVAL;
  }
  VecSet vs{};
  for (int i = 0; i < k; ++i) vs.x[i] = x[i];
  const int nb = grid_reduce(n);
  dfr_launch(c, DFR_K_OTHER, multi_norm2_kernel, dim3(nb), dim3(BLOCK), 0, n, k, vs, partials);
  DFR_HIP(hipGetLastError());
  dfr_launch(c, DFR_K_FINALIZE, multi_sum_kernel, dim3(1), dim3(BLOCK), 0, nb, k, (const double *)partials,
             c->d_mail->nrm2, &c->d_mail->seq, seq);
  DFR_HIP(hipGetLastError());
  return DFR_OK;
}

__device__ __forceinline__ void lincomb_body(int blk, int nblk, int64_t n, const LinComb &lc) {
  for (int64_t j = (int64_t)blk * BLOCK + threadIdx.x; j < n; j += (int64_t)nblk * BLOCK) {
    double x[4];
#pragma unroll
    for (int i = 0; i < 4; ++i) x[i] = i < lc.nin ? lc.in[i][j] : 0.0;
#pragma unroll
    for (int o = 0; o < 4; ++o) {
      if (o >= lc.nout) break;
      double s = 0.0;
#pragma unroll
      for (int i = 0; i < 4; ++i)
        if (i < lc.nin) s += lc.a[o][i] * x[i];
      lc.out[o][j] = s;
    }
  }
}
__global__ __launch_bounds__(BLOCK) void lincomb_kernel(int64_t n, const LinComb lc) {
  lincomb_body(blockIdx.x, gridDim.x, n, lc);
}
__global__ __launch_bounds__(BLOCK) void lincomb_batch(const LinCombCall *__restrict__ calls, int ncalls) {
  const LinCombCall &c = calls[find_call(calls, ncalls)];
  lincomb_body(blockIdx.x - c.b0, c.nblk, c.n, c.lc);
}

int launch_lincomb(Ctx *c, int64_t n, const LinComb &lc) {
  if (lc.nin < 1 || lc.nin > 4 || lc.nout < 1 || lc.nout > 4) {
    set_error("launch_lincomb: one to four inputs and outputs");
    return DFR_E_INVAL;
  }
  dfr_launch(c, DFR_K_OTHER, lincomb_kernel, dim3(grid_for(n)), dim3(BLOCK), 0, n, lc);
  DFR_HIP(hipGetLastError());
  return DFR_OK;
}

int launch_lincomb_batch(hipStream_t s, Stage &st, std::vector<LinCombCall> &calls) {
  for (auto &c : calls)
    if (c.lc.nin < 1 || c.lc.nin > 4 || c.lc.nout < 1 || c.lc.nout > 4) {
      set_error("launch_lincomb_batch: one to four inputs and outputs");
      return DFR_E_INVAL;
    }
  return launch_calls(s, st, calls, lincomb_batch);
}

}  // namespace dfrsw
