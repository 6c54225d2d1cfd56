// Pair physics for the tile skeleton (pairs.hpp).  Each functor stages the
// per-atom fields it needs (field-major in LDS) and evaluates one listed pair,
// adding both atoms' contributions to the LDS accumulators.
//
// R is the pair-arithmetic type: double (TK_FP64) or float (TK_MIXED).  With
// float the pair vector is formed in FP64 from the FP64 coordinates, the
// cutoff test stays in FP64 (identical pair decisions in both precisions),
// radial functions of same-molecule pairs are evaluated in FP64 (their
// screened-minus-bare differences cancel badly), pairs closer than 2 A are
// evaluated entirely in FP64 (their large forces would carry FP32 rounding of
// the same relative size), and every accumulation (LDS atomics, energies,
// virial) is FP64.  The van der Waals and point-charge terms are evaluated in
// FP64 in both forms (see VdwPh and ChargePh).
#pragma once

#include <type_traits>

#include "math.hpp"
#include "pairs.hpp"

namespace tk {

// Mixed form: pairs closer than 2 A (contacts; their forces are large, and
// FP32 rounding scales with them) are evaluated entirely in FP64.
constexpr double kMixedCloseR2 = 4.0;

template <class R>
inline const char* prec_tag() { return std::is_same<R, double>::value ? "_fp64" : "_fp32"; }

// Geometry and Ewald constants shared by the electrostatic terms.
struct Geom {
  double box, inv_box, rc2, beta, beta2, bsp_inv, cself;
  int bare;   // beta == 0: no screening, B_n = R_n
  void set(double b, double rc, double be) {
    box = b;
    inv_box = 1.0 / b;
    rc2 = rc * rc;
    beta = be;
    beta2 = be * be;
    bare = be == 0.0;
    bsp_inv = bare ? 0.0 : 1.0 / (be * kSqrtPi);
    cself = 4.0 * be * be * be / (3.0 * kSqrtPi);
  }
};

// B_0..B_N (Ewald-screened) and R_0..R_N (bare) at distance r:
//   B0 = erfc(beta r)/r,  Bn = [(2n-1) B(n-1) + (2 beta^2)^n exp(-beta^2 r^2)/(beta sqrt(pi))]/r^2
// erfc(beta r) = exp(-beta^2 r^2) erfcx(beta r): one exponential serves both.
template <class R, int N>
__device__ __forceinline__ void radial(const Geom& g, R r, R rinv, R* B, R* Rb, double r2d) {
  const R rinv2 = rinv * rinv;
  Rb[0] = rinv;
#pragma unroll
  for (int n = 1; n <= N; ++n) Rb[n] = R(2 * n - 1) * Rb[n - 1] * rinv2;
  if (g.bare) {
#pragma unroll
    for (int n = 0; n <= N; ++n) B[n] = Rb[n];
    return;
  }
  const R y = R(g.beta) * r;
  R e;
  if (std::is_same<R, float>::value)
    e = R(exp_neg_f32_of(-g.beta2 * r2d));   // argument -beta^2 r^2 kept in FP64
  else
    e = R(exp_neg((double)(-y * y)));
  const R b2 = R(2.0 * g.beta2);
  const R ex = e * R(g.bsp_inv);
  B[0] = e * erfcx(y) * rinv;
  R pw = b2;
#pragma unroll
  for (int n = 1; n <= N; ++n) {
    B[n] = (R(2 * n - 1) * B[n - 1] + pw * ex) * rinv2;
    pw *= b2;
  }
}

// g_n = B_n - w_n R_n; for R = float and same-molecule pairs the radial
// functions come from FP64 (B carries the FP64 difference B - R, Rb is zero).
template <class R, int N>
__device__ __forceinline__ void radial_pair(const Geom& g, double r2, bool same_mol, R* B, R* Rb) {
  if (std::is_same<R, float>::value && same_mol) {
    const double ri = rsqrt_r(r2), r = r2 * ri;
    double Bd[N + 1], Rd[N + 1];
    radial<double, N>(g, r, ri, Bd, Rd, r2);
#pragma unroll
    for (int n = 0; n <= N; ++n) {
      B[n] = R(Bd[n] - Rd[n]);
      Rb[n] = R(0);
    }
    return;
  }
  const R rinv = rsqrt_r(R(r2));
  const R r = R(r2) * rinv;
  radial<R, N>(g, r, rinv, B, Rb, r2);
}

// Thole factors l3, l5, l7 with x = a_ij r^3 isa_i isa_j, isa = 1/sqrt(alpha)
// (0 when alpha = 0, which makes every factor 1).
template <class R>
__device__ __forceinline__ void thole_damp(R r, R isa_i, R isa_j, R ti, R tj, R& l3, R& l5, R& l7) {
  const R pr = isa_i * isa_j;
  if (pr == R(0)) {
    l3 = l5 = l7 = R(1);
    return;
  }
  const R a = ti < tj ? ti : tj;
  const R x = a * r * r * r * pr;
  const R e = exp_neg(-x);
  l3 = R(1) - e;
  l5 = R(1) - (R(1) + x) * e;
  l7 = R(1) - (R(1) + x + R(0.6) * x * x) * e;
}

// l3, l5, l7 and l9 = 1 - (1 + x + 18/35 x^2 + 9/35 x^3) e^-x; the family
// (l_(2n+1) R_n) obeys the same gradient rule as B_n and R_n, l9 being the
// factor the gradient of the damped quadrupole field needs.
template <class R>
__device__ __forceinline__ void thole_damp9(R r, R isa_i, R isa_j, R ti, R tj, R* l) {
  const R pr = isa_i * isa_j;
  if (pr == R(0)) {
    l[0] = l[1] = l[2] = l[3] = R(1);
    return;
  }
  const R a = ti < tj ? ti : tj;
  const R x = a * r * r * r * pr;
  const R e = exp_neg(-x);
  const R x2 = x * x;
  l[0] = R(1) - e;
  l[1] = R(1) - (R(1) + x) * e;
  l[2] = R(1) - (R(1) + x + R(0.6) * x2) * e;
  l[3] = R(1) - (R(1) + x + R(18.0 / 35.0) * x2 + R(9.0 / 35.0) * x2 * x) * e;
}

__device__ __forceinline__ double inv_sqrt_alpha(double a) { return a > 0.0 ? 1.0 / sqrt(a) : 0.0; }

// --------------------------------------------------------------------------
// Permanent multipoles: energy, forces, virial.
// Fields: x y z | q mux muy muz Txx Txy Txz Tyy Tyz Tzz | molid
template <class R>
struct EmpolePh {
  static constexpr int NF = 14, NA = 3, NS = 11;
  static constexpr const char* kName = "empole";
  static constexpr int kWaves = 2;   // waves per unit (pairs.hpp launch_units)
  static constexpr const char* kTag = std::is_same<R, double>::value ? "_fp64" : "_fp32";
  __device__ bool skip() const { return false; }
  __device__ void prologue(int tid, int nt) const { erfcx_stage<R>(tid, nt); }
  const double* xyz;
  const double* mpole;
  const int32_t* molid;
  Geom g;
  __device__ void set_sys(const SysDev& d, int) {
    g.box = d.box;
    g.inv_box = d.inv_box;
  }
    static constexpr int NG = 14;   // fields gathered once per call (sorted SoA)
  const double* sorted = nullptr;
  long gstride = 0;
  __device__ void stage_dyn(double*, int, int, int) const {}
  __device__ void gather(int i, double* g) const {
#pragma unroll
    for (int c = 0; c < 3; ++c) g[c] = xyz[3 * i + c];
#pragma unroll
    for (int k = 0; k < 10; ++k) g[3 + k] = mpole[10 * i + k];
    g[13] = (double)molid[i];
  }
  // pair energy and de/dr in arithmetic type T
  template <class T>
  __device__ __forceinline__ void eval(const double* LH, const double* LK, int cap, int a, int b,
                                       const double* dd, double r2, bool excl, double* de,
                                       double& en) const {
    T B[6], Rb[6];
    radial_pair<T, 5>(g, r2, excl, B, Rb);
    T gg[6];
#pragma unroll
    for (int n = 0; n < 6; ++n) gg[n] = excl ? B[n] - Rb[n] : B[n];
    const T d[3] = {T(dd[0]), T(dd[1]), T(dd[2])};
    const T qi = T(LH[3 * cap + a]), qj = T(LK[3 * cap + b]);
    const T ui[3] = {T(LH[4 * cap + a]), T(LH[5 * cap + a]), T(LH[6 * cap + a])};
    const T uj[3] = {T(LK[4 * cap + b]), T(LK[5 * cap + b]), T(LK[6 * cap + b])};
    // Theta as 6 unique components xx xy xz yy yz zz
    const T ti[6] = {T(LH[7 * cap + a]), T(LH[8 * cap + a]), T(LH[9 * cap + a]),
                     T(LH[10 * cap + a]), T(LH[11 * cap + a]), T(LH[12 * cap + a])};
    const T tj[6] = {T(LK[7 * cap + b]), T(LK[8 * cap + b]), T(LK[9 * cap + b]),
                     T(LK[10 * cap + b]), T(LK[11 * cap + b]), T(LK[12 * cap + b])};
    auto tmul = [](const T* t, const T* x, T* y) {
      y[0] = t[0] * x[0] + t[1] * x[1] + t[2] * x[2];
      y[1] = t[1] * x[0] + t[3] * x[1] + t[4] * x[2];
      y[2] = t[2] * x[0] + t[4] * x[1] + t[5] * x[2];
    };
    auto dot = [](const T* x, const T* y) { return x[0] * y[0] + x[1] * y[1] + x[2] * y[2]; };
    T vi[3], vj[3];
    tmul(ti, d, vi);
    tmul(tj, d, vj);
    const T di = dot(ui, d), dj = dot(uj, d), Qi = dot(d, vi), Qj = dot(d, vj);
    const T tt = ti[0] * tj[0] + ti[3] * tj[3] + ti[5] * tj[5] +
                 T(2) * (ti[1] * tj[1] + ti[2] * tj[2] + ti[4] * tj[4]);
    const T c0 = qi * qj;
    const T c1 = qj * di - qi * dj + dot(ui, uj);
    const T c2 = qi * Qj + qj * Qi - di * dj + T(2) * (dot(uj, vi) - dot(ui, vj) + tt);
    const T c3 = di * Qj - dj * Qi - T(4) * dot(vi, vj);
    const T c4 = Qi * Qj;
    T tiuj[3], tjui[3], tivj[3], tjvi[3];
    tmul(ti, uj, tiuj);
    tmul(tj, ui, tjui);
    tmul(ti, vj, tivj);
    tmul(tj, vi, tjvi);
    const T e = c0 * gg[0] + c1 * gg[1] + c2 * gg[2] + c3 * gg[3] + c4 * gg[4];
    const T sr = c0 * gg[1] + c1 * gg[2] + c2 * gg[3] + c3 * gg[4] + c4 * gg[5];
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      const T dc1 = qj * ui[c] - qi * uj[c];
      const T dc2 = T(2) * (qi * vj[c] + qj * vi[c]) - dj * ui[c] - di * uj[c] +
                    T(2) * (tiuj[c] - tjui[c]);
      const T dc3 = Qj * ui[c] + T(2) * di * vj[c] - Qi * uj[c] - T(2) * dj * vi[c] -
                    T(4) * (tivj[c] + tjvi[c]);
      const T dc4 = T(2) * (Qj * vi[c] + Qi * vj[c]);
      de[c] = kCoulomb * (double)(dc1 * gg[1] + dc2 * gg[2] + dc3 * gg[3] + dc4 * gg[4] - sr * d[c]);
    }
    en = kCoulomb * (double)e;
  }
  __device__ void pair(const double* LH, const double* LK, int cap, int a, int b, double* AH,
                       double* AK, double* sc, long) const {
    double dd[3];
    const double r2 = image3(LH, LK, cap, a, b, g.box, g.inv_box, dd);
    if (!(r2 <= g.rc2)) return;
    const bool excl = LH[13 * cap + a] == LK[13 * cap + b];
    double de[3], en;
    if (std::is_same<R, float>::value && r2 < kMixedCloseR2)
      eval<double>(LH, LK, cap, a, b, dd, r2, excl, de, en);
    else
      eval<R>(LH, LK, cap, a, b, dd, r2, excl, de, en);
    sc[excl ? 1 : 0] += en;
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      lds_add(&AH[c * cap + a], de[c]);
      lds_add(&AK[c * cap + b], -de[c]);
#pragma unroll
      for (int q = 0; q < 3; ++q) sc[2 + 3 * c + q] += dd[c] * de[q];
    }
  }
};

// Point charges: e = C qi qj g0, de/dr = -C qi qj g1 r.
// Fields: x y z | q | molid
template <class R>
struct ChargePh {
  static constexpr int NF = 5, NA = 3, NS = 11;
  static constexpr const char* kName = "charge";
  // waves per unit (pairs.hpp launch_units): on the 12 A lists of the charge
  // path two measured faster than four (332 against 352 us, 96,000 atoms)
  static constexpr int kWaves = 2;
  static constexpr const char* kTag = std::is_same<R, double>::value ? "_fp64" : "_fp32";
  __device__ bool skip() const { return false; }
  __device__ void prologue(int tid, int nt) const { erfcx_stage<R>(tid, nt); }
  const double* xyz;
  const double* q;
  const int32_t* molid;
  Geom g;
  __device__ void set_sys(const SysDev& d, int) {
    g.box = d.box;
    g.inv_box = d.inv_box;
  }
    static constexpr int NG = 5;   // fields gathered once per call (sorted SoA)
  const double* sorted = nullptr;
  long gstride = 0;
  __device__ void stage_dyn(double*, int, int, int) const {}
  __device__ void gather(int i, double* g) const {
#pragma unroll
    for (int c = 0; c < 3; ++c) g[c] = xyz[3 * i + c];
    g[3] = q[i];
    g[4] = (double)molid[i];
  }
  __device__ void pair(const double* LH, const double* LK, int cap, int a, int b, double* AH,
                       double* AK, double* sc, long) const {
    double dd[3];
    const double r2 = image3(LH, LK, cap, a, b, g.box, g.inv_box, dd);
    if (!(r2 <= g.rc2)) return;
    const bool excl = LH[4 * cap + a] == LK[4 * cap + b];
    // Both forms evaluate the pair once in FP64: the energy of a point-charge
    // system is a large cancelling sum that needs its screened term g0 in
    // FP64, and the FP64 erfc and exponential that give g0 give g1 too, so an
    // FP32 force on top would cost more than it saves.
    double B[2], Rb[2];
    radial_pair<double, 1>(g, r2, excl, B, Rb);
    const double g0 = excl ? B[0] - Rb[0] : B[0];
    const double g1 = excl ? B[1] - Rb[1] : B[1];
    const double qq = kCoulomb * LH[3 * cap + a] * LK[3 * cap + b];
    const double en = qq * g0;
    const double f = -qq * g1;
    sc[excl ? 1 : 0] += en;
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      const double de = f * dd[c];
      lds_add(&AH[c * cap + a], de);
      lds_add(&AK[c * cap + b], -de);
#pragma unroll
      for (int k = 0; k < 3; ++k) sc[2 + 3 * c + k] += dd[c] * f * dd[k];
    }
  }
};

// Permanent field (right-hand side of the polarization equations).
// Fields: x y z | q mu(3) Theta(6) | molid | isa | thole
template <class R>
struct EfieldPh {
  static constexpr int NF = 16, NA = 3, NS = 0;
  static constexpr const char* kName = "efield";
  static constexpr int kWaves = 2;   // waves per unit (pairs.hpp launch_units)
  static constexpr const char* kTag = std::is_same<R, double>::value ? "_fp64" : "_fp32";
  __device__ bool skip() const { return false; }
  __device__ void prologue(int tid, int nt) const { erfcx_stage<R>(tid, nt); }
  const double* xyz;
  const double* mpole;
  const int32_t* molid;
  const double* polarity;
  const double* thole;
  Geom g;
  __device__ void set_sys(const SysDev& d, int) {
    g.box = d.box;
    g.inv_box = d.inv_box;
  }
    static constexpr int NG = 16;   // fields gathered once per call (sorted SoA)
  const double* sorted = nullptr;
  long gstride = 0;
  __device__ void stage_dyn(double*, int, int, int) const {}
  __device__ void gather(int i, double* g) const {
#pragma unroll
    for (int c = 0; c < 3; ++c) g[c] = xyz[3 * i + c];
#pragma unroll
    for (int k = 0; k < 10; ++k) g[3 + k] = mpole[10 * i + k];
    g[13] = (double)molid[i];
    g[14] = inv_sqrt_alpha(polarity[i]);
    g[15] = thole[i];
  }
  // Optional by-product for the solver: the mutual-field radial factors of
  // the pair (same molecule included, Thole-damped), gc[p] = g1, gc[gcs + p]
  // = g2, zero beyond the cutoff.  The permanent and mutual kernels differ
  // only on same-molecule pairs (scale 0 vs 1), so one pass yields both.
  using GC = R;
  GC* gc = nullptr;
  long gcs = 0;
  // factor on the damped part of same-molecule pairs (0: the direct field)
  double intra = 0.0;
  // field contributions at both atoms (fi at H's atom, fj at K's) in type T
  template <class T>
  __device__ __forceinline__ void eval(const double* LH, const double* LK, int cap, int a, int b,
                                       const double* dd, double r2, bool excl, double* fi,
                                       double* fj, long p) const {
    T B[4], Rb[4];
    radial_pair<T, 3>(g, r2, excl, B, Rb);
    T g1, g2, g3;
    T l3, l5, l7;
    if (!excl || gc || intra != 0.0) {
      const T r = T(r2) * rsqrt_r(T(r2));
      thole_damp<T>(r, T(LH[14 * cap + a]), T(LK[14 * cap + b]), T(LH[15 * cap + a]),
                    T(LK[15 * cap + b]), l3, l5, l7);
    }
    if (excl) {
      if (intra == 0.0) {
        g1 = B[1] - Rb[1];
        g2 = B[2] - Rb[2];
        g3 = B[3] - Rb[3];
      } else if (std::is_same<T, float>::value) {
        // B carries the FP64 difference B - R; add the scaled damped bare part in FP64
        const double ri = rsqrt_r(r2);
        const double R1 = ri * ri * ri, R2 = 3.0 * R1 * ri * ri, R3 = 5.0 * R2 * ri * ri;
        g1 = T((double)B[1] + intra * (double)l3 * R1);
        g2 = T((double)B[2] + intra * (double)l5 * R2);
        g3 = T((double)B[3] + intra * (double)l7 * R3);
      } else {
        g1 = B[1] - (T(1) - T(intra) * l3) * Rb[1];
        g2 = B[2] - (T(1) - T(intra) * l5) * Rb[2];
        g3 = B[3] - (T(1) - T(intra) * l7) * Rb[3];
      }
      if (gc) {
        if (std::is_same<T, float>::value) {
          // B carries the FP64 difference B - R; re-add the damped bare part in FP64
          const double ri = rsqrt_r(r2);
          const double R1 = ri * ri * ri, R2 = 3.0 * R1 * ri * ri;
          gc[p] = GC((double)B[1] + (double)l3 * R1);
          gc[gcs + p] = GC((double)B[2] + (double)l5 * R2);
        } else {
          gc[p] = GC(B[1] - (T(1) - l3) * Rb[1]);
          gc[gcs + p] = GC(B[2] - (T(1) - l5) * Rb[2]);
        }
      }
    } else {
      g1 = B[1] - (T(1) - l3) * Rb[1];
      g2 = B[2] - (T(1) - l5) * Rb[2];
      g3 = B[3] - (T(1) - l7) * Rb[3];
      if (gc) {
        gc[p] = GC(g1);
        gc[gcs + p] = GC(g2);
      }
    }
    const T d[3] = {T(dd[0]), T(dd[1]), T(dd[2])};
    const T qi = T(LH[3 * cap + a]), qj = T(LK[3 * cap + b]);
    const T ui[3] = {T(LH[4 * cap + a]), T(LH[5 * cap + a]), T(LH[6 * cap + a])};
    const T uj[3] = {T(LK[4 * cap + b]), T(LK[5 * cap + b]), T(LK[6 * cap + b])};
    const T ti[6] = {T(LH[7 * cap + a]), T(LH[8 * cap + a]), T(LH[9 * cap + a]),
                     T(LH[10 * cap + a]), T(LH[11 * cap + a]), T(LH[12 * cap + a])};
    const T tj[6] = {T(LK[7 * cap + b]), T(LK[8 * cap + b]), T(LK[9 * cap + b]),
                     T(LK[10 * cap + b]), T(LK[11 * cap + b]), T(LK[12 * cap + b])};
    T vi[3], vj[3];
    vi[0] = ti[0] * d[0] + ti[1] * d[1] + ti[2] * d[2];
    vi[1] = ti[1] * d[0] + ti[3] * d[1] + ti[4] * d[2];
    vi[2] = ti[2] * d[0] + ti[4] * d[1] + ti[5] * d[2];
    vj[0] = tj[0] * d[0] + tj[1] * d[1] + tj[2] * d[2];
    vj[1] = tj[1] * d[0] + tj[3] * d[1] + tj[4] * d[2];
    vj[2] = tj[2] * d[0] + tj[4] * d[1] + tj[5] * d[2];
    const T di = ui[0] * d[0] + ui[1] * d[1] + ui[2] * d[2];
    const T dj = uj[0] * d[0] + uj[1] * d[1] + uj[2] * d[2];
    const T Qi = d[0] * vi[0] + d[1] * vi[1] + d[2] * vi[2];
    const T Qj = d[0] * vj[0] + d[1] * vj[1] + d[2] * vj[2];
    // field at i from j: d(-qj g1 + dj g2 - Qj g3) - uj g1 + 2 vj g2
    // field at j from i: d( qi g1 + di g2 + Qi g3) - ui g1 - 2 vi g2
    const T si = -qj * g1 + dj * g2 - Qj * g3;
    const T sj = qi * g1 + di * g2 + Qi * g3;
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      fi[c] = (double)(d[c] * si - uj[c] * g1 + T(2) * vj[c] * g2);
      fj[c] = (double)(d[c] * sj - ui[c] * g1 - T(2) * vi[c] * g2);
    }
  }
  __device__ void pair(const double* LH, const double* LK, int cap, int a, int b, double* AH,
                       double* AK, double*, long p) const {
    double dd[3];
    const double r2 = image3(LH, LK, cap, a, b, g.box, g.inv_box, dd);
    if (!(r2 <= g.rc2)) {
      if (gc) {
        gc[p] = GC(0);
        gc[gcs + p] = GC(0);
      }
      return;
    }
    const bool excl = LH[13 * cap + a] == LK[13 * cap + b];
    double fi[3], fj[3];
    if (std::is_same<R, float>::value && r2 < kMixedCloseR2)
      eval<double>(LH, LK, cap, a, b, dd, r2, excl, fi, fj, p);
    else
      eval<R>(LH, LK, cap, a, b, dd, r2, excl, fi, fj, p);
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      lds_add(&AH[c * cap + a], fi[c]);
      lds_add(&AK[c * cap + b], fj[c]);
    }
  }
};

// Permanent multipoles and their field in one pass over the list: the
// multipole energy, forces and virial (as EmpolePh) and the Thole-damped
// permanent field at both atoms (as EfieldPh), the two routines of the Rel
// profile that walk the same pairs with the same radial functions.  The pair
// vector, B_0..B_5, the quadrupole contractions Theta d and d.Theta.d and the
// dipole projections are formed once for both; the solver's mutual-field
// factors are cached per pair code (gc, as EfieldPh).  Accumulators: force
// (3), field (3).
// Fields: x y z | q mu(3) Theta(6) | molid | isa | thole
template <class R>
struct MpoleFieldPh {
  static constexpr int NF = 16, NA = 6, NS = 11;
  static constexpr const char* kName = "mpole_field";
  static constexpr int kWaves = 1;   // one wave per unit: 73 us against 89 with two (water box)
  static constexpr const char* kTag = std::is_same<R, double>::value ? "_fp64" : "_fp32";
  __device__ bool skip() const { return false; }
  __device__ void prologue(int tid, int nt) const { erfcx_stage<R>(tid, nt); }
  const double* xyz;
  const double* mpole;
  const int32_t* molid;
  const double* polarity;
  const double* thole;
  Geom g;
  __device__ void set_sys(const SysDev& d, int) {
    g.box = d.box;
    g.inv_box = d.inv_box;
  }
  static constexpr int NG = 16;   // fields gathered once per call (sorted SoA)
  const double* sorted = nullptr;
  long gstride = 0;
  __device__ void stage_dyn(double*, int, int, int) const {}
  __device__ void gather(int i, double* g) const {
#pragma unroll
    for (int c = 0; c < 3; ++c) g[c] = xyz[3 * i + c];
#pragma unroll
    for (int k = 0; k < 10; ++k) g[3 + k] = mpole[10 * i + k];
    g[13] = (double)molid[i];
    g[14] = inv_sqrt_alpha(polarity[i]);
    g[15] = thole[i];
  }
  using GC = R;
  GC* gc = nullptr;   // [2][gcs]: g1 | g2 per pair code
  long gcs = 0;
  // de: dE/dr (the force on K's atom is -de), en: pair energy, fi/fj: the
  // permanent field at H's and K's atom, all in type T
  template <class T>
  __device__ __forceinline__ void eval(const double* LH, const double* LK, int cap, int a, int b,
                                       const double* dd, double r2, bool excl, double* de,
                                       double& en, double* fi, double* fj, long p) const {
    T B[6], Rb[6];
    radial_pair<T, 5>(g, r2, excl, B, Rb);
    T gg[6];
#pragma unroll
    for (int n = 0; n < 6; ++n) gg[n] = excl ? B[n] - Rb[n] : B[n];
    T l3, l5, l7;
    const T r = T(r2) * rsqrt_r(T(r2));
    thole_damp<T>(r, T(LH[14 * cap + a]), T(LK[14 * cap + b]), T(LH[15 * cap + a]),
                  T(LK[15 * cap + b]), l3, l5, l7);
    // field factors: bare Coulomb removed within a molecule (the permanent
    // field), Thole-damped otherwise; the mutual factors (damped for every
    // pair) go to the cache
    T g1, g2, g3;
    if (excl) {
      g1 = B[1] - Rb[1];
      g2 = B[2] - Rb[2];
      g3 = B[3] - Rb[3];
      if (gc) {
        if (std::is_same<T, float>::value) {
          // B carries the FP64 difference B - R; re-add the damped bare part in FP64
          const double ri = rsqrt_r(r2);
          const double R1 = ri * ri * ri, R2 = 3.0 * R1 * ri * ri;
          gc[p] = GC((double)B[1] + (double)l3 * R1);
          gc[gcs + p] = GC((double)B[2] + (double)l5 * R2);
        } else {
          gc[p] = GC(B[1] - (T(1) - l3) * Rb[1]);
          gc[gcs + p] = GC(B[2] - (T(1) - l5) * Rb[2]);
        }
      }
    } else {
      g1 = B[1] - (T(1) - l3) * Rb[1];
      g2 = B[2] - (T(1) - l5) * Rb[2];
      g3 = B[3] - (T(1) - l7) * Rb[3];
      if (gc) {
        gc[p] = GC(g1);
        gc[gcs + p] = GC(g2);
      }
    }
    const T d[3] = {T(dd[0]), T(dd[1]), T(dd[2])};
    const T qi = T(LH[3 * cap + a]), qj = T(LK[3 * cap + b]);
    const T ui[3] = {T(LH[4 * cap + a]), T(LH[5 * cap + a]), T(LH[6 * cap + a])};
    const T uj[3] = {T(LK[4 * cap + b]), T(LK[5 * cap + b]), T(LK[6 * cap + b])};
    const T ti[6] = {T(LH[7 * cap + a]), T(LH[8 * cap + a]), T(LH[9 * cap + a]),
                     T(LH[10 * cap + a]), T(LH[11 * cap + a]), T(LH[12 * cap + a])};
    const T tj[6] = {T(LK[7 * cap + b]), T(LK[8 * cap + b]), T(LK[9 * cap + b]),
                     T(LK[10 * cap + b]), T(LK[11 * cap + b]), T(LK[12 * cap + b])};
    auto tmul = [](const T* t, const T* x, T* y) {
      y[0] = t[0] * x[0] + t[1] * x[1] + t[2] * x[2];
      y[1] = t[1] * x[0] + t[3] * x[1] + t[4] * x[2];
      y[2] = t[2] * x[0] + t[4] * x[1] + t[5] * x[2];
    };
    auto dot = [](const T* x, const T* y) { return x[0] * y[0] + x[1] * y[1] + x[2] * y[2]; };
    T vi[3], vj[3];
    tmul(ti, d, vi);
    tmul(tj, d, vj);
    const T di = dot(ui, d), dj = dot(uj, d), Qi = dot(d, vi), Qj = dot(d, vj);
    // multipole energy and its gradient
    const T tt = ti[0] * tj[0] + ti[3] * tj[3] + ti[5] * tj[5] +
                 T(2) * (ti[1] * tj[1] + ti[2] * tj[2] + ti[4] * tj[4]);
    const T c0 = qi * qj;
    const T c1 = qj * di - qi * dj + dot(ui, uj);
    const T c2 = qi * Qj + qj * Qi - di * dj + T(2) * (dot(uj, vi) - dot(ui, vj) + tt);
    const T c3 = di * Qj - dj * Qi - T(4) * dot(vi, vj);
    const T c4 = Qi * Qj;
    T tiuj[3], tjui[3], tivj[3], tjvi[3];
    tmul(ti, uj, tiuj);
    tmul(tj, ui, tjui);
    tmul(ti, vj, tivj);
    tmul(tj, vi, tjvi);
    const T e = c0 * gg[0] + c1 * gg[1] + c2 * gg[2] + c3 * gg[3] + c4 * gg[4];
    const T sr = c0 * gg[1] + c1 * gg[2] + c2 * gg[3] + c3 * gg[4] + c4 * gg[5];
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      const T dc1 = qj * ui[c] - qi * uj[c];
      const T dc2 = T(2) * (qi * vj[c] + qj * vi[c]) - dj * ui[c] - di * uj[c] +
                    T(2) * (tiuj[c] - tjui[c]);
      const T dc3 = Qj * ui[c] + T(2) * di * vj[c] - Qi * uj[c] - T(2) * dj * vi[c] -
                    T(4) * (tivj[c] + tjvi[c]);
      const T dc4 = T(2) * (Qj * vi[c] + Qi * vj[c]);
      de[c] = kCoulomb * (double)(dc1 * gg[1] + dc2 * gg[2] + dc3 * gg[3] + dc4 * gg[4] - sr * d[c]);
    }
    en = kCoulomb * (double)e;
    // permanent field: at i from j: d(-qj g1 + dj g2 - Qj g3) - uj g1 + 2 vj g2;
    // at j from i: d(qi g1 + di g2 + Qi g3) - ui g1 - 2 vi g2
    const T si = -qj * g1 + dj * g2 - Qj * g3;
    const T sj = qi * g1 + di * g2 + Qi * g3;
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      fi[c] = (double)(d[c] * si - uj[c] * g1 + T(2) * vj[c] * g2);
      fj[c] = (double)(d[c] * sj - ui[c] * g1 - T(2) * vi[c] * g2);
    }
  }
  __device__ void pair(const double* LH, const double* LK, int cap, int a, int b, double* AH,
                       double* AK, double* sc, long p) const {
    double dd[3];
    const double r2 = image3(LH, LK, cap, a, b, g.box, g.inv_box, dd);
    if (!(r2 <= g.rc2)) {
      if (gc) {
        gc[p] = GC(0);
        gc[gcs + p] = GC(0);
      }
      return;
    }
    const bool excl = LH[13 * cap + a] == LK[13 * cap + b];
    double de[3], en, fi[3], fj[3];
    if (std::is_same<R, float>::value && r2 < kMixedCloseR2)
      eval<double>(LH, LK, cap, a, b, dd, r2, excl, de, en, fi, fj, p);
    else
      eval<R>(LH, LK, cap, a, b, dd, r2, excl, de, en, fi, fj, p);
    sc[excl ? 1 : 0] += en;
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      lds_add(&AH[c * cap + a], de[c]);
      lds_add(&AK[c * cap + b], -de[c]);
      lds_add(&AH[(3 + c) * cap + a], fi[c]);
      lds_add(&AK[(3 + c) * cap + b], fj[c]);
#pragma unroll
      for (int q = 0; q < 3; ++q) sc[2 + 3 * c + q] += dd[c] * de[q];
    }
  }
};

// Mutual induced-dipole field: E_i += T2 mu_j, E_j += T2 mu_i (all pairs).
// Fields: x y z | isa | thole | molid | mu(3)
template <class R>
struct TmatPh {
  static constexpr int NF = 9, NA = 3, NS = 0;
  static constexpr const char* kName = "tmat";
  static constexpr int kWaves = 4;   // waves per unit (pairs.hpp launch_units)
  static constexpr const char* kTag = std::is_same<R, double>::value ? "_fp64" : "_fp32";
  const int* done = nullptr;   // solver flag (status; 0 while iterating)
  int run_when_done = 0;       // 0: skip once the solver has finished; 1: skip until it has
  __device__ bool skip() const { return done && ((*done != 0) != (run_when_done != 0)); }
  __device__ void prologue(int tid, int nt) const { erfcx_stage<R>(tid, nt); }
  const double* xyz;
  const double* mu;
  int mu_sorted;   // mu indexed by sorted position (solver-internal vectors)
  const double* polarity;
  const double* thole;
  const int32_t* molid;
  Geom g;
  __device__ void set_sys(const SysDev& d, int) {
    g.box = d.box;
    g.inv_box = d.inv_box;
  }
  const double* zdir = nullptr;      // solver: stage p = z + beta * p (search direction)
  const double* beta_dir = nullptr;  // device scalar beta
  static constexpr int NG = 6;       // x y z isa thole molid, gathered once per call
  const double* sorted = nullptr;
  long gstride = 0;
  __device__ void gather(int i, double* g) const {
#pragma unroll
    for (int c = 0; c < 3; ++c) g[c] = xyz[3 * i + c];
    g[3] = inv_sqrt_alpha(polarity[i]);
    g[4] = thole[i];
    g[5] = molid ? (double)molid[i] : (double)i;
  }
  // dipoles (or the solver's search direction) are read per call
  __device__ void stage_dyn(double* L, int cap, int t, int s) const {
    const int32_t* pm = perm_;
    const int m = mu_sorted ? s : pm[s];
    const double bd = zdir ? *beta_dir : 0.0;
#pragma unroll
    for (int c = 0; c < 3; ++c)
      L[(6 + c) * cap + t] = zdir ? fma(bd, mu[3 * m + c], zdir[3 * m + c]) : mu[3 * m + c];
  }
  const int32_t* perm_ = nullptr;

  // field contributions at both atoms in type T
  template <class T>
  __device__ __forceinline__ void eval(const double* LH, const double* LK, int cap, int a, int b,
                                       const double* dd, double r2, bool same, double* fi,
                                       double* fj) const {
    T B[3], Rb[3];
    radial_pair<T, 2>(g, r2, same, B, Rb);
    T l3, l5, l7;
    const T r = T(r2) * rsqrt_r(T(r2));
    thole_damp<T>(r, T(LH[3 * cap + a]), T(LK[3 * cap + b]), T(LH[4 * cap + a]),
                  T(LK[4 * cap + b]), l3, l5, l7);
    // g1 = B1 - (1 - l3) R1, g2 = B2 - (1 - l5) R2 (for FP32 same-molecule pairs
    // B carries the FP64 difference B - R and the bare part is re-added with l)
    T g1, g2;
    if (std::is_same<T, float>::value && same) {
      const double ri = rsqrt_r(r2);
      const double R1 = ri * ri * ri, R2 = 3.0 * R1 * ri * ri;
      g1 = T((double)B[1] + (double)l3 * R1);
      g2 = T((double)B[2] + (double)l5 * R2);
    } else {
      g1 = B[1] - (T(1) - l3) * Rb[1];
      g2 = B[2] - (T(1) - l5) * Rb[2];
    }
    const T d[3] = {T(dd[0]), T(dd[1]), T(dd[2])};
    const T ui[3] = {T(LH[6 * cap + a]), T(LH[7 * cap + a]), T(LH[8 * cap + a])};
    const T uj[3] = {T(LK[6 * cap + b]), T(LK[7 * cap + b]), T(LK[8 * cap + b])};
    const T di = ui[0] * d[0] + ui[1] * d[1] + ui[2] * d[2];
    const T dj = uj[0] * d[0] + uj[1] * d[1] + uj[2] * d[2];
    const T si = dj * g2, sj = di * g2;
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      fi[c] = (double)(d[c] * si - uj[c] * g1);
      fj[c] = (double)(d[c] * sj - ui[c] * g1);
    }
  }
  __device__ void pair(const double* LH, const double* LK, int cap, int a, int b, double* AH,
                       double* AK, double*, long) const {
    double dd[3];
    const double r2 = image3(LH, LK, cap, a, b, g.box, g.inv_box, dd);
    if (!(r2 <= g.rc2)) return;
    const bool same = LH[5 * cap + a] == LK[5 * cap + b];
    double fi[3], fj[3];
    if (std::is_same<R, float>::value && r2 < kMixedCloseR2)
      eval<double>(LH, LK, cap, a, b, dd, r2, same, fi, fj);
    else
      eval<R>(LH, LK, cap, a, b, dd, r2, same, fi, fj);
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      lds_add(&AH[c * cap + a], fi[c]);
      lds_add(&AK[c * cap + b], fj[c]);
    }
  }
};


// Halgren 14-7 / LJ 12-6 with the quintic taper.
// Fields: x y z | radius (HAL R or LJ sigma) | sqrt(eps) | molid
template <class R>
struct VdwPh {
  static constexpr int NF = 6, NA = 3, NS = 10;
  static constexpr const char* kName = "vdw";
  static constexpr int kWaves = 4;   // waves per unit (pairs.hpp launch_units)
  static constexpr const char* kTag = std::is_same<R, double>::value ? "_fp64" : "_fp32";
  __device__ bool skip() const { return false; }
  __device__ void prologue(int, int) const {}
  const double* xyz;
  const double* rad;
  const double* eps;
  const int32_t* molid;
  int form;
  double box, inv_box, rc2, ron, rc, tw_inv, dhal, ghal, taper;
  const double* sys_cut = nullptr;   // batch: per-system cutoff (nullptr: rc for all)
  __host__ __device__ void set_cut(double cutoff) {
    rc = cutoff;
    rc2 = cutoff * cutoff;
    ron = taper * cutoff;
    tw_inv = cutoff > ron ? 1.0 / (cutoff - ron) : 0.0;
  }
  void set(const tk_system* sys, int f, const double* r_, const double* e_, double cutoff,
           double tp, double d, double gm) {
    xyz = sys->xyz;
    rad = r_;
    eps = e_;
    molid = sys->molid;
    form = f;
    box = sys->box;
    inv_box = 1.0 / sys->box;
    taper = tp;
    set_cut(cutoff);
    dhal = d;
    ghal = gm;
  }
  __device__ void set_sys(const SysDev& d, int sy) {
    box = d.box;
    inv_box = d.inv_box;
    if (sys_cut) set_cut(sys_cut[sy]);
  }
    static constexpr int NG = 6;   // fields gathered once per call (sorted SoA)
  const double* sorted = nullptr;
  long gstride = 0;
  __device__ void stage_dyn(double*, int, int, int) const {}
  __device__ void gather(int i, double* g) const {
#pragma unroll
    for (int c = 0; c < 3; ++c) g[c] = xyz[3 * i + c];
    g[3] = rad[i];
    g[4] = sqrt(eps[i]);
    g[5] = (double)molid[i];
  }
  // HAL / LJ pair energy and de/dr with the taper, in arithmetic type T;
  // ir = 1/r.  The HAL form's three denominators (combining rule for eps,
  // rho + ghal rv^7, r + dhal rv) share one reciprocal of their product.
  template <class T>
  __device__ __forceinline__ void eval(double r2, T ri, T rj, T si, T sj, T& e, T& dedr,
                                       T& ir) const {
    const T irr = rsqrt_r(T(r2));
    const T r = T(r2) * irr;
    ir = irr;
    if (form == TK_VDW_HAL) {
      const T ri2 = ri * ri, rj2 = rj * rj;
      const T rv = (ri2 * ri + rj2 * rj) / (ri2 + rj2);
      const T se = si + sj;
      const bool has = se > T(0);
      const T se2 = has ? se * se : T(1);
      const T rv2 = rv * rv, rv7 = rv2 * rv2 * rv2 * rv;
      const T r6 = T(r2) * T(r2) * T(r2), rik7 = r6 * r;
      const T d3 = rik7 + T(ghal) * rv7, d4 = r + T(dhal) * rv;
      const T ip = T(1) / (se2 * d3 * d4);
      const T invrho = se2 * d4 * ip, invtmp = se2 * d3 * ip;
      const T ep = has ? T(4) * (si * si) * (sj * sj) * (d3 * d4 * ip) : T(0);
      const T tb = T(1.0 + dhal) * rv * invtmp;
      const T tb2 = tb * tb, t7 = tb2 * tb2 * tb2 * tb;
      const T w = T(1.0 + ghal) * rv7 * invrho;
      e = ep * t7 * (w - T(2));
      dedr = ep * (T(-7) * t7 * invtmp * (w - T(2)) - T(7) * t7 * r6 * w * invrho);
    } else {
      const T sg = T(0.5) * (ri + rj);
      const T ep = si * sj;
      const T q = sg * sg * (irr * irr);
      const T sr6 = q * q * q;
      e = T(4) * ep * (sr6 * sr6 - sr6);
      dedr = T(4) * ep * (T(-12) * sr6 * sr6 + T(6) * sr6) * irr;
    }
    if ((double)r > ron) {
      const T x = (r - T(ron)) * T(tw_inv);
      const T x2 = x * x, x3 = x2 * x;
      const T S = T(1) - T(10) * x3 + T(15) * x3 * x - T(6) * x3 * x2;
      const T dS = (T(-30) * x2 + T(60) * x3 - T(30) * x3 * x) * T(tw_inv);
      dedr = dedr * S + e * dS;
      e *= S;
    }
  }
  __device__ void pair(const double* LH, const double* LK, int cap, int a, int b, double* AH,
                       double* AK, double* sc, long) const {
    if (LH[5 * cap + a] == LK[5 * cap + b]) return;
    double dd[3];
    const double r2 = image3(LH, LK, cap, a, b, box, inv_box, dd);
    if (!(r2 <= rc2)) return;
    // Both forms evaluate the pair once in FP64.  The vdW energy is a sum of
    // cancelling attractive and repulsive terms that needs FP64, and without
    // packed FP32 instructions FP32 arithmetic issues at the FP64 rate, so one
    // FP64 evaluation costs less than an FP32 force plus an FP64 energy.
    double e, dedr, ir;
    eval<double>(r2, LH[3 * cap + a], LK[3 * cap + b], LH[4 * cap + a], LK[4 * cap + b], e, dedr,
                 ir);
    const double en = e, f = dedr * ir;
    sc[0] += en;
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      const double de = f * dd[c];
      lds_add(&AH[c * cap + a], de);
      lds_add(&AK[c * cap + b], -de);
#pragma unroll
      for (int k = 0; k < 3; ++k) sc[1 + 3 * c + k] += dd[c] * f * dd[k];
    }
  }
};

// The 12-6 form.  It runs on the 12 A lists of the charge path, whose cells
// hold about twice the atoms of the 9 A cells of the HAL term, and there two
// waves per unit measured faster than four (269 against 297 us, 96,000
// atoms), where HAL on the water box wants four (54 against 62 us).
template <class R>
struct VdwLjPh : VdwPh<R> {
  static constexpr const char* kName = "vdw_lj";
  static constexpr int kWaves = 2;
};

// Forces of a combination of polarization pair energies (the gradient of a
// truncated solve): the induced-permanent term for dipoles a, plus the
// bilinear induced-induced terms for the pairs (b1, c1) and (b2, c2):
//   e = [U(a_i, M_j; gp) + U(M_i, a_j; gp)]
//     + sum_m [U(b_i, c_j; gm) + U(c_i, b_j; gm)],
// radial families as EpolarPh.  Forces -de/dx only.  FP64.
// Fields: x y z | q mu(3) Theta(6) | molid | isa | thole | a b1 c1 b2 c2 (3 each)
template <class R>
struct PolGradPh {
  static constexpr int NF = 31, NA = 3, NS = 0;
  static constexpr const char* kName = "polgrad";
  static constexpr int kWaves = 2;
  static constexpr const char* kTag = "_fp64";
  __device__ bool skip() const { return false; }
  __device__ void prologue(int tid, int nt) const { erfcx_stage<double>(tid, nt); }
  const double* xyz;
  const double* mpole;
  const int32_t* molid;
  const double* polarity;
  const double* thole;
  const double* vec[5];   // a, b1, c1, b2, c2: [n][3] each
  Geom g;
  __device__ void set_sys(const SysDev& d, int) {
    g.box = d.box;
    g.inv_box = d.inv_box;
  }
  static constexpr int NG = 31;
  const double* sorted = nullptr;
  long gstride = 0;
  __device__ void stage_dyn(double*, int, int, int) const {}
  __device__ void gather(int i, double* gg) const {
#pragma unroll
    for (int c = 0; c < 3; ++c) gg[c] = xyz[3 * i + c];
#pragma unroll
    for (int k = 0; k < 10; ++k) gg[3 + k] = mpole[10 * i + k];
    gg[13] = (double)molid[i];
    gg[14] = inv_sqrt_alpha(polarity[i]);
    gg[15] = thole[i];
#pragma unroll
    for (int v = 0; v < 5; ++v)
#pragma unroll
      for (int c = 0; c < 3; ++c) gg[16 + 3 * v + c] = vec[v][3 * i + c];
  }
  __device__ void pair(const double* LH, const double* LK, int cap, int a, int b, double* AH,
                       double* AK, double*, long) const {
    double dd[3];
    const double r2 = image3(LH, LK, cap, a, b, g.box, g.inv_box, dd);
    if (!(r2 <= g.rc2)) return;
    const bool excl = LH[13 * cap + a] == LK[13 * cap + b];
    const double rinv = rsqrt_r(r2), r = r2 * rinv;
    double B[5], Rb[5];
    radial<double, 4>(g, r, rinv, B, Rb, r2);
    double l[4];
    thole_damp9<double>(r, LH[14 * cap + a], LK[14 * cap + b], LH[15 * cap + a],
                        LK[15 * cap + b], l);
    double gp[5], gm[4];
#pragma unroll
    for (int n = 1; n <= 4; ++n) {
      const double bare = Rb[n] - l[n - 1] * Rb[n];
      gp[n] = excl ? B[n] - Rb[n] : B[n] - bare;
      if (n <= 3) gm[n] = B[n] - bare;
    }
    const double* d = dd;
    const auto dot = [](const double* x, const double* y) { return x[0] * y[0] + x[1] * y[1] + x[2] * y[2]; };
    const auto fld = [&](const double* L, int f, int s, double* v) {
      v[0] = L[f * cap + s];
      v[1] = L[(f + 1) * cap + s];
      v[2] = L[(f + 2) * cap + s];
    };
    double de[3] = {0.0, 0.0, 0.0};
    {  // induced-permanent term, dipoles a (as EpolarPh)
      const double qi = LH[3 * cap + a], qj = LK[3 * cap + b];
      double ui[3], uj[3], pi[3], pj[3];
      fld(LH, 4, a, ui);
      fld(LK, 4, b, uj);
      fld(LH, 16, a, pi);
      fld(LK, 16, b, pj);
      double ti[6], tj[6];
#pragma unroll
      for (int k = 0; k < 6; ++k) {
        ti[k] = LH[(7 + k) * cap + a];
        tj[k] = LK[(7 + k) * cap + b];
      }
      const auto tmul = [](const double* t, const double* x, double* y) {
        y[0] = t[0] * x[0] + t[1] * x[1] + t[2] * x[2];
        y[1] = t[1] * x[0] + t[3] * x[1] + t[4] * x[2];
        y[2] = t[2] * x[0] + t[4] * x[1] + t[5] * x[2];
      };
      double vi[3], vj[3], tipj[3], tjpi[3];
      tmul(ti, d, vi);
      tmul(tj, d, vj);
      tmul(ti, pj, tipj);
      tmul(tj, pi, tjpi);
      const double di = dot(ui, d), dj = dot(uj, d), Qi = dot(d, vi), Qj = dot(d, vj);
      const double ei = dot(pi, d), ej = dot(pj, d);
      const double c1 = qj * ei - qi * ej + dot(pi, uj) + dot(ui, pj);
      const double c2 = -(ei * dj + di * ej) + 2.0 * (dot(pj, vi) - dot(pi, vj));
      const double c3 = ei * Qj - ej * Qi;
      const double sp = c1 * gp[2] + c2 * gp[3] + c3 * gp[4];
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        const double dc1 = qj * pi[c] - qi * pj[c];
        const double dc2 = -(dj * pi[c] + ei * uj[c] + ej * ui[c] + di * pj[c]) + 2.0 * (tipj[c] - tjpi[c]);
        const double dc3 = Qj * pi[c] + 2.0 * ei * vj[c] - Qi * pj[c] - 2.0 * ej * vi[c];
        de[c] += dc1 * gp[1] + dc2 * gp[2] + dc3 * gp[3] - sp * d[c];
      }
    }
    // bilinear induced-induced terms: U(x_i, y_j) = x.y gm1 - (x.d)(y.d) gm2
    const auto bil = [&](const double* x, const double* y) {
      const double ex = dot(x, d), ey = dot(y, d), xy = dot(x, y);
      const double sm = xy * gm[2] - ex * ey * gm[3];
#pragma unroll
      for (int c = 0; c < 3; ++c) de[c] += -(ey * x[c] + ex * y[c]) * gm[2] - sm * d[c];
    };
#pragma unroll
    for (int m = 0; m < 2; ++m) {
      double bi[3], bj[3], ci[3], cj[3];
      fld(LH, 19 + 6 * m, a, bi);
      fld(LK, 19 + 6 * m, b, bj);
      fld(LH, 22 + 6 * m, a, ci);
      fld(LK, 22 + 6 * m, b, cj);
      bil(bi, cj);
      bil(ci, bj);
    }
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      lds_add(&AH[c * cap + a], kCoulomb * de[c]);
      lds_add(&AK[c * cap + b], -kCoulomb * de[c]);
    }
  }
};

// Derivatives of the permanent-multipole energy with respect to each site's
// own (lab-frame) multipoles, G_i,c = dE/dM_i,c (10 per site, stored layout:
// an off-diagonal quadrupole component counts both of its matrix entries).
// E is bilinear, so G_i is minus the potential/field/field-gradient that the
// other sites make at i, in the energy's own radial families (g_n = B_n, or
// B_n - R_n within a molecule).  FP64.  Fields as EmpolePh.
template <class R>
struct MderivPh {
  static constexpr int NF = 14, NA = 10, NS = 0;
  static constexpr const char* kName = "mderiv";
  static constexpr int kWaves = 2;
  static constexpr const char* kTag = "_fp64";
  __device__ bool skip() const { return false; }
  __device__ void prologue(int tid, int nt) const { erfcx_stage<double>(tid, nt); }
  const double* xyz;
  const double* mpole;
  const int32_t* molid;
  Geom g;
  __device__ void set_sys(const SysDev& d, int) {
    g.box = d.box;
    g.inv_box = d.inv_box;
  }
  static constexpr int NG = 14;
  const double* sorted = nullptr;
  long gstride = 0;
  __device__ void stage_dyn(double*, int, int, int) const {}
  __device__ void gather(int i, double* gg) const {
#pragma unroll
    for (int c = 0; c < 3; ++c) gg[c] = xyz[3 * i + c];
#pragma unroll
    for (int k = 0; k < 10; ++k) gg[3 + k] = mpole[10 * i + k];
    gg[13] = (double)molid[i];
  }
  __device__ void pair(const double* LH, const double* LK, int cap, int a, int b, double* AH,
                       double* AK, double*, long) const {
    double dd[3];
    const double r2 = image3(LH, LK, cap, a, b, g.box, g.inv_box, dd);
    if (!(r2 <= g.rc2)) return;
    const bool excl = LH[13 * cap + a] == LK[13 * cap + b];
    double B[5], Rb[5];
    radial_pair<double, 4>(g, r2, excl, B, Rb);
    double gn[5];
#pragma unroll
    for (int n = 0; n < 5; ++n) gn[n] = excl ? B[n] - Rb[n] : B[n];
    const double* d = dd;
    const double qi = LH[3 * cap + a], qj = LK[3 * cap + b];
    const double ui[3] = {LH[4 * cap + a], LH[5 * cap + a], LH[6 * cap + a]};
    const double uj[3] = {LK[4 * cap + b], LK[5 * cap + b], LK[6 * cap + b]};
    double ti[3][3], tj[3][3];
    {
      const double* h = LH + 7 * cap + a;
      const double* k = LK + 7 * cap + b;
      ti[0][0] = h[0]; ti[0][1] = ti[1][0] = h[cap]; ti[0][2] = ti[2][0] = h[2 * cap];
      ti[1][1] = h[3 * cap]; ti[1][2] = ti[2][1] = h[4 * cap]; ti[2][2] = h[5 * cap];
      tj[0][0] = k[0]; tj[0][1] = tj[1][0] = k[cap]; tj[0][2] = tj[2][0] = k[2 * cap];
      tj[1][1] = k[3 * cap]; tj[1][2] = tj[2][1] = k[4 * cap]; tj[2][2] = k[5 * cap];
    }
    double vi[3], vj[3];
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      vi[c] = ti[c][0] * d[0] + ti[c][1] * d[1] + ti[c][2] * d[2];
      vj[c] = tj[c][0] * d[0] + tj[c][1] * d[1] + tj[c][2] * d[2];
    }
    const double di = ui[0] * d[0] + ui[1] * d[1] + ui[2] * d[2];
    const double dj = uj[0] * d[0] + uj[1] * d[1] + uj[2] * d[2];
    const double Qi = d[0] * vi[0] + d[1] * vi[1] + d[2] * vi[2];
    const double Qj = d[0] * vj[0] + d[1] * vj[1] + d[2] * vj[2];
    double Gi[10], Gj[10];
    // d/dq, d/dmu (from c0..c3)
    Gi[0] = qj * gn[0] - dj * gn[1] + Qj * gn[2];
    Gj[0] = qi * gn[0] + di * gn[1] + Qi * gn[2];
    const double si = qj * gn[1] - dj * gn[2] + Qj * gn[3];
    const double sj = -qi * gn[1] - di * gn[2] - Qi * gn[3];
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      Gi[1 + c] = si * d[c] + gn[1] * uj[c] - 2.0 * gn[2] * vj[c];
      Gj[1 + c] = sj * d[c] + gn[1] * ui[c] + 2.0 * gn[2] * vi[c];
    }
    // d/dTheta_ab (c2, c3, c4), stored components: off-diagonal = ab + ba
    const double wi = qj * gn[2] - dj * gn[3] + Qj * gn[4];
    const double wj = qi * gn[2] + di * gn[3] + Qi * gn[4];
    const int ia[6] = {0, 0, 0, 1, 1, 2}, ib[6] = {0, 1, 2, 1, 2, 2};
#pragma unroll
    for (int k = 0; k < 6; ++k) {
      const int p = ia[k], q = ib[k];
      const auto ent_i = [&](int x, int y) {
        return wi * d[x] * d[y] + 2.0 * gn[2] * (uj[x] * d[y] + tj[x][y]) - 4.0 * gn[3] * vj[x] * d[y];
      };
      const auto ent_j = [&](int x, int y) {
        return wj * d[x] * d[y] + 2.0 * gn[2] * (-ui[x] * d[y] + ti[x][y]) - 4.0 * gn[3] * vi[x] * d[y];
      };
      Gi[4 + k] = p == q ? ent_i(p, p) : ent_i(p, q) + ent_i(q, p);
      Gj[4 + k] = p == q ? ent_j(p, p) : ent_j(p, q) + ent_j(q, p);
    }
#pragma unroll
    for (int c = 0; c < 10; ++c) {
      lds_add(&AH[c * cap + a], kCoulomb * Gi[c]);
      lds_add(&AK[c * cap + b], kCoulomb * Gj[c]);
    }
  }
};

// The same derivatives for the induced-permanent polarization energy at
// fixed induced dipoles p: each site sees the other's induced dipole as a
// pure dipole source, in the damped family gp_n = B_n - (1 - s l_(2n+1)) R_n
// of EpolarPh.  FP64.  Fields: x y z | molid | isa | thole | p(3)
template <class R>
struct MderivPolPh {
  static constexpr int NF = 9, NA = 10, NS = 0;
  static constexpr const char* kName = "mderiv_pol";
  static constexpr int kWaves = 2;
  static constexpr const char* kTag = "_fp64";
  __device__ bool skip() const { return false; }
  __device__ void prologue(int tid, int nt) const { erfcx_stage<double>(tid, nt); }
  const double* xyz;
  const double* mu;
  const int32_t* molid;
  const double* polarity;
  const double* thole;
  Geom g;
  __device__ void set_sys(const SysDev& d, int) {
    g.box = d.box;
    g.inv_box = d.inv_box;
  }
  static constexpr int NG = 9;
  const double* sorted = nullptr;
  long gstride = 0;
  __device__ void stage_dyn(double*, int, int, int) const {}
  __device__ void gather(int i, double* gg) const {
#pragma unroll
    for (int c = 0; c < 3; ++c) gg[c] = xyz[3 * i + c];
    gg[3] = (double)molid[i];
    gg[4] = inv_sqrt_alpha(polarity[i]);
    gg[5] = thole[i];
#pragma unroll
    for (int c = 0; c < 3; ++c) gg[6 + c] = mu[3 * i + c];
  }
  __device__ void pair(const double* LH, const double* LK, int cap, int a, int b, double* AH,
                       double* AK, double*, long) const {
    double dd[3];
    const double r2 = image3(LH, LK, cap, a, b, g.box, g.inv_box, dd);
    if (!(r2 <= g.rc2)) return;
    const bool excl = LH[3 * cap + a] == LK[3 * cap + b];
    const double rinv = rsqrt_r(r2), r = r2 * rinv;
    double B[4], Rb[4];
    radial<double, 3>(g, r, rinv, B, Rb, r2);
    double l3, l5, l7;
    thole_damp<double>(r, LH[4 * cap + a], LK[4 * cap + b], LH[5 * cap + a], LK[5 * cap + b], l3,
                       l5, l7);
    const double lf[4] = {0.0, l3, l5, l7};
    double gp[4];
#pragma unroll
    for (int n = 1; n <= 3; ++n) gp[n] = excl ? B[n] - Rb[n] : B[n] - (Rb[n] - lf[n] * Rb[n]);
    const double* d = dd;
    const double pi[3] = {LH[6 * cap + a], LH[7 * cap + a], LH[8 * cap + a]};
    const double pj[3] = {LK[6 * cap + b], LK[7 * cap + b], LK[8 * cap + b]};
    const double di = pi[0] * d[0] + pi[1] * d[1] + pi[2] * d[2];
    const double dj = pj[0] * d[0] + pj[1] * d[1] + pj[2] * d[2];
    double Gi[10], Gj[10];
    Gi[0] = -dj * gp[1];
    Gj[0] = di * gp[1];
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      Gi[1 + c] = -dj * gp[2] * d[c] + gp[1] * pj[c];
      Gj[1 + c] = -di * gp[2] * d[c] + gp[1] * pi[c];
    }
    const int ia[6] = {0, 0, 0, 1, 1, 2}, ib[6] = {0, 1, 2, 1, 2, 2};
#pragma unroll
    for (int k = 0; k < 6; ++k) {
      const int p = ia[k], q = ib[k];
      const auto ei = [&](int x, int y) { return -dj * gp[3] * d[x] * d[y] + 2.0 * gp[2] * pj[x] * d[y]; };
      const auto ej = [&](int x, int y) { return di * gp[3] * d[x] * d[y] - 2.0 * gp[2] * pi[x] * d[y]; };
      Gi[4 + k] = p == q ? ei(p, p) : ei(p, q) + ei(q, p);
      Gj[4 + k] = p == q ? ej(p, p) : ej(p, q) + ej(q, p);
    }
#pragma unroll
    for (int c = 0; c < 10; ++c) {
      lds_add(&AH[c * cap + a], kCoulomb * Gi[c]);
      lds_add(&AK[c * cap + b], kCoulomb * Gj[c]);
    }
  }
};

struct EpiStore10 {   // the sums are the site's dE/dM (10), caller order
  double* out;
  __device__ void operator()(int, int i, const double* a) const {
#pragma unroll
    for (int c = 0; c < 10; ++c) out[10 * i + c] = a[c];
  }
};

// Polarization forces at fixed induced dipoles p: the pair energies
//   e_ip = U(p_i, M_j; gp) + U(M_i, p_j; gp),   e_ii = U(p_i, p_j; gm)
// (U the multipole pair energy, an induced dipole the multipole (0, p, 0)),
// gp_n = B_n - (1 - s l_(2n+1)) R_n with s = 0 within a molecule,
// gm_n = B_n - (1 - l_(2n+1)) R_n; forces -de/dx, virial r_a de/dr_b.
// With one side a pure dipole only n = 1..3 carry coefficients.
// Fields: x y z | q mu(3) Theta(6) | molid | isa | thole | p(3)
template <class R>
struct EpolarPh {
  static constexpr int NF = 19, NA = 3, NS = 11;
  static constexpr const char* kName = "epolar";
  static constexpr int kWaves = 2;   // waves per unit (pairs.hpp launch_units)
  static constexpr const char* kTag = std::is_same<R, double>::value ? "_fp64" : "_fp32";
  __device__ bool skip() const { return false; }
  __device__ void prologue(int tid, int nt) const { erfcx_stage<R>(tid, nt); }
  const double* xyz;
  const double* mpole;
  const int32_t* molid;
  const double* polarity;
  const double* thole;
  const double* mu;
  Geom g;
  __device__ void set_sys(const SysDev& d, int) {
    g.box = d.box;
    g.inv_box = d.inv_box;
  }
  static constexpr int NG = 19;   // fields gathered once per call (sorted SoA)
  const double* sorted = nullptr;
  long gstride = 0;
  __device__ void stage_dyn(double*, int, int, int) const {}
  __device__ void gather(int i, double* g) const {
#pragma unroll
    for (int c = 0; c < 3; ++c) g[c] = xyz[3 * i + c];
#pragma unroll
    for (int k = 0; k < 10; ++k) g[3 + k] = mpole[10 * i + k];
    g[13] = (double)molid[i];
    g[14] = inv_sqrt_alpha(polarity[i]);
    g[15] = thole[i];
#pragma unroll
    for (int c = 0; c < 3; ++c) g[16 + c] = mu[3 * i + c];
  }
  // pair energies (e_ip, e_ii) and de/dr in arithmetic type T; with T = float
  // the caller routes same-molecule pairs to T = double
  template <class T>
  __device__ __forceinline__ void eval(const double* LH, const double* LK, int cap, int a, int b,
                                       const double* dd, double r2, bool excl, double* de,
                                       double& eip, double& eii) const {
    const T rinv = rsqrt_r(T(r2));
    const T r = T(r2) * rinv;
    T B[5], Rb[5];
    radial<T, 4>(g, r, rinv, B, Rb, r2);
    T l[4];
    thole_damp9<T>(r, T(LH[14 * cap + a]), T(LK[14 * cap + b]), T(LH[15 * cap + a]),
                   T(LK[15 * cap + b]), l);
    T gp[5], gm[4];   // indexed by n; entry 0 unused
#pragma unroll
    for (int n = 1; n <= 4; ++n) {
      const T bare = Rb[n] - l[n - 1] * Rb[n];   // (1 - l_(2n+1)) R_n
      gp[n] = excl ? B[n] - Rb[n] : B[n] - bare;
      if (n <= 3) gm[n] = B[n] - bare;
    }
    const T d[3] = {T(dd[0]), T(dd[1]), T(dd[2])};
    const T qi = T(LH[3 * cap + a]), qj = T(LK[3 * cap + b]);
    const T ui[3] = {T(LH[4 * cap + a]), T(LH[5 * cap + a]), T(LH[6 * cap + a])};
    const T uj[3] = {T(LK[4 * cap + b]), T(LK[5 * cap + b]), T(LK[6 * cap + b])};
    const T ti[6] = {T(LH[7 * cap + a]), T(LH[8 * cap + a]), T(LH[9 * cap + a]),
                     T(LH[10 * cap + a]), T(LH[11 * cap + a]), T(LH[12 * cap + a])};
    const T tj[6] = {T(LK[7 * cap + b]), T(LK[8 * cap + b]), T(LK[9 * cap + b]),
                     T(LK[10 * cap + b]), T(LK[11 * cap + b]), T(LK[12 * cap + b])};
    const T pi[3] = {T(LH[16 * cap + a]), T(LH[17 * cap + a]), T(LH[18 * cap + a])};
    const T pj[3] = {T(LK[16 * cap + b]), T(LK[17 * cap + b]), T(LK[18 * cap + b])};
    auto tmul = [](const T* t, const T* x, T* y) {
      y[0] = t[0] * x[0] + t[1] * x[1] + t[2] * x[2];
      y[1] = t[1] * x[0] + t[3] * x[1] + t[4] * x[2];
      y[2] = t[2] * x[0] + t[4] * x[1] + t[5] * x[2];
    };
    auto dot = [](const T* x, const T* y) { return x[0] * y[0] + x[1] * y[1] + x[2] * y[2]; };
    T vi[3], vj[3], tipj[3], tjpi[3];
    tmul(ti, d, vi);
    tmul(tj, d, vj);
    tmul(ti, pj, tipj);
    tmul(tj, pi, tjpi);
    const T di = dot(ui, d), dj = dot(uj, d), Qi = dot(d, vi), Qj = dot(d, vj);
    const T ei = dot(pi, d), ej = dot(pj, d), pp = dot(pi, pj);
    // induced-permanent coefficients (n = 1..3)
    const T c1 = qj * ei - qi * ej + dot(pi, uj) + dot(ui, pj);
    const T c2 = -(ei * dj + di * ej) + T(2) * (dot(pj, vi) - dot(pi, vj));
    const T c3 = ei * Qj - ej * Qi;
    const T sp = c1 * gp[2] + c2 * gp[3] + c3 * gp[4];
    const T sm = pp * gm[2] - ei * ej * gm[3];
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      const T dc1 = qj * pi[c] - qi * pj[c];
      const T dc2 = -(dj * pi[c] + ei * uj[c] + ej * ui[c] + di * pj[c]) +
                    T(2) * (tipj[c] - tjpi[c]);
      const T dc3 = Qj * pi[c] + T(2) * ei * vj[c] - Qi * pj[c] - T(2) * ej * vi[c];
      const T dm2 = -(ej * pi[c] + ei * pj[c]);
      de[c] = kCoulomb * (double)(dc1 * gp[1] + dc2 * gp[2] + dc3 * gp[3] + dm2 * gm[2] -
                                  (sp + sm) * d[c]);
    }
    eip = kCoulomb * (double)(c1 * gp[1] + c2 * gp[2] + c3 * gp[3]);
    eii = kCoulomb * (double)(pp * gm[1] - ei * ej * gm[2]);
  }
  __device__ void pair(const double* LH, const double* LK, int cap, int a, int b, double* AH,
                       double* AK, double* sc, long) const {
    double dd[3];
    const double r2 = image3(LH, LK, cap, a, b, g.box, g.inv_box, dd);
    if (!(r2 <= g.rc2)) return;
    const bool excl = LH[13 * cap + a] == LK[13 * cap + b];
    double de[3], eip, eii;
    if (std::is_same<R, float>::value && (excl || r2 < kMixedCloseR2))
      eval<double>(LH, LK, cap, a, b, dd, r2, excl, de, eip, eii);
    else
      eval<R>(LH, LK, cap, a, b, dd, r2, excl, de, eip, eii);
    sc[0] += eip;
    sc[1] += eii;
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      lds_add(&AH[c * cap + a], de[c]);
      lds_add(&AK[c * cap + b], -de[c]);
#pragma unroll
      for (int q = 0; q < 3; ++q) sc[2 + 3 * c + q] += dd[c] * de[q];
    }
  }
};

// Polarization forces with the two dipole sets (d: driven by the field
// without same-molecule pairs, p: by the field with them scaled by pscale) at
// fixed sets.  Each set meets the field that drives the other, and the
// induced pair term is the sets' bilinear form:
//   e_ip = 1/2 [U(d_i, M_j; gd) + U(M_i, d_j; gd)] + 1/2 [U(p_i, M_j; gq) + U(M_i, p_j; gq)]
//   e_ii = 1/2 [U(d_i, p_j; gm) + U(p_i, d_j; gm)]
// with gd = gq = B - (1 - l) R between molecules and, within one,
// gd = B - (1 - pscale l) R, gq = B - R.  The induced-permanent terms are
// one term of the mean set (d + p)/2, plus within a molecule d/2 in
// pscale l R.  FP64.
// Fields: x y z | q mu(3) Theta(6) | molid | isa | thole | d(3) | p(3)
struct Epolar2Ph {
  static constexpr int NF = 22, NA = 3, NS = 11;
  static constexpr const char* kName = "epolar2";
  static constexpr int kWaves = 2;   // waves per unit (pairs.hpp launch_units)
  static constexpr const char* kTag = "_fp64";
  __device__ bool skip() const { return false; }
  __device__ void prologue(int tid, int nt) const { erfcx_stage<double>(tid, nt); }
  const double* xyz;
  const double* mpole;
  const int32_t* molid;
  const double* polarity;
  const double* thole;
  const double* mu2;   // [2][n][3]: d, then p
  long n2 = 0;         // offset of the p block (3n)
  double pscale = 0.0;
  Geom g;
  __device__ void set_sys(const SysDev& d, int) {
    g.box = d.box;
    g.inv_box = d.inv_box;
  }
  static constexpr int NG = 22;   // fields gathered once per call (sorted SoA)
  const double* sorted = nullptr;
  long gstride = 0;
  __device__ void stage_dyn(double*, int, int, int) const {}
  __device__ void gather(int i, double* gg) const {
#pragma unroll
    for (int c = 0; c < 3; ++c) gg[c] = xyz[3 * i + c];
#pragma unroll
    for (int k = 0; k < 10; ++k) gg[3 + k] = mpole[10 * i + k];
    gg[13] = (double)molid[i];
    gg[14] = inv_sqrt_alpha(polarity[i]);
    gg[15] = thole[i];
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      gg[16 + c] = mu2[3 * i + c];
      gg[19 + c] = mu2[n2 + 3 * i + c];
    }
  }
  __device__ void pair(const double* LH, const double* LK, int cap, int a, int b, double* AH,
                       double* AK, double* sc, long) const {
    double dd[3];
    const double r2 = image3(LH, LK, cap, a, b, g.box, g.inv_box, dd);
    if (!(r2 <= g.rc2)) return;
    const bool excl = LH[13 * cap + a] == LK[13 * cap + b];
    const double rinv = rsqrt_r(r2), r = r2 * rinv;
    double B[5], Rb[5];
    radial<double, 4>(g, r, rinv, B, Rb, r2);
    double l[4];
    thole_damp9<double>(r, LH[14 * cap + a], LK[14 * cap + b], LH[15 * cap + a],
                        LK[15 * cap + b], l);
    const double* d = dd;
    const auto dot = [](const double* x, const double* y) {
      return x[0] * y[0] + x[1] * y[1] + x[2] * y[2];
    };
    const auto fld = [&](const double* L, int f, int s, double* v) {
      v[0] = L[f * cap + s];
      v[1] = L[(f + 1) * cap + s];
      v[2] = L[(f + 2) * cap + s];
    };
    const double qi = LH[3 * cap + a], qj = LK[3 * cap + b];
    double ui[3], uj[3], ti[6], tj[6];
    fld(LH, 4, a, ui);
    fld(LK, 4, b, uj);
#pragma unroll
    for (int k = 0; k < 6; ++k) {
      ti[k] = LH[(7 + k) * cap + a];
      tj[k] = LK[(7 + k) * cap + b];
    }
    const auto tmul = [](const double* t, const double* x, double* y) {
      y[0] = t[0] * x[0] + t[1] * x[1] + t[2] * x[2];
      y[1] = t[1] * x[0] + t[3] * x[1] + t[4] * x[2];
      y[2] = t[2] * x[0] + t[4] * x[1] + t[5] * x[2];
    };
    double vi[3], vj[3];
    tmul(ti, d, vi);
    tmul(tj, d, vj);
    const double di = dot(ui, d), dj = dot(uj, d), Qi = dot(d, vi), Qj = dot(d, vj);
    double de[3] = {0.0, 0.0, 0.0}, eip = 0.0, eii = 0.0;
    // induced-permanent term of dipoles (pi, pj) in the family gf[1..4]
    const auto ip = [&](const double* pi, const double* pj, const double* gf) {
      double tipj[3], tjpi[3];
      tmul(ti, pj, tipj);
      tmul(tj, pi, tjpi);
      const double ei = dot(pi, d), ej = dot(pj, d);
      const double c1 = qj * ei - qi * ej + dot(pi, uj) + dot(ui, pj);
      const double c2 = -(ei * dj + di * ej) + 2.0 * (dot(pj, vi) - dot(pi, vj));
      const double c3 = ei * Qj - ej * Qi;
      const double sp = c1 * gf[2] + c2 * gf[3] + c3 * gf[4];
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        const double dc1 = qj * pi[c] - qi * pj[c];
        const double dc2 =
            -(dj * pi[c] + ei * uj[c] + ej * ui[c] + di * pj[c]) + 2.0 * (tipj[c] - tjpi[c]);
        const double dc3 = Qj * pi[c] + 2.0 * ei * vj[c] - Qi * pj[c] - 2.0 * ej * vi[c];
        de[c] += dc1 * gf[1] + dc2 * gf[2] + dc3 * gf[3] - sp * d[c];
      }
      eip += c1 * gf[1] + c2 * gf[2] + c3 * gf[3];
    };
    double xdi[3], xdj[3], xpi[3], xpj[3];
    fld(LH, 16, a, xdi);
    fld(LK, 16, b, xdj);
    fld(LH, 19, a, xpi);
    fld(LK, 19, b, xpj);
    // induced-induced: 1/2 [U(d_i, p_j) + U(p_i, d_j)], U(x_i, y_j) = x.y gm1 - (x.d)(y.d) gm2
    double gm[4];
#pragma unroll
    for (int n = 1; n <= 3; ++n) gm[n] = B[n] - (Rb[n] - l[n - 1] * Rb[n]);
    const auto bil = [&](const double* x, const double* y) {
      const double ex = dot(x, d), ey = dot(y, d), xy = dot(x, y);
      const double sm = xy * gm[2] - ex * ey * gm[3];
#pragma unroll
      for (int c = 0; c < 3; ++c) de[c] += 0.5 * (-(ey * x[c] + ex * y[c]) * gm[2] - sm * d[c]);
      eii += 0.5 * (xy * gm[1] - ex * ey * gm[2]);
    };
    bil(xdi, xpj);
    bil(xpi, xdj);
    // pass 0: the mean set (d + p)/2 in gp (between molecules) or B - R
    // (within one); pass 1, within a molecule: d/2 in pscale l R, which
    // makes d's family B - (1 - pscale l) R
    const int passes = excl && pscale != 0.0 ? 2 : 1;
#pragma unroll 1
    for (int k = 0; k < passes; ++k) {
      double gf[5], mi[3], mj[3];
#pragma unroll
      for (int n = 1; n <= 4; ++n)
        gf[n] = k == 1 ? pscale * l[n - 1] * Rb[n]
                       : excl ? B[n] - Rb[n] : B[n] - (Rb[n] - l[n - 1] * Rb[n]);
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        mi[c] = 0.5 * (k == 1 ? xdi[c] : xdi[c] + xpi[c]);
        mj[c] = 0.5 * (k == 1 ? xdj[c] : xdj[c] + xpj[c]);
      }
      ip(mi, mj, gf);
    }
    sc[0] += kCoulomb * eip;
    sc[1] += kCoulomb * eii;
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      const double f = kCoulomb * de[c];
      lds_add(&AH[c * cap + a], f);
      lds_add(&AK[c * cap + b], -f);
#pragma unroll
      for (int q = 0; q < 3; ++q) sc[2 + 3 * c + q] += dd[c] * (kCoulomb * de[q]);
    }
  }
};

// Epilogues of the per-atom reduction.
struct EpiForce {   // the sums are the atom's force; caller order
  double* force;
  __device__ void operator()(int, int i, const double* a) const {
    force[3 * i] = a[0];
    force[3 * i + 1] = a[1];
    force[3 * i + 2] = a[2];
  }
};

struct EpiPermField {   // permanent field + Ewald self field c * mu_perm
  double* out;
  const double* mpole;
  double cself;
  int sorted_out;
  __device__ void operator()(int s, int i, const double* a) const {
    const int o = sorted_out ? s : i;
#pragma unroll
    for (int c = 0; c < 3; ++c) out[3 * o + c] = a[c] + cself * mpole[10 * i + 1 + c];
  }
};

struct EpiForceField {   // force (caller order) and permanent field + self field (sorted order)
  double* force;
  double* field;
  const double* mpole;
  double cself;
  __device__ void operator()(int s, int i, const double* a) const {
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      force[3 * i + c] = a[c];
      field[3 * s + c] = a[3 + c] + cself * mpole[10 * i + 1 + c];
    }
  }
};

struct EpiMutual {   // mutual field (T + cI) mu, or A mu = mu/alpha - field
  double* out;
  const double* mu;
  const double* alpha;
  double cself;
  int include_diag;
  __device__ void operator()(int, int i, const double* a) const {
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      const double m = mu[3 * i + c];
      double f = a[c] + cself * m;
      if (include_diag) {
        const double al = alpha[i];
        f = al > 0.0 ? m / al - f : 0.0;
      }
      out[3 * i + c] = f;
    }
  }
};

// Launch one pair term over a plan: units -> per-atom reduce (Epi) ->
// per-system energies and virial (terms with unit scalars; energy and virial
// are device arrays of [nsys][NS - 9] and [nsys][9]).
template <class Ph>
inline size_t term_ws_doubles(const Plan& P) {
  return (size_t)pad64(P.n) * (kMaxSlots * Ph::NA + Ph::NG);
}

template <class Ph, class Epi>
tk_status run_term(tk_ctx* ctx, hipStream_t st, const Plan& P, const Ph& ph, const Epi& epi,
                   double* energy, double* virial, const TermWs* ws = nullptr,
                   DeferredSums* defer = nullptr) {
  const long pstride = pad64(P.n);
  void *partial, *uscal;
  tk_status s;
  const size_t ns1 = Ph::NS > 0 ? Ph::NS : 1;
  const bool sums = Ph::NS > 0 && energy && virial;
  if (ws && (!ws->partial || !ws->gathered || (sums && (!ws->uscal || !ws->cpart))))
    return TK_E_ARG;
  if (ws) {
    partial = ws->partial;
    uscal = ws->uscal;
  } else if ((s = scratch(ctx, per_stream("partial", st).c_str(),
                          sizeof(double) * kMaxSlots * Ph::NA * pstride, &partial)) ||
             (s = scratch(ctx, per_stream("uscal", st).c_str(),
                          sizeof(double) * (size_t)P.nunits * ns1, &uscal)))
    return s;
  PlanView pv = P.view();
  if (unit_lds_bytes<Ph>(P, 1) > kMaxLds) return TK_E_CAPACITY;
  void* gathered;
  if (ws)
    gathered = ws->gathered;
  else if ((s = scratch(ctx, per_stream("gathered", st).c_str(),
                        sizeof(double) * Ph::NG * pstride, &gathered)))
    return s;
  Ph phg = ph;
  phg.sorted = (const double*)gathered;
  phg.gstride = pstride;
  k_gather<Ph><<<ceil_div(P.n, 256), 256, 0, st>>>(pv, phg, (double*)gathered, pstride);
  {
    // no timing events on the caller-supplied-buffer path (creating one may allocate)
    ProfScope ps(ctx, st, ws ? std::string() : std::string("units_") + Ph::kName + Ph::kTag);
    launch_units(P, phg, (double*)partial, pstride, (double*)uscal, st);
  }
  const int nchunk = sums ? total_chunks(P) : 0;
  void* cpart = ws ? ws->cpart : nullptr;
  if (!ws && sums &&
      (s = scratch(ctx, per_stream("chunk_sums", st).c_str(),
                   sizeof(double) * ns1 * (size_t)(nchunk > 0 ? nchunk : 1), &cpart)))
    return s;
  {
    ProfScope ps(ctx, st, ws ? std::string() : std::string("reduce_atoms"));
    const int nb = std::max(ceil_div((long)P.n * kRedLanes, 256), nchunk);
    k_reduce<Ph::NA, Ph::NS, Epi><<<nb, 256, 0, st>>>(pv, (double*)partial, pstride, epi,
                                                      sums ? (const double*)uscal : nullptr,
                                                      (double*)cpart);
  }
  if constexpr (Ph::NS > 0) {
    if (sums && defer && Ph::NS == 11)   // the caller's next kernel finishes the sums
      *defer = DeferredSums{(const double*)cpart, energy, virial, P.nsys};
    else if (sums)
      k_sum_finish<Ph::NS><<<P.nsys, 64, 0, st>>>((const double*)cpart, pv.sys, energy, virial);
  }
  TK_HIP(hipGetLastError());
  return TK_OK;
}

template <class R>
inline tk_status launch_efield(tk_ctx* ctx, hipStream_t st, const Plan& P, const tk_system* sys,
                        const double* mpole, const double* polarity, const double* thole,
                        double beta, double cutoff, double* out, int sorted_out,
                        R* gc = nullptr, long gcs = 0, double intra = 0.0) {
  EfieldPh<R> ph;
  ph.gc = gc;
  ph.gcs = gcs;
  ph.intra = intra;
  ph.xyz = sys->xyz;
  ph.mpole = mpole;
  ph.molid = sys->molid;
  ph.polarity = polarity;
  ph.thole = thole;
  ph.g.set(sys->box, cutoff, beta);
  EpiPermField e2{out, mpole, ph.g.cself, sorted_out};
  return run_term(ctx, st, P, ph, e2, nullptr, nullptr);
}

// Multipole energy {total, non-excluded, exclusion correction}, forces and
// virial (device, caller order) and the permanent field (sorted order) in one
// pass; the solver's factors into gc.
template <class R>
inline tk_status launch_mpole_field(tk_ctx* ctx, hipStream_t st, const Plan& P,
                                    const tk_system* sys, const double* mpole,
                                    const double* polarity, const double* thole, double beta,
                                    double cutoff, double* energy, double* force, double* virial,
                                    double* field_sorted, R* gc, long gcs,
                                    DeferredSums* defer = nullptr) {
  MpoleFieldPh<R> ph;
  ph.gc = gc;
  ph.gcs = gcs;
  ph.xyz = sys->xyz;
  ph.mpole = mpole;
  ph.molid = sys->molid;
  ph.polarity = polarity;
  ph.thole = thole;
  ph.g.set(sys->box, cutoff, beta);
  EpiForceField epi{force, field_sorted, mpole, ph.g.cself};
  return run_term(ctx, st, P, ph, epi, energy, virial, nullptr, defer);
}

}  // namespace tk
