// Local-frame multipoles: rotation to the lab frame, and the permanent-
// multipole forces with the frame (torque) part (the rotation and torque
// steps that section "Hotspots" lists beside the multipole routines).
//
// Frames: the five AMOEBA types (none, Z-then-X, bisector, Z-only,
// Z-bisector, 3-fold) of up to three frame atoms; see make_frame.
// y = z x x, R = [x y z] (columns); mu = R mu_loc, Theta = R Theta_loc R^T.
//
// Forces: the direct pair forces at the lab-frame multipoles (the multipole
// pair kernel), plus the frame part.  With G = dE/dM per site (the
// multipole-derivative pair kernel), dE/dR = G_mu mu_loc^T + W R Theta_loc,
// W the stored-component quadrupole derivative as a symmetric matrix with its
// diagonal doubled; this is carried back through the frame construction by
// hand (unit vectors, the Gram-Schmidt step, the cross product) to d_z, d_x
// and d_y, whose atoms receive the forces.  The frame forces of a site go to
// up to four atoms and are added with FP64 atomics: at most a few per atom,
// so the sum is reproducible to rounding but not bitwise.
#include <cmath>

#include "pairs.hpp"
#include "terms.hpp"

namespace tk {

namespace {

struct V3 {
  double x, y, z;
};
__device__ __forceinline__ V3 v3(double a, double b, double c) { return V3{a, b, c}; }
__device__ __forceinline__ V3 operator+(V3 a, V3 b) { return v3(a.x + b.x, a.y + b.y, a.z + b.z); }
__device__ __forceinline__ V3 operator-(V3 a, V3 b) { return v3(a.x - b.x, a.y - b.y, a.z - b.z); }
__device__ __forceinline__ V3 operator*(double s, V3 a) { return v3(s * a.x, s * a.y, s * a.z); }
__device__ __forceinline__ double dot(V3 a, V3 b) { return a.x * b.x + a.y * b.y + a.z * b.z; }
__device__ __forceinline__ V3 cross(V3 a, V3 b) {
  return v3(a.y * b.z - a.z * b.y, a.z * b.x - a.x * b.z, a.x * b.y - a.y * b.x);
}

__device__ __forceinline__ V3 image(const double* xyz, int i, int j, double box, double inv_box) {
  double t[3];
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    const double s = xyz[3 * j + c] - xyz[3 * i + c];
    t[c] = s - box * rint(s * inv_box);
  }
  return v3(t[0], t[1], t[2]);
}

// The frame of site i and the intermediates its reverse pass needs.  Every
// type takes z and a vector a, then x = unit(a - (a.z) z), y = z x x:
//   1 Z-then-X:   z = u_z,                   a = d_x
//   2 bisector:   z = unit(u_z + u_x),       a = u_x
//   3 Z-only:     z = u_z,                   a = global x, or global y when |z_x| > 0.866
//   4 Z-bisector: z = u_z,                   a = u_x + u_y
//   5 3-fold:     z = unit(u_z + u_x + u_y), a = u_x
// with d_k = r_katom - r_i (minimum image) and u_k = d_k / |d_k|.
struct Frame {
  V3 x, y, z;
  V3 dz, dx, dy;    // the frame vectors d_k (zero where a type takes none)
  V3 uz, ux, uy;    // unit vectors to the frame atoms
  V3 a;             // the vector orthogonalised against z
  double nz, nx, ny, ns, nw;   // |d_z|, |d_x|, |d_y|, |sum| (types 2, 5), |a - (a.z) z|
};

// frame atoms a type takes: z (1-5), x (1, 2, 4, 5), y (4, 5)
__device__ __forceinline__ int frame_natoms(int type) {
  return type == 0 ? 0 : type == 3 ? 1 : type <= 2 ? 2 : 3;
}

// fa: the site's three frame atoms (z, x, y); those a type takes are in
// [0, n), not the site, and distinct
__device__ __forceinline__ bool frame_ok(int type, int i, const int32_t* fa, int n) {
  if (type < 0 || type > 5) return false;
  const int m = frame_natoms(type);
  for (int k = 0; k < m; ++k) {
    const int a = fa[k];
    if (a < 0 || a >= n || a == i) return false;
    for (int l = 0; l < k; ++l)
      if (fa[l] == a) return false;
  }
  return true;
}

__device__ __forceinline__ Frame make_frame(const double* xyz, double box, double inv_box, int type,
                                            int i, const int32_t* fa) {
  Frame f;
  f.dz = image(xyz, i, fa[0], box, inv_box);
  f.nz = sqrt(dot(f.dz, f.dz));
  f.uz = (1.0 / f.nz) * f.dz;
  f.dx = f.dy = v3(0.0, 0.0, 0.0);
  f.ux = f.uy = f.dx;
  f.nx = f.ny = 1.0;
  if (type != 3) {
    f.dx = image(xyz, i, fa[1], box, inv_box);
    f.nx = sqrt(dot(f.dx, f.dx));
    f.ux = (1.0 / f.nx) * f.dx;
  }
  if (type >= 4) {
    f.dy = image(xyz, i, fa[2], box, inv_box);
    f.ny = sqrt(dot(f.dy, f.dy));
    f.uy = (1.0 / f.ny) * f.dy;
  }
  f.ns = 0.0;
  if (type == 2 || type == 5) {
    const V3 s = type == 2 ? f.uz + f.ux : f.uz + f.ux + f.uy;
    f.ns = sqrt(dot(s, s));
    f.z = (1.0 / f.ns) * s;
  } else {
    f.z = f.uz;
  }
  if (type == 1) f.a = f.dx;
  else if (type == 3) f.a = fabs(f.z.x) > 0.866 ? v3(0.0, 1.0, 0.0) : v3(1.0, 0.0, 0.0);
  else if (type == 4) f.a = f.ux + f.uy;
  else f.a = f.ux;
  const V3 w = f.a - dot(f.a, f.z) * f.z;
  f.nw = sqrt(dot(w, w));
  f.x = (1.0 / f.nw) * w;
  f.y = cross(f.z, f.x);
  return f;
}

// M = rotate(R, loc), stored layout
__device__ __forceinline__ void rotate(const V3 col[3], const double* loc, double* out) {
  const double R[3][3] = {{col[0].x, col[1].x, col[2].x},
                          {col[0].y, col[1].y, col[2].y},
                          {col[0].z, col[1].z, col[2].z}};
  const double tl[3][3] = {{loc[4], loc[5], loc[6]}, {loc[5], loc[7], loc[8]},
                           {loc[6], loc[8], loc[9]}};
  out[0] = loc[0];
#pragma unroll
  for (int a = 0; a < 3; ++a) out[1 + a] = R[a][0] * loc[1] + R[a][1] * loc[2] + R[a][2] * loc[3];
  double RT[3][3];   // R Theta_loc
#pragma unroll
  for (int a = 0; a < 3; ++a)
#pragma unroll
    for (int d = 0; d < 3; ++d) RT[a][d] = R[a][0] * tl[0][d] + R[a][1] * tl[1][d] + R[a][2] * tl[2][d];
  const int ia[6] = {0, 0, 0, 1, 1, 2}, ib[6] = {0, 1, 2, 1, 2, 2};
#pragma unroll
  for (int k = 0; k < 6; ++k)
    out[4 + k] = RT[ia[k]][0] * R[ib[k]][0] + RT[ia[k]][1] * R[ib[k]][1] + RT[ia[k]][2] * R[ib[k]][2];
}

__global__ __launch_bounds__(256) void k_frames_rotate(int n, const double* __restrict__ xyz,
                                                       double box, const int32_t* __restrict__ ftype,
                                                       const int32_t* __restrict__ fatoms,
                                                       const double* __restrict__ loc,
                                                       double* __restrict__ glob,
                                                       int* __restrict__ flag) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const int type = ftype[i];
  const int32_t fa[3] = {fatoms[3 * i], fatoms[3 * i + 1], fatoms[3 * i + 2]};
  const double* l = loc + 10 * i;
  double* o = glob + 10 * i;
  if (!frame_ok(type, i, fa, n)) {
    atomicOr(flag, 1);
#pragma unroll
    for (int k = 0; k < 10; ++k) o[k] = l[k];
    return;
  }
  if (type == 0) {
#pragma unroll
    for (int k = 0; k < 10; ++k) o[k] = l[k];
    return;
  }
  const Frame f = make_frame(xyz, box, 1.0 / box, type, i, fa);
  const V3 col[3] = {f.x, f.y, f.z};
  rotate(col, l, o);
}

// Reverse pass through unit(v): gradient of a unit vector u = v/|v| given
// the gradient g with respect to u.
__device__ __forceinline__ V3 back_unit(V3 g, V3 u, double nrm) {
  return (1.0 / nrm) * (g - dot(g, u) * u);
}

// Frame forces of site i: dE/dM = G (10) -> dE/dR -> dE/d(d_z, d_x, d_y).
// vpart (nullable): per-workgroup partials of the frame virial
// sum_k d_k (x) dE/dd_k (M depends on positions only through the frame
// vectors), summed in a fixed order: waves, then the workgroup's waves.
__global__ __launch_bounds__(256) void k_frames_torque(int n, const double* __restrict__ xyz,
                                                       double box, const int32_t* __restrict__ ftype,
                                                       const int32_t* __restrict__ fatoms,
                                                       const double* __restrict__ loc,
                                                       const double* __restrict__ G,
                                                       double* __restrict__ force,
                                                       const int* __restrict__ flag,
                                                       double* __restrict__ energy,
                                                       double* __restrict__ vpart) {
  // G: dE/dM per site (10)
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i == 0 && flag[0]) {   // a frame was refused: no number is returned as if it were right
#pragma unroll
    for (int k = 0; k < 3; ++k) energy[k] = __builtin_nan("");
  }
  double wv[9];
#pragma unroll
  for (int k = 0; k < 9; ++k) wv[k] = 0.0;
  const int type = i < n ? ftype[i] : 0;
  int32_t fa[3] = {-1, -1, -1};
  if (i < n) {
    fa[0] = fatoms[3 * i];
    fa[1] = fatoms[3 * i + 1];
    fa[2] = fatoms[3 * i + 2];
  }
  if (type != 0 && frame_ok(type, i, fa, n)) {
    const Frame f = make_frame(xyz, box, 1.0 / box, type, i, fa);
    const double* l = loc + 10 * i;
    const double* g = G + 10 * i;
    const double R[3][3] = {{f.x.x, f.y.x, f.z.x}, {f.x.y, f.y.y, f.z.y}, {f.x.z, f.y.z, f.z.z}};
    const double tl[3][3] = {{l[4], l[5], l[6]}, {l[5], l[7], l[8]}, {l[6], l[8], l[9]}};
    // W: stored-component derivative as a symmetric matrix, diagonal doubled
    const double W[3][3] = {{2.0 * g[4], g[5], g[6]}, {g[5], 2.0 * g[7], g[8]}, {g[6], g[8], 2.0 * g[9]}};
    double RT[3][3];
  #pragma unroll
    for (int a = 0; a < 3; ++a)
  #pragma unroll
      for (int d = 0; d < 3; ++d) RT[a][d] = R[a][0] * tl[0][d] + R[a][1] * tl[1][d] + R[a][2] * tl[2][d];
    double dR[3][3];   // dE/dR_cd = G_mu,c mu_loc,d + (W R Theta_loc)_cd
  #pragma unroll
    for (int c = 0; c < 3; ++c)
  #pragma unroll
      for (int d = 0; d < 3; ++d)
        dR[c][d] = g[1 + c] * l[1 + d] + W[c][0] * RT[0][d] + W[c][1] * RT[1][d] + W[c][2] * RT[2][d];
    V3 gx = v3(dR[0][0], dR[1][0], dR[2][0]);
    V3 gy = v3(dR[0][1], dR[1][1], dR[2][1]);
    V3 gz = v3(dR[0][2], dR[1][2], dR[2][2]);
    // y = z x x
    gz = gz + cross(f.x, gy);
    gx = gx + cross(gy, f.z);
    // x = unit(w), w = a - (a.z) z
    const V3 gw = back_unit(gx, f.x, f.nw);
    const double az = dot(f.a, f.z), gwz = dot(gw, f.z);
    const V3 ga = gw - gwz * f.z;
    gz = gz - az * gw - gwz * f.a;
    // back through z and a to d_z, d_x, d_y
    const V3 zero = v3(0.0, 0.0, 0.0);
    V3 gdz, gdx = zero, gdy = zero;
    if (type == 2 || type == 5) {   // z = unit(s), s = u_z + u_x (+ u_y)
      const V3 gs = back_unit(gz, f.z, f.ns);
      gdz = back_unit(gs, f.uz, f.nz);
      gdx = back_unit(gs + ga, f.ux, f.nx);   // a = u_x
      if (type == 5) gdy = back_unit(gs, f.uy, f.ny);
    } else {                        // z = u_z
      gdz = back_unit(gz, f.uz, f.nz);
      if (type == 1) gdx = ga;      // a = d_x
      if (type == 4) {              // a = u_x + u_y
        gdx = back_unit(ga, f.ux, f.nx);
        gdy = back_unit(ga, f.uy, f.ny);
      }                             // type 3: a is fixed
    }
    // d_k = r_k - r_i; F = -dE/dr
    const int m = frame_natoms(type);
    const double gzv[3] = {gdz.x, gdz.y, gdz.z}, gxv[3] = {gdx.x, gdx.y, gdx.z},
                 gyv[3] = {gdy.x, gdy.y, gdy.z};
  #pragma unroll
    for (int c = 0; c < 3; ++c) {
      atomicAdd(&force[3 * fa[0] + c], -gzv[c]);
      if (m >= 2) atomicAdd(&force[3 * fa[1] + c], -gxv[c]);
      if (m >= 3) atomicAdd(&force[3 * fa[2] + c], -gyv[c]);
      atomicAdd(&force[3 * i + c], gzv[c] + gxv[c] + gyv[c]);
    }
    const double dzv[3] = {f.dz.x, f.dz.y, f.dz.z}, dxv[3] = {f.dx.x, f.dx.y, f.dx.z},
                 dyv[3] = {f.dy.x, f.dy.y, f.dy.z};
  #pragma unroll
    for (int a = 0; a < 3; ++a)
  #pragma unroll
      for (int b = 0; b < 3; ++b)
        wv[3 * a + b] = dzv[a] * gzv[b] + dxv[a] * gxv[b] + dyv[a] * gyv[b];
  }
  if (!vpart) return;   // uniform over the launch
  __shared__ double red[4][9];
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
#pragma unroll
  for (int k = 0; k < 9; ++k) {
    for (int o = 32; o > 0; o >>= 1) wv[k] += __shfl_xor(wv[k], o);
    if (lane == 0) red[wid][k] = wv[k];
  }
  __syncthreads();
  if (threadIdx.x < 9) {
    double t = 0.0;
    for (int ww = 0; ww < (int)(blockDim.x >> 6); ++ww) t += red[ww][threadIdx.x];
    vpart[9 * blockIdx.x + threadIdx.x] = t;
  }
}

// virial[k] += the frame partials of nb workgroups, in order; NaN when a
// frame was refused
__global__ void k_frames_virial(int nb, const double* __restrict__ vpart,
                                const int* __restrict__ flag, double* __restrict__ virial) {
  const int k = threadIdx.x;
  if (k >= 9) return;
  double t = 0.0;
  for (int b = 0; b < nb; ++b) t += vpart[9 * b + k];
  virial[k] = flag[0] ? __builtin_nan("") : virial[k] + t;
}

// vdW hydrogen reduction: site i at r_p + red_i (r_i - r_p) (minimum image)
// for a parent p, else at r_i; an invalid parent gives a NaN site.
__global__ __launch_bounds__(256) void k_vdw_sites(int n, const double* __restrict__ xyz, double box,
                                                   const int32_t* __restrict__ parent,
                                                   const double* __restrict__ red,
                                                   double* __restrict__ sites) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const int p = parent[i];
  if (p < 0) {
#pragma unroll
    for (int a = 0; a < 3; ++a) sites[3 * i + a] = xyz[3 * i + a];
    return;
  }
  if (p >= n || p == i) {
#pragma unroll
    for (int a = 0; a < 3; ++a) sites[3 * i + a] = __builtin_nan("");
    return;
  }
  const double inv = 1.0 / box, r = red[i];
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    const double d = xyz[3 * i + a] - xyz[3 * p + a];
    sites[3 * i + a] = xyz[3 * p + a] + r * (d - box * rint(d * inv));
  }
}

// Site forces to atoms: atom i takes red_i f_i (all of f_i without a
// parent), then each parent adds (1 - red_i) f_i with an atomic add.
__global__ __launch_bounds__(256) void k_vdw_own(int n, const int32_t* __restrict__ parent,
                                                 const double* __restrict__ red,
                                                 const double* __restrict__ fsite,
                                                 double* __restrict__ fatom) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const int p = parent[i];
  const double r = (p >= 0 && p < n && p != i) ? red[i] : 1.0;
#pragma unroll
  for (int a = 0; a < 3; ++a) fatom[3 * i + a] = r * fsite[3 * i + a];
}

__global__ __launch_bounds__(256) void k_vdw_parent(int n, const int32_t* __restrict__ parent,
                                                    const double* __restrict__ red,
                                                    const double* __restrict__ fsite,
                                                    double* __restrict__ fatom) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const int p = parent[i];
  if (p < 0 || p >= n || p == i) return;
  const double w = 1.0 - red[i];
#pragma unroll
  for (int a = 0; a < 3; ++a) atomicAdd(&fatom[3 * p + a], w * fsite[3 * i + a]);
}

}  // namespace

}  // namespace tk

using namespace tk;

extern "C" {

tk_status tk_rotate_mpole(tk_ctx* ctx, void* stream, const tk_system* sys,
                          const int32_t* frame_type, const int32_t* frame_atoms,
                          const double* mpole_local, double* mpole_global) {
  if (!ctx) return TK_E_ARG;
  tk_status s = check_system(sys);
  if (s) return s;
  if (sys->n == 0) return TK_OK;
  if (!frame_type || !frame_atoms || !mpole_local || !mpole_global) return TK_E_ARG;
  hipStream_t st = (hipStream_t)stream;
  void* flag;   // the kernel's refusal flag (read only by tk_empole_frames, which clears it)
  if ((s = scratch(ctx, per_stream("frames_flag", st).c_str(), 64, &flag))) return s;
  k_frames_rotate<<<ceil_div(sys->n, 256), 256, 0, st>>>(sys->n, sys->xyz, sys->box, frame_type,
                                                         frame_atoms, mpole_local, mpole_global,
                                                         (int*)flag);
  TK_HIP(hipGetLastError());
  return TK_OK;
}

tk_status tk_empole_frames(tk_ctx* ctx, void* stream, const tk_system* sys,
                           const tk_nblist* list, const int32_t* frame_type,
                           const int32_t* frame_atoms, const double* mpole_local,
                           double ewald_beta, double cutoff, double* energy, double* force,
                           double* virial, double* mpole_global) {
  if (!ctx) return TK_E_ARG;
  tk_status s = check_system(sys);
  if (s) return s;
  const Plan* P;
  if ((s = get_plan(ctx, sys, list, cutoff, &P))) return s;
  if (!(ewald_beta >= 0.0) || !std::isfinite(ewald_beta) || !energy) return TK_E_ARG;
  hipStream_t st = (hipStream_t)stream;
  const int n = sys->n;
  if (n == 0) {
    TK_HIP(hipMemsetAsync(energy, 0, 3 * sizeof(double), st));
    if (virial) TK_HIP(hipMemsetAsync(virial, 0, 9 * sizeof(double), st));
    return TK_OK;
  }
  if (!frame_type || !frame_atoms || !mpole_local || !force) return TK_E_ARG;
  void *mg, *G, *vir, *flag;
  if ((s = scratch(ctx, per_stream("frames_G", st).c_str(), sizeof(double) * 10 * (size_t)n, &G)) ||
      (s = scratch(ctx, per_stream("frames_vir", st).c_str(),
                   sizeof(double) * 9 * (1 + (size_t)ceil_div(n, 256)), &vir)) ||
      (s = scratch(ctx, per_stream("frames_flag", st).c_str(), 64, &flag)))
    return s;
  if (mpole_global) {
    mg = mpole_global;
  } else if ((s = scratch(ctx, per_stream("frames_M", st).c_str(), sizeof(double) * 10 * (size_t)n,
                          &mg))) {
    return s;
  }
  TK_HIP(hipMemsetAsync(flag, 0, sizeof(int), st));
  k_frames_rotate<<<ceil_div(n, 256), 256, 0, st>>>(n, sys->xyz, sys->box, frame_type, frame_atoms,
                                                    mpole_local, (double*)mg, (int*)flag);
  // direct forces and the energies at the lab-frame multipoles
  EmpolePh<double> ph;
  ph.xyz = sys->xyz;
  ph.mpole = (const double*)mg;
  ph.molid = sys->molid;
  ph.g.set(sys->box, cutoff, ewald_beta);
  // the pair virial goes to the caller's array (or scratch); the frame
  // partials follow it in the scratch
  double* wpair = virial ? virial : (double*)vir;
  double* wpart = virial ? (double*)vir + 9 : nullptr;
  if ((s = run_term(ctx, st, *P, ph, EpiForce{force}, energy, wpair))) return s;
  // dE/dM per site, then the frame forces
  MderivPh<double> pd;
  pd.xyz = sys->xyz;
  pd.mpole = (const double*)mg;
  pd.molid = sys->molid;
  pd.g.set(sys->box, cutoff, ewald_beta);
  if ((s = run_term(ctx, st, *P, pd, EpiStore10{(double*)G}, nullptr, nullptr))) return s;
  {
    ProfScope ps(ctx, st, "frames_torque");
    k_frames_torque<<<ceil_div(n, 256), 256, 0, st>>>(n, sys->xyz, sys->box, frame_type,
                                                      frame_atoms, mpole_local, (const double*)G,
                                                      force, (const int*)flag, energy, wpart);
  }
  if (virial)
    k_frames_virial<<<1, 64, 0, st>>>(ceil_div(n, 256), wpart, (const int*)flag, virial);
  TK_HIP(hipGetLastError());
  return TK_OK;
}

tk_status tk_epolar_frames(tk_ctx* ctx, void* stream, const tk_system* sys,
                           const tk_nblist* list, const int32_t* frame_type,
                           const int32_t* frame_atoms, const double* mpole_local,
                           const double* polarity, const double* thole, const double* mu,
                           double ewald_beta, double cutoff, double* energy, double* force,
                           double* virial) {
  if (!ctx) return TK_E_ARG;
  tk_status s = check_system(sys);
  if (s) return s;
  const Plan* P;
  if ((s = get_plan(ctx, sys, list, cutoff, &P))) return s;
  if (!(ewald_beta >= 0.0) || !std::isfinite(ewald_beta) || !energy) return TK_E_ARG;
  hipStream_t st = (hipStream_t)stream;
  const int n = sys->n;
  if (n == 0) {
    TK_HIP(hipMemsetAsync(energy, 0, 3 * sizeof(double), st));
    if (virial) TK_HIP(hipMemsetAsync(virial, 0, 9 * sizeof(double), st));
    return TK_OK;
  }
  if (!frame_type || !frame_atoms || !mpole_local || !polarity || !thole || !mu || !force)
    return TK_E_ARG;
  void *mg, *G, *vir, *flag;
  if ((s = scratch(ctx, per_stream("frames_G", st).c_str(), sizeof(double) * 10 * (size_t)n, &G)) ||
      (s = scratch(ctx, per_stream("frames_vir", st).c_str(),
                   sizeof(double) * 9 * (1 + (size_t)ceil_div(n, 256)), &vir)) ||
      (s = scratch(ctx, per_stream("frames_flag", st).c_str(), 64, &flag)) ||
      (s = scratch(ctx, per_stream("frames_M", st).c_str(), sizeof(double) * 10 * (size_t)n, &mg)))
    return s;
  TK_HIP(hipMemsetAsync(flag, 0, sizeof(int), st));
  k_frames_rotate<<<ceil_div(n, 256), 256, 0, st>>>(n, sys->xyz, sys->box, frame_type, frame_atoms,
                                                    mpole_local, (double*)mg, (int*)flag);
  // direct forces and the pair energies at the lab-frame multipoles
  EpolarPh<double> ph;
  ph.xyz = sys->xyz;
  ph.mpole = (const double*)mg;
  ph.molid = sys->molid;
  ph.polarity = polarity;
  ph.thole = thole;
  ph.mu = mu;
  ph.g.set(sys->box, cutoff, ewald_beta);
  // the pair virial goes to the caller's array (or scratch); the frame
  // partials follow it in the scratch
  double* wpair = virial ? virial : (double*)vir;
  double* wpart = virial ? (double*)vir + 9 : nullptr;
  if ((s = run_term(ctx, st, *P, ph, EpiForce{force}, energy, wpair))) return s;
  // dE/dM of the induced-permanent energy, then the frame forces
  MderivPolPh<double> pd;
  pd.xyz = sys->xyz;
  pd.mu = mu;
  pd.molid = sys->molid;
  pd.polarity = polarity;
  pd.thole = thole;
  pd.g.set(sys->box, cutoff, ewald_beta);
  if ((s = run_term(ctx, st, *P, pd, EpiStore10{(double*)G}, nullptr, nullptr))) return s;
  {
    ProfScope ps(ctx, st, "frames_torque");
    k_frames_torque<<<ceil_div(n, 256), 256, 0, st>>>(n, sys->xyz, sys->box, frame_type,
                                                      frame_atoms, mpole_local, (const double*)G,
                                                      force, (const int*)flag, energy, wpart);
  }
  if (virial)
    k_frames_virial<<<1, 64, 0, st>>>(ceil_div(n, 256), wpart, (const int*)flag, virial);
  TK_HIP(hipGetLastError());
  return TK_OK;
}

tk_status tk_vdw_sites(tk_ctx* ctx, void* stream, const tk_system* sys, const int32_t* parent,
                       const double* red, double* sites) {
  if (!ctx) return TK_E_ARG;
  tk_status s = check_system(sys);
  if (s) return s;
  if (sys->n == 0) return TK_OK;
  if (!parent || !red || !sites) return TK_E_ARG;
  k_vdw_sites<<<ceil_div(sys->n, 256), 256, 0, (hipStream_t)stream>>>(sys->n, sys->xyz, sys->box,
                                                                     parent, red, sites);
  TK_HIP(hipGetLastError());
  return TK_OK;
}

tk_status tk_vdw_site_forces(tk_ctx* ctx, void* stream, int32_t n, const int32_t* parent,
                             const double* red, const double* site_force, double* atom_force) {
  if (!ctx || n < 0) return TK_E_ARG;
  if (n == 0) return TK_OK;
  if (!parent || !red || !site_force || !atom_force || site_force == atom_force) return TK_E_ARG;
  hipStream_t st = (hipStream_t)stream;
  k_vdw_own<<<ceil_div(n, 256), 256, 0, st>>>(n, parent, red, site_force, atom_force);
  k_vdw_parent<<<ceil_div(n, 256), 256, 0, st>>>(n, parent, red, site_force, atom_force);
  TK_HIP(hipGetLastError());
  return TK_OK;
}

}  // extern "C"
