// Local-frame multipoles: rotation to the lab frame, and the permanent-
// multipole forces with the frame (torque) part (the rotation and torque
// steps that section "Hotspots" lists beside the multipole routines).
//
// Frames (d_z = r_zatom - r_i, d_x = r_xatom - r_i, minimum image):
//   0 none:      R = I
//   1 Z-then-X:  z = unit(d_z), x = unit(d_x - (d_x.z) z)
//   2 bisector:  z = unit(unit(d_z) + unit(d_x)), x = unit(u - (u.z) z), u = unit(d_x)
// y = z x x, R = [x y z] (columns); mu = R mu_loc, Theta = R Theta_loc R^T.
//
// Forces: the direct pair forces at the lab-frame multipoles (the multipole
// pair kernel), plus the frame part.  With G = dE/dM per site (the
// multipole-derivative pair kernel), dE/dR = G_mu mu_loc^T + W R Theta_loc,
// W the stored-component quadrupole derivative as a symmetric matrix with its
// diagonal doubled; this is carried back through the frame construction by
// hand (unit vectors, the Gram-Schmidt step, the cross product) to d_z and
// d_x, whose atoms receive the forces.  The frame forces of a site go to
// three atoms and are added with FP64 atomics: at most a few per atom, so the
// sum is reproducible to rounding but not bitwise.
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

// The frame of site i and the intermediates its reverse pass needs.
struct Frame {
  V3 x, y, z;
  V3 dz, dx;      // frame vectors
  V3 uz, ux;      // unit(d_z), unit(d_x) (bisector)
  V3 a;           // the vector orthogonalised against z (d_x, or ux)
  double nz, nx, ns, nw;   // |d_z|, |d_x|, |uz + ux|, |a - (a.z) z|
};

__device__ __forceinline__ bool frame_ok(int type, int i, int iz, int ix, int n) {
  if (type == 0) return true;
  if (type != 1 && type != 2) return false;
  return iz >= 0 && iz < n && ix >= 0 && ix < n && iz != i && ix != i && iz != ix;
}

__device__ __forceinline__ Frame make_frame(const double* xyz, double box, double inv_box, int type,
                                            int i, int iz, int ix) {
  Frame f;
  f.dz = image(xyz, i, iz, box, inv_box);
  f.dx = image(xyz, i, ix, box, inv_box);
  f.nz = sqrt(dot(f.dz, f.dz));
  f.nx = sqrt(dot(f.dx, f.dx));
  f.uz = (1.0 / f.nz) * f.dz;
  f.ux = (1.0 / f.nx) * f.dx;
  if (type == 1) {
    f.z = f.uz;
    f.a = f.dx;
    f.ns = 0.0;
  } else {
    const V3 s = f.uz + f.ux;
    f.ns = sqrt(dot(s, s));
    f.z = (1.0 / f.ns) * s;
    f.a = f.ux;
  }
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
  const int type = ftype[i], iz = fatoms[2 * i], ix = fatoms[2 * i + 1];
  const double* l = loc + 10 * i;
  double* o = glob + 10 * i;
  if (!frame_ok(type, i, iz, ix, n)) {
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
  const Frame f = make_frame(xyz, box, 1.0 / box, type, i, iz, ix);
  const V3 col[3] = {f.x, f.y, f.z};
  rotate(col, l, o);
}

// Reverse pass through unit(v): gradient of a unit vector u = v/|v| given
// the gradient g with respect to u.
__device__ __forceinline__ V3 back_unit(V3 g, V3 u, double nrm) {
  return (1.0 / nrm) * (g - dot(g, u) * u);
}

// Frame forces of site i: dE/dM = G (10) -> dE/dR -> dE/d(d_z, d_x).
__global__ __launch_bounds__(256) void k_frames_torque(int n, const double* __restrict__ xyz,
                                                       double box, const int32_t* __restrict__ ftype,
                                                       const int32_t* __restrict__ fatoms,
                                                       const double* __restrict__ loc,
                                                       const double* __restrict__ G,
                                                       double* __restrict__ force,
                                                       const int* __restrict__ flag,
                                                       double* __restrict__ energy) {
  // G: dE/dM per site (10)
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i == 0 && flag[0]) {   // a frame was refused: no number is returned as if it were right
#pragma unroll
    for (int k = 0; k < 3; ++k) energy[k] = __builtin_nan("");
  }
  if (i >= n) return;
  const int type = ftype[i], iz = fatoms[2 * i], ix = fatoms[2 * i + 1];
  if (type == 0 || !frame_ok(type, i, iz, ix, n)) return;
  const Frame f = make_frame(xyz, box, 1.0 / box, type, i, iz, ix);
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
  V3 gdz, gdx;
  if (type == 1) {   // z = unit(d_z), a = d_x
    gdz = back_unit(gz, f.z, f.nz);
    gdx = ga;
  } else {           // z = unit(uz + ux), a = ux
    const V3 gs = back_unit(gz, f.z, f.ns);
    gdz = back_unit(gs, f.uz, f.nz);
    gdx = back_unit(gs + ga, f.ux, f.nx);
  }
  // d_z = r_z - r_i, d_x = r_x - r_i; F = -dE/dr
  const double gzv[3] = {gdz.x, gdz.y, gdz.z}, gxv[3] = {gdx.x, gdx.y, gdx.z};
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    atomicAdd(&force[3 * iz + c], -gzv[c]);
    atomicAdd(&force[3 * ix + c], -gxv[c]);
    atomicAdd(&force[3 * i + c], gzv[c] + gxv[c]);
  }
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
                           double* mpole_global) {
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
    return TK_OK;
  }
  if (!frame_type || !frame_atoms || !mpole_local || !force) return TK_E_ARG;
  void *mg, *G, *vir, *flag;
  if ((s = scratch(ctx, per_stream("frames_G", st).c_str(), sizeof(double) * 10 * (size_t)n, &G)) ||
      (s = scratch(ctx, per_stream("frames_vir", st).c_str(), sizeof(double) * 9, &vir)) ||
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
  if ((s = run_term(ctx, st, *P, ph, EpiForce{force}, energy, (double*)vir))) return s;
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
                                                      force, (const int*)flag, energy);
  }
  TK_HIP(hipGetLastError());
  return TK_OK;
}

tk_status tk_epolar_frames(tk_ctx* ctx, void* stream, const tk_system* sys,
                           const tk_nblist* list, const int32_t* frame_type,
                           const int32_t* frame_atoms, const double* mpole_local,
                           const double* polarity, const double* thole, const double* mu,
                           double ewald_beta, double cutoff, double* energy, double* force) {
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
    return TK_OK;
  }
  if (!frame_type || !frame_atoms || !mpole_local || !polarity || !thole || !mu || !force)
    return TK_E_ARG;
  void *mg, *G, *vir, *flag;
  if ((s = scratch(ctx, per_stream("frames_G", st).c_str(), sizeof(double) * 10 * (size_t)n, &G)) ||
      (s = scratch(ctx, per_stream("frames_vir", st).c_str(), sizeof(double) * 9, &vir)) ||
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
  if ((s = run_term(ctx, st, *P, ph, EpiForce{force}, energy, (double*)vir))) return s;
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
                                                      force, (const int*)flag, energy);
  }
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
