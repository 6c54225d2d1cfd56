/*
 * tk_oracle.c -- serial FP64 reference implementation of the real-space AMOEBA
 * pair terms (multipoles, Thole-damped dipole field, induced-dipole PCG,
 * Halgren 14-7 and Lennard-Jones van der Waals, Ewald point charges).
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the oracle that the GPU library is
 * checked against.  It shares no code, header, table or constant with the GPU
 * library; only the test suite, the smoke check and the CPU leg of the
 * benchmark may load it.  Every quantity is the plain definition evaluated
 * pair by pair, in FP64, with no blocking, fusion or reordering; the one
 * iteration (the conjugate-gradient solve) follows its algorithm step by step.
 *
 * Paper: "Raising the Performance of the Tinker-HP Molecular Modeling
 * Package" (arXiv 1906.01211).  The paper names the terms but never writes
 * their formulas: section "Polarizable AMOEBA force field" names permanent
 * multipoles through quadrupoles, Thole-damped induced point dipoles and the
 * Halgren buffered 14-7 vdW; section "Hotspots" (Table of the Rel profile)
 * names the routines this file mirrors: the polarization mat-vec, the
 * permanent-field right-hand side, the multipole energy, the 14-7 energy, the
 * LJ 12-6 and charge-charge energies, and the cell-list neighbour builders.
 * The only formula-level content is the 14-7 compute loop (Listing
 * "calculation", section "Typical compute loop") and the neighbour selection
 * mask (Listing "creationmask", section "Typical selection loop").  All other
 * formulas are the textbook Ewald / multipole / Thole definitions, written out
 * here; the readings taken where the paper is silent are listed in the
 * design notes of the repository and restated at each function below.
 *
 * Conventions: r = r_j - r_i for a pair (i, j); forces are F = -dE/dx;
 * units are Angstrom, elementary charge, kcal/mol.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define OR_OK 0
#define OR_E_ARG (-1)
#define OR_E_CUTOFF (-2)
#define OR_E_CAPACITY (-3)
#define OR_E_NOCONV (-4)
#define OR_E_BREAKDOWN (-5)

/* Reading: Coulomb constant e^2/(4 pi eps0) in kcal*A/(mol*e^2), and the
 * e*A -> Debye factor.  The paper states neither. */
static const double OR_COULOMB = 332.0637;
static const double OR_DEBYE = 4.80320;
static const double OR_SQRTPI = 1.7724538509055160273;

double or_coulomb_constant(void) { return OR_COULOMB; }
double or_debye_factor(void) { return OR_DEBYE; }

/* ------------------------------------------------------------------------ */
/* Geometry: minimum image in FP64.  The pair vector is d = x_j - x_i with
 * d := d - L*rint(d/L) written as one fused multiply-add, and
 * r^2 = fma(dx,dx, fma(dy,dy, dz*dz)).  (The paper's "image" routine wraps
 * pair vectors; section "Hotspots".) */
static void or_image(const double* xi, const double* xj, double box, double d[3],
                     double* r2) {
  for (int a = 0; a < 3; ++a) {
    double t = xj[a] - xi[a];
    d[a] = fma(-box, rint(t / box), t);
  }
  *r2 = fma(d[0], d[0], fma(d[1], d[1], d[2] * d[2]));
}

/* ------------------------------------------------------------------------ */
/* Neighbour list (the cell-list builders of the Rel profile table; the
 * selection of neighbours by cutoff, section "General Structure").
 * Reading: the list is integer and exact.  Each coordinate is mapped to a
 * 32-bit fraction of the box, u = floor(frac(x/L) * 2^32); the minimum-image
 * difference is the wrapped 32-bit difference; a pair is listed iff
 * dx^2+dy^2+dz^2 <= rq^2 in exact 64-bit integer arithmetic, with
 * rq = floor((rc/L) * 2^32).  Rows hold j > i in ascending order (CSR). */
int or_quantize(int n, const double* xyz, double box, uint32_t* u) {
  if (n < 0 || !(box > 0.0) || !isfinite(box)) return OR_E_ARG;
  for (int i = 0; i < 3 * n; ++i) {
    double x = xyz[i];
    if (!isfinite(x)) return OR_E_ARG;
    double t = x / box;
    double f = t - floor(t);
    if (f >= 1.0) f = 0.0; /* t slightly below an integer can round f up to 1 */
    u[i] = (uint32_t)(f * 4294967296.0);
  }
  return OR_OK;
}

uint32_t or_cutoff_quantum(double rc, double box) {
  return (uint32_t)floor((rc / box) * 4294967296.0);
}

static int or_pair_in(const uint32_t* u, int i, int j, uint64_t rq2) {
  uint64_t d2 = 0;
  for (int a = 0; a < 3; ++a) {
    int64_t d = (int32_t)(u[3 * j + a] - u[3 * i + a]);
    d2 += (uint64_t)(d * d);
  }
  return d2 <= rq2;
}

static int or_list_args(int n, double box, double rc) {
  if (n < 0 || !(box > 0.0) || !(rc > 0.0) || !isfinite(rc)) return OR_E_ARG;
  if (rc > 0.5 * box) return OR_E_CUTOFF;
  return OR_OK;
}

/* O(N^2) definition: every unordered pair is tested once. */
int or_nblist_brute(int n, const double* xyz, double box, double rc, int32_t* row_ptr,
                    int32_t* col, int64_t cap, int64_t* npairs) {
  int st = or_list_args(n, box, rc);
  if (st) return st;
  uint32_t* u = (uint32_t*)malloc(sizeof(uint32_t) * 3 * (size_t)(n > 0 ? n : 1));
  st = or_quantize(n, xyz, box, u);
  if (st) { free(u); return st; }
  uint64_t rq = or_cutoff_quantum(rc, box);
  uint64_t rq2 = rq * rq;
  int64_t np = 0;
  for (int i = 0; i < n; ++i) {
    row_ptr[i] = (int32_t)(np < cap ? np : cap);
    for (int j = i + 1; j < n; ++j) {
      if (or_pair_in(u, i, j, rq2)) {
        if (np < cap) col[np] = j;
        ++np;
      }
    }
  }
  row_ptr[n] = (int32_t)(np < cap ? np : cap);
  *npairs = np;
  free(u);
  return np > cap ? OR_E_CAPACITY : OR_OK;
}

static int or_cmp_int(const void* a, const void* b) {
  int x = *(const int*)a, y = *(const int*)b;
  return (x > y) - (x < y);
}

/* Cell list: ncell = floor(L/rc) cells per dimension (each at least rc wide
 * in the 32-bit fixed point), the unique cells among the 27 around the cell
 * of i are scanned, and each row is sorted ascending. */
int or_nblist_cell(int n, const double* xyz, double box, double rc, int32_t* row_ptr,
                   int32_t* col, int64_t cap, int64_t* npairs) {
  int st = or_list_args(n, box, rc);
  if (st) return st;
  size_t nn = (size_t)(n > 0 ? n : 1);
  uint32_t* u = (uint32_t*)malloc(sizeof(uint32_t) * 3 * nn);
  st = or_quantize(n, xyz, box, u);
  if (st) { free(u); return st; }
  uint64_t rq = or_cutoff_quantum(rc, box);
  uint64_t rq2 = rq * rq;
  int nc = (int)floor(box / rc);
  if (nc < 1) nc = 1;
  int ncell = nc * nc * nc;
  int* cell = (int*)malloc(sizeof(int) * nn);
  int* cstart = (int*)calloc((size_t)ncell + 1, sizeof(int));
  int* cfill = (int*)calloc((size_t)ncell, sizeof(int));
  int* catom = (int*)malloc(sizeof(int) * nn);
  for (int i = 0; i < n; ++i) {
    int c[3];
    for (int a = 0; a < 3; ++a) c[a] = (int)(((uint64_t)u[3 * i + a] * (uint64_t)nc) >> 32);
    cell[i] = (c[0] * nc + c[1]) * nc + c[2];
    cstart[cell[i] + 1]++;
  }
  for (int c = 0; c < ncell; ++c) cstart[c + 1] += cstart[c];
  for (int i = 0; i < n; ++i) catom[cstart[cell[i]] + cfill[cell[i]]++] = i;
  int* buf = (int*)malloc(sizeof(int) * nn);
  int64_t np = 0;
  for (int i = 0; i < n; ++i) {
    int ci[3] = {cell[i] / (nc * nc), (cell[i] / nc) % nc, cell[i] % nc};
    int nb[3][3], cnt[3];
    for (int a = 0; a < 3; ++a) { /* unique neighbour cells per dimension */
      cnt[a] = 0;
      for (int o = -1; o <= 1; ++o) {
        int v = ((ci[a] + o) % nc + nc) % nc, dup = 0;
        for (int k = 0; k < cnt[a]; ++k) dup |= (nb[a][k] == v);
        if (!dup) nb[a][cnt[a]++] = v;
      }
    }
    int m = 0;
    for (int x = 0; x < cnt[0]; ++x)
      for (int y = 0; y < cnt[1]; ++y)
        for (int z = 0; z < cnt[2]; ++z) {
          int c = (nb[0][x] * nc + nb[1][y]) * nc + nb[2][z];
          for (int k = cstart[c]; k < cstart[c + 1]; ++k) {
            int j = catom[k];
            if (j > i && or_pair_in(u, i, j, rq2)) buf[m++] = j;
          }
        }
    qsort(buf, (size_t)m, sizeof(int), or_cmp_int);
    row_ptr[i] = (int32_t)(np < cap ? np : cap);
    for (int k = 0; k < m; ++k) {
      if (np < cap) col[np] = buf[k];
      ++np;
    }
  }
  row_ptr[n] = (int32_t)(np < cap ? np : cap);
  *npairs = np;
  free(u); free(cell); free(cstart); free(cfill); free(catom); free(buf);
  return np > cap ? OR_E_CAPACITY : OR_OK;
}

/* ------------------------------------------------------------------------ */
/* Radial kernel families.  Ewald-screened:
 *   B0 = erfc(beta r)/r,
 *   Bn = [(2n-1) B(n-1) + (2 beta^2)^n exp(-beta^2 r^2)/(beta sqrt(pi))] / r^2;
 * bare Coulomb Rn = (2n-1)!!/r^(2n+1) (= Bn at beta = 0).  Both families obey
 * f(n+1) = -(1/r) d f(n)/dr, so the gradient of f(n) along r is -r f(n+1). */
void or_radial(double r, double beta, int nmax, double* B, double* R) {
  double r2 = r * r;
  R[0] = 1.0 / r;
  for (int k = 1; k <= nmax; ++k) R[k] = (2 * k - 1) * R[k - 1] / r2;
  if (beta == 0.0) {
    for (int k = 0; k <= nmax; ++k) B[k] = R[k];
    return;
  }
  double ex = exp(-beta * beta * r2) / (beta * OR_SQRTPI);
  double b2 = 2.0 * beta * beta, pw = 1.0;
  B[0] = erfc(beta * r) / r;
  for (int k = 1; k <= nmax; ++k) {
    pw *= b2;
    B[k] = ((2 * k - 1) * B[k - 1] + pw * ex) / r2;
  }
}

/* Thole damping, exponential AMOEBA form.  Reading: pair parameter
 * a_ij = min(a_i, a_j); x = a_ij * r^3 / sqrt(alpha_i alpha_j);
 * l3 = 1 - e^-x, l5 = 1 - (1+x) e^-x, l7 = 1 - (1 + x + 0.6 x^2) e^-x;
 * all three are 1 when alpha_i alpha_j = 0. */
void or_thole(double r, double ai, double aj, double ti, double tj, double* l3,
              double* l5, double* l7) {
  double prod = ai * aj;
  if (prod == 0.0) { *l3 = *l5 = *l7 = 1.0; return; }
  double a = ti < tj ? ti : tj;
  double x = a * r * r * r / sqrt(prod);
  double e = exp(-x);
  *l3 = 1.0 - e;
  *l5 = 1.0 - (1.0 + x) * e;
  *l7 = 1.0 - (1.0 + x + 0.6 * x * x) * e;
}

/* ------------------------------------------------------------------------ */
/* Multipole pair energy and its gradient with respect to r = r_j - r_i.
 * Site k carries (q, mu, Theta) with Theta symmetric and traceless; its
 * potential at y is [q - mu.grad + Theta:grad grad] f0(|y - r_k|).  With
 * d = mu.r, v = Theta r, Q = r.Theta.r the interaction is C * sum_n c_n g_n:
 *   c0 = qi qj
 *   c1 = qj di - qi dj + mui.muj
 *   c2 = qi Qj + qj Qi - di dj + 2 (muj.vi - mui.vj + Thi:Thj)
 *   c3 = di Qj - dj Qi - 4 vi.vj
 *   c4 = Qi Qj
 * and de/dr = C * sum_n [ (dc_n/dr) g_n - c_n r g(n+1) ].
 * mpole layout per site: q, mux, muy, muz, Txx, Txy, Txz, Tyy, Tyz, Tzz. */
static void or_unpack(const double* m, double* q, double mu[3], double th[3][3]) {
  *q = m[0];
  mu[0] = m[1]; mu[1] = m[2]; mu[2] = m[3];
  th[0][0] = m[4]; th[0][1] = th[1][0] = m[5]; th[0][2] = th[2][0] = m[6];
  th[1][1] = m[7]; th[1][2] = th[2][1] = m[8]; th[2][2] = m[9];
}

static double or_dot(const double a[3], const double b[3]) {
  return a[0] * b[0] + a[1] * b[1] + a[2] * b[2];
}

static void or_matvec3(double th[3][3], const double x[3], double y[3]) {
  for (int a = 0; a < 3; ++a) y[a] = th[a][0] * x[0] + th[a][1] * x[1] + th[a][2] * x[2];
}

void or_mpole_pair(const double r[3], const double* mi, const double* mj, const double* g,
                   double* e, double de[3]) {
  double qi, qj, ui[3], uj[3], ti[3][3], tj[3][3];
  or_unpack(mi, &qi, ui, ti);
  or_unpack(mj, &qj, uj, tj);
  double di = or_dot(ui, r), dj = or_dot(uj, r);
  double vi[3], vj[3];
  or_matvec3(ti, r, vi);
  or_matvec3(tj, r, vj);
  double Qi = or_dot(r, vi), Qj = or_dot(r, vj);
  double tt = 0.0;
  for (int a = 0; a < 3; ++a)
    for (int b = 0; b < 3; ++b) tt += ti[a][b] * tj[a][b];
  double c[5];
  c[0] = qi * qj;
  c[1] = qj * di - qi * dj + or_dot(ui, uj);
  c[2] = qi * Qj + qj * Qi - di * dj + 2.0 * (or_dot(uj, vi) - or_dot(ui, vj) + tt);
  c[3] = di * Qj - dj * Qi - 4.0 * or_dot(vi, vj);
  c[4] = Qi * Qj;
  double tivj[3], tjvi[3], tiuj[3], tjui[3];
  or_matvec3(ti, vj, tivj);
  or_matvec3(tj, vi, tjvi);
  or_matvec3(ti, uj, tiuj);
  or_matvec3(tj, ui, tjui);
  double dc[5][3];
  for (int a = 0; a < 3; ++a) {
    dc[0][a] = 0.0;
    dc[1][a] = qj * ui[a] - qi * uj[a];
    dc[2][a] = 2.0 * qi * vj[a] + 2.0 * qj * vi[a] - dj * ui[a] - di * uj[a] +
               2.0 * (tiuj[a] - tjui[a]);
    dc[3][a] = Qj * ui[a] + 2.0 * di * vj[a] - Qi * uj[a] - 2.0 * dj * vi[a] -
               4.0 * (tivj[a] + tjvi[a]);
    dc[4][a] = 2.0 * Qj * vi[a] + 2.0 * Qi * vj[a];
  }
  double en = 0.0;
  double gr[3] = {0.0, 0.0, 0.0};
  for (int k = 0; k <= 4; ++k) {
    en += c[k] * g[k];
    for (int a = 0; a < 3; ++a) gr[a] += dc[k][a] * g[k] - c[k] * r[a] * g[k + 1];
  }
  *e = OR_COULOMB * en;
  for (int a = 0; a < 3; ++a) de[a] = OR_COULOMB * gr[a];
}

static int or_pair_args(int n, double box, double rc) {
  if (n < 0 || !(box > 0.0) || !(rc > 0.0)) return OR_E_ARG;
  if (rc > 0.5 * box) return OR_E_CUTOFF;
  return OR_OK;
}

/* Real-space Ewald permanent-multipole energy, forces and virial over the
 * listed pairs with r <= rc (section "Hotspots": the multipolar permanent
 * electrostatic energy and forces).  Reading: pairs with equal molid are
 * excluded from the direct interaction; for them g_n = B_n - R_n (the Ewald
 * correction that removes the screened part carried by reciprocal space);
 * for all other pairs g_n = B_n.  energy[0] = total, energy[1] = sum over
 * non-excluded pairs, energy[2] = sum of the exclusion corrections.
 * Virial W_ab = sum over pairs of r_a * de/dr_b. */
int or_empole_real(int n, const double* xyz, double box, const int32_t* molid,
                   const int32_t* row_ptr, const int32_t* col, const double* mpole,
                   double beta, double rc, double* energy, double* force, double* virial) {
  int st = or_pair_args(n, box, rc);
  if (st) return st;
  double rc2 = rc * rc;
  energy[0] = energy[1] = energy[2] = 0.0;
  for (int k = 0; k < 9; ++k) virial[k] = 0.0;
  for (int k = 0; k < 3 * n; ++k) force[k] = 0.0;
  for (int i = 0; i < n; ++i) {
    for (int p = row_ptr[i]; p < row_ptr[i + 1]; ++p) {
      int j = col[p];
      double d[3], r2;
      or_image(xyz + 3 * i, xyz + 3 * j, box, d, &r2);
      if (!(r2 <= rc2)) continue;
      double r = sqrt(r2), B[6], R[6], g[6];
      or_radial(r, beta, 5, B, R);
      int excl = molid[i] == molid[j];
      for (int k = 0; k <= 5; ++k) g[k] = excl ? B[k] - R[k] : B[k];
      double e, de[3];
      or_mpole_pair(d, mpole + 10 * i, mpole + 10 * j, g, &e, de);
      energy[excl ? 2 : 1] += e;
      for (int a = 0; a < 3; ++a) {
        force[3 * i + a] += de[a];
        force[3 * j + a] -= de[a];
        for (int b = 0; b < 3; ++b) virial[3 * a + b] += d[a] * de[b];
      }
    }
  }
  energy[0] = energy[1] + energy[2];
  return OR_OK;
}

/* Point-charge Ewald real space: e = C qi qj g0 (the charge-charge routine of
 * the CHARMM profile).  Same exclusion reading as above. */
int or_echarge_real(int n, const double* xyz, double box, const int32_t* molid,
                    const int32_t* row_ptr, const int32_t* col, const double* q, double beta,
                    double rc, double* energy, double* force, double* virial) {
  int st = or_pair_args(n, box, rc);
  if (st) return st;
  double rc2 = rc * rc;
  energy[0] = energy[1] = energy[2] = 0.0;
  for (int k = 0; k < 9; ++k) virial[k] = 0.0;
  for (int k = 0; k < 3 * n; ++k) force[k] = 0.0;
  for (int i = 0; i < n; ++i) {
    for (int p = row_ptr[i]; p < row_ptr[i + 1]; ++p) {
      int j = col[p];
      double d[3], r2;
      or_image(xyz + 3 * i, xyz + 3 * j, box, d, &r2);
      if (!(r2 <= rc2)) continue;
      double r = sqrt(r2), B[2], R[2];
      or_radial(r, beta, 1, B, R);
      int excl = molid[i] == molid[j];
      double g0 = excl ? B[0] - R[0] : B[0];
      double g1 = excl ? B[1] - R[1] : B[1];
      double e = OR_COULOMB * q[i] * q[j] * g0;
      energy[excl ? 2 : 1] += e;
      for (int a = 0; a < 3; ++a) {
        double de = -OR_COULOMB * q[i] * q[j] * g1 * d[a];
        force[3 * i + a] += de;
        force[3 * j + a] -= de;
        for (int b = 0; b < 3; ++b) virial[3 * a + b] += d[a] * (-OR_COULOMB * q[i] * q[j] * g1 * d[b]);
      }
    }
  }
  energy[0] = energy[1] + energy[2];
  return OR_OK;
}

/* ------------------------------------------------------------------------ */
/* Permanent field (the right-hand side of the polarization equations;
 * section "Hotspots").  Field at i from the multipoles of j, with
 * T1 = -r g1, T2 = r r g2 - I g1, (T3:Theta)_a = -r_a Q g3 + 2 (Theta r)_a g2:
 *   E_i += qj T1 + T2 muj + T3:Thj,     E_j += -qi T1 + T2 mui - T3:Thi,
 * with g_n = B_n - (1 - s l_(2n+1)) R_n, s = intra for equal molid, else 1
 * (the Ewald correction of the scaled-out part is kept).
 * Plus the Ewald self field c mu_i, c = 4 beta^3 / (3 sqrt(pi)).
 * The field carries no Coulomb constant (units e/A^2). */
static int or_efield_scaled(int n, const double* xyz, double box, const int32_t* molid,
                            const int32_t* row_ptr, const int32_t* col, const double* mpole,
                            const double* polarity, const double* thole, double beta, double rc,
                            double intra, double* field) {
  int st = or_pair_args(n, box, rc);
  if (st) return st;
  double rc2 = rc * rc;
  double cself = 4.0 * beta * beta * beta / (3.0 * OR_SQRTPI);
  for (int i = 0; i < n; ++i)
    for (int a = 0; a < 3; ++a) field[3 * i + a] = cself * mpole[10 * i + 1 + a];
  for (int i = 0; i < n; ++i) {
    for (int p = row_ptr[i]; p < row_ptr[i + 1]; ++p) {
      int j = col[p];
      double d[3], r2;
      or_image(xyz + 3 * i, xyz + 3 * j, box, d, &r2);
      if (!(r2 <= rc2)) continue;
      double r = sqrt(r2), B[4], R[4], l3, l5, l7;
      or_radial(r, beta, 3, B, R);
      or_thole(r, polarity[i], polarity[j], thole[i], thole[j], &l3, &l5, &l7);
      double s = molid[i] == molid[j] ? intra : 1.0;
      double g1 = B[1] - (1.0 - s * l3) * R[1];
      double g2 = B[2] - (1.0 - s * l5) * R[2];
      double g3 = B[3] - (1.0 - s * l7) * R[3];
      double qi, qj, ui[3], uj[3], ti[3][3], tj[3][3];
      or_unpack(mpole + 10 * i, &qi, ui, ti);
      or_unpack(mpole + 10 * j, &qj, uj, tj);
      double di = or_dot(ui, d), dj = or_dot(uj, d), vi[3], vj[3];
      or_matvec3(ti, d, vi);
      or_matvec3(tj, d, vj);
      double Qi = or_dot(d, vi), Qj = or_dot(d, vj);
      for (int a = 0; a < 3; ++a) {
        double T1 = -d[a] * g1;
        double T2uj = d[a] * dj * g2 - uj[a] * g1;
        double T2ui = d[a] * di * g2 - ui[a] * g1;
        double T3j = -d[a] * Qj * g3 + 2.0 * vj[a] * g2;
        double T3i = -d[a] * Qi * g3 + 2.0 * vi[a] * g2;
        field[3 * i + a] += qj * T1 + T2uj + T3j;
        field[3 * j + a] += -qi * T1 + T2ui - T3i;
      }
    }
  }
  return OR_OK;
}

/* The field that drives the induced dipoles (reading: no direct field
 * inside a molecule, intra = 0). */
int or_efield_direct(int n, const double* xyz, double box, const int32_t* molid,
                     const int32_t* row_ptr, const int32_t* col, const double* mpole,
                     const double* polarity, const double* thole, double beta, double rc,
                     double* field) {
  return or_efield_scaled(n, xyz, box, molid, row_ptr, col, mpole, polarity, thole, beta, rc, 0.0,
                          field);
}

/* The same field with same-molecule pairs scaled by intra in [0, 1] (the
 * second field of the two-right-hand-side solve below). */
int or_efield_intra(int n, const double* xyz, double box, const int32_t* molid,
                    const int32_t* row_ptr, const int32_t* col, const double* mpole,
                    const double* polarity, const double* thole, double beta, double rc,
                    double intra, double* field) {
  if (!(intra >= 0.0 && intra <= 1.0)) return OR_E_ARG;
  return or_efield_scaled(n, xyz, box, molid, row_ptr, col, mpole, polarity, thole, beta, rc,
                          intra, field);
}

/* Mutual induced-dipole field (the polarization-solver mat-vec, the largest
 * hotspot of the Rel profile).  For every listed pair with r <= rc, the same
 * molecule included (reading: mutual scale 1):
 *   E_i += T2 mu_j,  E_j += T2 mu_i,  g1 = B1 - (1-l3) R1, g2 = B2 - (1-l5) R2,
 * plus the self field c mu_i.  include_diag = 0 returns this field (T + cI) mu;
 * include_diag = 1 returns A mu = mu/alpha - (T + cI) mu, the operator of the
 * polarization equations (zero rows for alpha = 0, reading). */
int or_tmatvec(int n, const double* xyz, double box, const int32_t* row_ptr,
               const int32_t* col, const double* polarity, const double* thole, double beta,
               double rc, int include_diag, const double* mu, double* out) {
  int st = or_pair_args(n, box, rc);
  if (st) return st;
  double rc2 = rc * rc;
  double cself = 4.0 * beta * beta * beta / (3.0 * OR_SQRTPI);
  double* fld = (double*)malloc(sizeof(double) * 3 * (size_t)(n > 0 ? n : 1));
  for (int k = 0; k < 3 * n; ++k) fld[k] = cself * mu[k];
  for (int i = 0; i < n; ++i) {
    for (int p = row_ptr[i]; p < row_ptr[i + 1]; ++p) {
      int j = col[p];
      double d[3], r2;
      or_image(xyz + 3 * i, xyz + 3 * j, box, d, &r2);
      if (!(r2 <= rc2)) continue;
      double r = sqrt(r2), B[3], R[3], l3, l5, l7;
      or_radial(r, beta, 2, B, R);
      or_thole(r, polarity[i], polarity[j], thole[i], thole[j], &l3, &l5, &l7);
      double g1 = B[1] - (1.0 - l3) * R[1];
      double g2 = B[2] - (1.0 - l5) * R[2];
      double di = or_dot(mu + 3 * i, d), dj = or_dot(mu + 3 * j, d);
      for (int a = 0; a < 3; ++a) {
        fld[3 * i + a] += d[a] * dj * g2 - mu[3 * j + a] * g1;
        fld[3 * j + a] += d[a] * di * g2 - mu[3 * i + a] * g1;
      }
    }
  }
  for (int i = 0; i < n; ++i)
    for (int a = 0; a < 3; ++a) {
      int k = 3 * i + a;
      if (!include_diag) out[k] = fld[k];
      else out[k] = polarity[i] > 0.0 ? mu[k] / polarity[i] - fld[k] : 0.0;
    }
  free(fld);
  return OR_OK;
}

/* ------------------------------------------------------------------------ */
/* Induced dipoles by preconditioned conjugate gradient (the polarization
 * solver of section "Hotspots", which calls the mat-vec up to 12 times per
 * step).  Reading: diagonal preconditioner M^-1 = alpha; initial guess
 * alpha * E_perm unless a guess is given; the convergence measure is the RMS
 * over polarizable atoms of the preconditioned residual z = alpha r, in Debye,
 * checked before each mat-vec; E_pol = -1/2 C sum_i mu_i . E_perm_i. */
typedef struct {
  int32_t status, iters, refinements, converged;
  double rms_debye, rms_true_debye, epol;
} or_pcg_info;

static double or_rmsd(int n, const double* z, int npol) {
  if (npol == 0) return 0.0;
  double s = 0.0;
  for (int k = 0; k < 3 * n; ++k) s += z[k] * z[k];
  return OR_DEBYE * sqrt(s / npol);
}

/* Optional reciprocal-space part of the polarization equations (the full
 * Ewald operator): the smooth-PME field of the dipoles themselves is added to
 * the dipole field of the operator, and the PME field of the permanent
 * multipoles to the right-hand side.  K = 0: real space only. */
typedef struct {
  int K, p;
} or_recip;

int or_pme_mpole(int n, const double* xyz, double box, const double* mpole, double beta, int K,
                 int p, double* energy, double* force, double* field);

/* PME field of dipoles v (no charges or quadrupoles) into fld. */
static void or_recip_dipole_field(int n, const double* xyz, double box, double beta,
                                  const or_recip* rp, const double* v, double* fld) {
  double* m = (double*)calloc((size_t)(n > 0 ? n : 1) * 10, sizeof(double));
  double* f = (double*)malloc(sizeof(double) * 3 * (size_t)(n > 0 ? n : 1));
  double e;
  for (int i = 0; i < n; ++i)
    for (int a = 0; a < 3; ++a) m[10 * i + 1 + a] = v[3 * i + a];
  or_pme_mpole(n, xyz, box, m, beta, rp->K, rp->p, &e, f, fld);
  free(m);
  free(f);
}

/* out = A v: the real-space operator of or_tmatvec minus, with a reciprocal
 * part, the PME dipole field (rows of alpha = 0 stay zero). */
static void or_apply_A(int n, const double* xyz, double box, const int32_t* row_ptr,
                       const int32_t* col, const double* polarity, const double* thole,
                       double beta, double rc, const or_recip* rp, const double* v, double* out) {
  or_tmatvec(n, xyz, box, row_ptr, col, polarity, thole, beta, rc, 1, v, out);
  if (!rp) return;
  double* fld = (double*)malloc(sizeof(double) * 3 * (size_t)(n > 0 ? n : 1));
  or_recip_dipole_field(n, xyz, box, beta, rp, v, fld);
  for (int i = 0; i < n; ++i)
    if (polarity[i] > 0.0)
      for (int a = 0; a < 3; ++a) out[3 * i + a] -= fld[3 * i + a];
  free(fld);
}

/* PCG on A x = b (b given, x = mu_out), E_pol = -1/2 C x.b. */
static int or_pcg_iterate(int n, const double* xyz, double box, const int32_t* row_ptr,
                          const int32_t* col, const double* polarity, const double* thole,
                          double beta, double rc, const or_recip* rp, const double* b,
                          double tol_debye, int maxiter, const double* mu_guess, double* mu_out,
                          or_pcg_info* info) {
  size_t m = 3 * (size_t)(n > 0 ? n : 1);
  double* r = (double*)malloc(sizeof(double) * m);
  double* z = (double*)malloc(sizeof(double) * m);
  double* p = (double*)malloc(sizeof(double) * m);
  double* q = (double*)malloc(sizeof(double) * m);
  double* x = mu_out;
  int npol = 0;
  for (int i = 0; i < n; ++i) npol += polarity[i] > 0.0;
  for (int i = 0; i < n; ++i)
    for (int a = 0; a < 3; ++a) {
      int k = 3 * i + a;
      x[k] = mu_guess ? (polarity[i] > 0.0 ? mu_guess[k] : 0.0) : polarity[i] * b[k];
    }
  or_apply_A(n, xyz, box, row_ptr, col, polarity, thole, beta, rc, rp, x, q);
  double rho = 0.0;
  for (int i = 0; i < n; ++i)
    for (int a = 0; a < 3; ++a) {
      int k = 3 * i + a;
      r[k] = polarity[i] > 0.0 ? b[k] - q[k] : 0.0;
      z[k] = polarity[i] * r[k];
      p[k] = z[k];
      rho += r[k] * z[k];
    }
  int status = OR_OK, converged = 0, it = 0;
  double rms = 0.0;
  for (it = 0;; ++it) {
    rms = or_rmsd(n, z, npol);
    if (rms <= tol_debye) { converged = 1; break; }
    if (it == maxiter) { status = OR_E_NOCONV; break; }
    or_apply_A(n, xyz, box, row_ptr, col, polarity, thole, beta, rc, rp, p, q);
    double gam = 0.0;
    for (int k = 0; k < 3 * n; ++k) gam += p[k] * q[k];
    if (!(gam > 0.0)) { status = OR_E_BREAKDOWN; break; }
    double alpha = rho / gam, rho1 = 0.0;
    for (int i = 0; i < n; ++i)
      for (int a = 0; a < 3; ++a) {
        int k = 3 * i + a;
        x[k] += alpha * p[k];
        r[k] -= alpha * q[k];
        z[k] = polarity[i] * r[k];
        rho1 += r[k] * z[k];
      }
    double bet = rho1 / rho;
    for (int k = 0; k < 3 * n; ++k) p[k] = z[k] + bet * p[k];
    rho = rho1;
  }
  /* final true residual, from a fresh mat-vec */
  or_apply_A(n, xyz, box, row_ptr, col, polarity, thole, beta, rc, rp, x, q);
  for (int i = 0; i < n; ++i)
    for (int a = 0; a < 3; ++a) {
      int k = 3 * i + a;
      z[k] = polarity[i] > 0.0 ? polarity[i] * (b[k] - q[k]) : 0.0;
    }
  double epol = 0.0;
  for (int k = 0; k < 3 * n; ++k) epol += x[k] * b[k];
  info->status = status;
  info->iters = it;
  info->refinements = 0;
  info->converged = converged;
  info->rms_debye = rms;
  info->rms_true_debye = or_rmsd(n, z, npol);
  info->epol = -0.5 * OR_COULOMB * epol;
  free(r); free(z); free(p); free(q);
  return status;
}

static int or_pcg_args(int n, double box, double rc, const double* polarity, double tol_debye,
                       int maxiter) {
  int st = or_pair_args(n, box, rc);
  if (st) return st;
  if (maxiter < 0 || !(tol_debye >= 0.0)) return OR_E_ARG;
  for (int i = 0; i < n; ++i)
    if (!(polarity[i] >= 0.0)) return OR_E_ARG;
  return OR_OK;
}

static int or_pcg(int n, const double* xyz, double box, const int32_t* molid,
                  const int32_t* row_ptr, const int32_t* col, const double* mpole,
                  const double* polarity, const double* thole, double beta, double rc,
                  const or_recip* rp, double tol_debye, int maxiter, const double* mu_guess,
                  double* mu_out, or_pcg_info* info) {
  int st = or_pcg_args(n, box, rc, polarity, tol_debye, maxiter);
  if (st) return st;
  size_t m = 3 * (size_t)(n > 0 ? n : 1);
  double* b = (double*)malloc(sizeof(double) * m);
  or_efield_direct(n, xyz, box, molid, row_ptr, col, mpole, polarity, thole, beta, rc, b);
  if (rp) {
    double e;
    double* f = (double*)malloc(sizeof(double) * m);
    double* fr = (double*)malloc(sizeof(double) * m);
    or_pme_mpole(n, xyz, box, mpole, beta, rp->K, rp->p, &e, f, fr);
    for (int k = 0; k < 3 * n; ++k) b[k] += fr[k];
    free(f);
    free(fr);
  }
  st = or_pcg_iterate(n, xyz, box, row_ptr, col, polarity, thole, beta, rc, rp, b, tol_debye,
                      maxiter, mu_guess, mu_out, info);
  free(b);
  return st;
}

int or_polarize_pcg(int n, const double* xyz, double box, const int32_t* molid,
                    const int32_t* row_ptr, const int32_t* col, const double* mpole,
                    const double* polarity, const double* thole, double beta, double rc,
                    double tol_debye, int maxiter, const double* mu_guess, double* mu_out,
                    or_pcg_info* info) {
  return or_pcg(n, xyz, box, molid, row_ptr, col, mpole, polarity, thole, beta, rc, NULL,
                tol_debye, maxiter, mu_guess, mu_out, info);
}

/* The same solve with the full Ewald operator: the PME reciprocal field of
 * the dipoles (grid K, order p) in A, that of the permanent multipoles in the
 * right-hand side (E_perm = real-space field + self field + reciprocal
 * field).  E_pol = -1/2 C mu.E_perm with the full field. */
int or_polarize_pcg_ewald(int n, const double* xyz, double box, const int32_t* molid,
                          const int32_t* row_ptr, const int32_t* col, const double* mpole,
                          const double* polarity, const double* thole, double beta, double rc,
                          int K, int p, double tol_debye, int maxiter, const double* mu_guess,
                          double* mu_out, or_pcg_info* info) {
  if (!(beta > 0.0) || K < 2 * p || p < 5 || p > 8) return OR_E_ARG;
  or_recip rp = {K, p};
  return or_pcg(n, xyz, box, molid, row_ptr, col, mpole, polarity, thole, beta, rc, &rp,
                tol_debye, maxiter, mu_guess, mu_out, info);
}

/* Two right-hand sides on the same operator (the polarization model of
 * section "Polarizable AMOEBA force field" with the solver of section
 * "Hotspots"; batched solves are named among the solver work of section
 * "Perspectives on Tinker-HP 1.2 performance").  Reading: AMOEBA induces two
 * dipole sets from two permanent fields that differ only in the factor on
 * same-molecule pairs: mu_d from E_d (factor 0, or_efield_direct) and mu_p
 * from E_p (factor pscale, or_efield_intra).  Both solve A mu = E with the
 * same A, each by its own PCG recurrence (same guess rule, same stopping
 * test).  The energy is E_pol = -1/2 C mu_d.E_p; by the symmetry of A this is
 * also -1/2 C mu_p.E_d, up to the residuals.  info[0] is mu_d's solve with
 * epol = -1/2 C mu_d.E_p; info[1] is mu_p's with epol = -1/2 C mu_p.E_d.
 * mu_guess (nullable) and mu_out are [2][n][3], mu_d first. */
static int or_pcg2(int n, const double* xyz, double box, const int32_t* molid,
                   const int32_t* row_ptr, const int32_t* col, const double* mpole,
                   const double* polarity, const double* thole, double beta, double rc,
                   const or_recip* rp, double pscale, double tol_debye, int maxiter,
                   const double* mu_guess, double* mu_out, or_pcg_info* info) {
  int st = or_pcg_args(n, box, rc, polarity, tol_debye, maxiter);
  if (st) return st;
  if (!(pscale >= 0.0 && pscale <= 1.0)) return OR_E_ARG;
  size_t m = 3 * (size_t)(n > 0 ? n : 1);
  double* ed = (double*)malloc(sizeof(double) * m);
  double* ep = (double*)malloc(sizeof(double) * m);
  or_efield_scaled(n, xyz, box, molid, row_ptr, col, mpole, polarity, thole, beta, rc, 0.0, ed);
  or_efield_scaled(n, xyz, box, molid, row_ptr, col, mpole, polarity, thole, beta, rc, pscale, ep);
  if (rp) {   /* the reciprocal permanent field joins both (no molecule scaling there) */
    double e;
    double* f = (double*)malloc(sizeof(double) * m);
    double* fr = (double*)malloc(sizeof(double) * m);
    or_pme_mpole(n, xyz, box, mpole, beta, rp->K, rp->p, &e, f, fr);
    for (int k = 0; k < 3 * n; ++k) {
      ed[k] += fr[k];
      ep[k] += fr[k];
    }
    free(f);
    free(fr);
  }
  double* mud = mu_out;
  double* mup = mu_out + 3 * (size_t)n;
  int sd = or_pcg_iterate(n, xyz, box, row_ptr, col, polarity, thole, beta, rc, rp, ed,
                          tol_debye, maxiter, mu_guess, mud, &info[0]);
  int sp = or_pcg_iterate(n, xyz, box, row_ptr, col, polarity, thole, beta, rc, rp, ep,
                          tol_debye, maxiter, mu_guess ? mu_guess + 3 * (size_t)n : NULL, mup,
                          &info[1]);
  double dp = 0.0, pd = 0.0;
  for (int k = 0; k < 3 * n; ++k) {
    dp += mud[k] * ep[k];
    pd += mup[k] * ed[k];
  }
  info[0].epol = -0.5 * OR_COULOMB * dp;
  info[1].epol = -0.5 * OR_COULOMB * pd;
  free(ed);
  free(ep);
  return sd ? sd : sp;
}

int or_polarize_pcg2(int n, const double* xyz, double box, const int32_t* molid,
                     const int32_t* row_ptr, const int32_t* col, const double* mpole,
                     const double* polarity, const double* thole, double beta, double rc,
                     double pscale, double tol_debye, int maxiter, const double* mu_guess,
                     double* mu_out, or_pcg_info* info) {
  return or_pcg2(n, xyz, box, molid, row_ptr, col, mpole, polarity, thole, beta, rc, NULL, pscale,
                 tol_debye, maxiter, mu_guess, mu_out, info);
}

/* Both sets with the full Ewald operator (as or_polarize_pcg_ewald): the PME
 * dipole field in A, and the PME field of the permanent multipoles added to
 * both right-hand sides. */
int or_polarize_pcg2_ewald(int n, const double* xyz, double box, const int32_t* molid,
                           const int32_t* row_ptr, const int32_t* col, const double* mpole,
                           const double* polarity, const double* thole, double beta, double rc,
                           int K, int p, double pscale, double tol_debye, int maxiter,
                           const double* mu_guess, double* mu_out, or_pcg_info* info) {
  if (!(beta > 0.0) || K < 2 * p || p < 5 || p > 8) return OR_E_ARG;
  or_recip rp = {K, p};
  return or_pcg2(n, xyz, box, molid, row_ptr, col, mpole, polarity, thole, beta, rc, &rp, pscale,
                 tol_debye, maxiter, mu_guess, mu_out, info);
}

/* ------------------------------------------------------------------------ */
/* Polarization forces (the induced-dipole gradient routine that the Rel
 * profile ranks second among the AMOEBA hotspots, section "Hotspots").
 *
 * With A = 1/alpha - (T + cI) the operator of the polarization equations and
 * E_p the permanent field, the polarization energy is the minimum over mu of
 *   E(r, mu) = C [ 1/2 mu.A(r) mu - mu.E_p(r) ],
 * reached where A mu = E_p, with value -1/2 C mu.E_p (the solver's E_pol).
 * Reading: the force is -dE/dr at fixed mu.  At the converged dipoles this
 * is the gradient of E_pol itself (dE/dmu = 0 there); at any other mu it is
 * the gradient of E(r, mu) for that mu.
 *
 * The position-dependent part of E(r, mu) is a sum over listed pairs with
 * r <= rc.  Writing an induced dipole as the multipole (0, mu, 0):
 *   e_ip = U(mu_i, M_j; gp) + U(M_i, mu_j; gp)     (= -C mu_i.E_i<-j - C mu_j.E_j<-i)
 *   e_ii = U(mu_i, mu_j; gm)                        (= -C mu_i.T2 mu_j)
 * where U is the multipole pair energy of or_mpole_pair and the radial
 * families are those of the two fields:
 *   gp_n = B_n - (1 - s l_(2n+1)) R_n   (s = 0 for equal molid, else 1),
 *   gm_n = B_n - (1 - l_(2n+1)) R_n     (every pair).
 * The Thole factors obey (l_(2n+1) R_n)' = -r l_(2n+3) R_(n+1), as B_n and
 * R_n do, so or_mpole_pair's gradient rule holds for these families too;
 * the gradient of the quadrupole field term needs one more factor,
 *   l9 = 1 - (1 + x + 18/35 x^2 + 9/35 x^3) e^-x.
 * energy[0] = e_ip + e_ii summed, energy[1] = sum of e_ip, energy[2] = sum
 * of e_ii; forces F = -dE/dx; virial W_ab = sum over pairs of r_a de/dr_b. */
double or_thole_l9(double r, double ai, double aj, double ti, double tj) {
  double prod = ai * aj;
  if (prod == 0.0) return 1.0;
  double a = ti < tj ? ti : tj;
  double x = a * r * r * r / sqrt(prod);
  return 1.0 - (1.0 + x + (18.0 / 35.0) * x * x + (9.0 / 35.0) * x * x * x) * exp(-x);
}

int or_epolar_real(int n, const double* xyz, double box, const int32_t* molid,
                   const int32_t* row_ptr, const int32_t* col, const double* mpole,
                   const double* polarity, const double* thole, const double* mu, double beta,
                   double rc, double* energy, double* force, double* virial) {
  int st = or_pair_args(n, box, rc);
  if (st) return st;
  double rc2 = rc * rc;
  energy[0] = energy[1] = energy[2] = 0.0;
  for (int k = 0; k < 9; ++k) virial[k] = 0.0;
  for (int k = 0; k < 3 * n; ++k) force[k] = 0.0;
  for (int i = 0; i < n; ++i) {
    for (int p = row_ptr[i]; p < row_ptr[i + 1]; ++p) {
      int j = col[p];
      double d[3], r2;
      or_image(xyz + 3 * i, xyz + 3 * j, box, d, &r2);
      if (!(r2 <= rc2)) continue;
      double r = sqrt(r2), B[6], R[6], l[5];
      or_radial(r, beta, 5, B, R);
      or_thole(r, polarity[i], polarity[j], thole[i], thole[j], &l[1], &l[2], &l[3]);
      l[4] = or_thole_l9(r, polarity[i], polarity[j], thole[i], thole[j]);
      double s = molid[i] == molid[j] ? 0.0 : 1.0;
      /* l[n] multiplies R_n; R_0 (and R_5) never meet a nonzero coefficient
       * when one side is a pure dipole: c0 = c4 = 0 */
      double gp[6], gm[6];
      gp[0] = gm[0] = 0.0;
      gp[5] = gm[5] = 0.0;
      for (int k = 1; k <= 4; ++k) {
        gp[k] = B[k] - (1.0 - s * l[k]) * R[k];
        gm[k] = B[k] - (1.0 - l[k]) * R[k];
      }
      double ind_i[10] = {0.0}, ind_j[10] = {0.0};
      for (int a = 0; a < 3; ++a) {
        ind_i[1 + a] = mu[3 * i + a];
        ind_j[1 + a] = mu[3 * j + a];
      }
      double e1, e2, e3, de1[3], de2[3], de3[3];
      or_mpole_pair(d, ind_i, mpole + 10 * j, gp, &e1, de1);
      or_mpole_pair(d, mpole + 10 * i, ind_j, gp, &e2, de2);
      or_mpole_pair(d, ind_i, ind_j, gm, &e3, de3);
      energy[1] += e1 + e2;
      energy[2] += e3;
      for (int a = 0; a < 3; ++a) {
        double de = de1[a] + de2[a] + de3[a];
        force[3 * i + a] += de;
        force[3 * j + a] -= de;
      }
      for (int a = 0; a < 3; ++a)
        for (int b = 0; b < 3; ++b) virial[3 * a + b] += d[a] * (de1[b] + de2[b] + de3[b]);
    }
  }
  energy[0] = energy[1] + energy[2];
  return OR_OK;
}

/* Polarization forces with the two dipole sets of or_polarize_pcg2.  The
 * energy -1/2 C E_d.A^-1 E_p is the stationary value, over (x, y), of
 *   L(r, x, y) = 1/2 C [ x.A(r) y - x.E_p(r) - y.E_d(r) ],
 * reached at x = mu_d, y = mu_p (A symmetric).  Reading: the force is
 * -dL/dr at fixed (mu_d, mu_p): at the solved sets the gradient of E_pol,
 * at any others that of L.  Its position-dependent part is a sum over listed
 * pairs with r <= rc:
 *   e_ip = 1/2 [U(mu_d,i, M_j; gp(pscale)) + U(M_i, mu_d,j; gp(pscale))]
 *        + 1/2 [U(mu_p,i, M_j; gp(0)) + U(M_i, mu_p,j; gp(0))]
 *   e_ii = 1/2 [U(mu_d,i, mu_p,j; gm) + U(mu_p,i, mu_d,j; gm)]
 * with the families of or_epolar_real, gp(s) taking s on same-molecule
 * pairs: each set meets the field that drives the other.  mu2 is
 * [2][n][3], mu_d first.  Outputs as or_epolar_real. */
int or_epolar2_real(int n, const double* xyz, double box, const int32_t* molid,
                    const int32_t* row_ptr, const int32_t* col, const double* mpole,
                    const double* polarity, const double* thole, const double* mu2,
                    double beta, double rc, double pscale, double* energy, double* force,
                    double* virial) {
  int st = or_pair_args(n, box, rc);
  if (st) return st;
  if (!(pscale >= 0.0 && pscale <= 1.0)) return OR_E_ARG;
  const double* mud = mu2;
  const double* mup = mu2 + 3 * (size_t)n;
  double rc2 = rc * rc;
  energy[0] = energy[1] = energy[2] = 0.0;
  for (int k = 0; k < 9; ++k) virial[k] = 0.0;
  for (int k = 0; k < 3 * n; ++k) force[k] = 0.0;
  for (int i = 0; i < n; ++i) {
    for (int p = row_ptr[i]; p < row_ptr[i + 1]; ++p) {
      int j = col[p];
      double d[3], r2;
      or_image(xyz + 3 * i, xyz + 3 * j, box, d, &r2);
      if (!(r2 <= rc2)) continue;
      double r = sqrt(r2), B[6], R[6], l[5];
      or_radial(r, beta, 5, B, R);
      or_thole(r, polarity[i], polarity[j], thole[i], thole[j], &l[1], &l[2], &l[3]);
      l[4] = or_thole_l9(r, polarity[i], polarity[j], thole[i], thole[j]);
      int same = molid[i] == molid[j];
      double sd = same ? pscale : 1.0, sp = same ? 0.0 : 1.0;
      double gd[6] = {0.0}, gq[6] = {0.0}, gm[6] = {0.0};
      for (int k = 1; k <= 4; ++k) {
        gd[k] = B[k] - (1.0 - sd * l[k]) * R[k];   /* field E_p, met by mu_d */
        gq[k] = B[k] - (1.0 - sp * l[k]) * R[k];   /* field E_d, met by mu_p */
        gm[k] = B[k] - (1.0 - l[k]) * R[k];
      }
      double di[10] = {0.0}, dj[10] = {0.0}, pi[10] = {0.0}, pj[10] = {0.0};
      for (int a = 0; a < 3; ++a) {
        di[1 + a] = mud[3 * i + a];
        dj[1 + a] = mud[3 * j + a];
        pi[1 + a] = mup[3 * i + a];
        pj[1 + a] = mup[3 * j + a];
      }
      double e[6], de[6][3];
      or_mpole_pair(d, di, mpole + 10 * j, gd, &e[0], de[0]);
      or_mpole_pair(d, mpole + 10 * i, dj, gd, &e[1], de[1]);
      or_mpole_pair(d, pi, mpole + 10 * j, gq, &e[2], de[2]);
      or_mpole_pair(d, mpole + 10 * i, pj, gq, &e[3], de[3]);
      or_mpole_pair(d, di, pj, gm, &e[4], de[4]);
      or_mpole_pair(d, pi, dj, gm, &e[5], de[5]);
      energy[1] += 0.5 * (e[0] + e[1] + e[2] + e[3]);
      energy[2] += 0.5 * (e[4] + e[5]);
      double g[3];
      for (int a = 0; a < 3; ++a) {
        g[a] = 0.5 * (de[0][a] + de[1][a] + de[2][a] + de[3][a] + de[4][a] + de[5][a]);
        force[3 * i + a] += g[a];
        force[3 * j + a] -= g[a];
      }
      for (int a = 0; a < 3; ++a)
        for (int b = 0; b < 3; ++b) virial[3 * a + b] += d[a] * g[b];
    }
  }
  energy[0] = energy[1] + energy[2];
  return OR_OK;
}

/* ------------------------------------------------------------------------ */
/* van der Waals (the Halgren 14-7 and LJ 12-6 routines of the Rel profile).
 * HAL, in the quantities of the paper's compute loop (Listing
 * "calculation"): rv = R_ij, rv7 = rv^7, rik7 = r^7,
 * invrho = 1/(rik7 + ghal rv7), invtmp = 1/(r + dhal rv):
 *   e = eps_ij [(1+dhal) rv invtmp]^7 [(1+ghal) rv7 invrho - 2].
 * Readings: R_ij = (Ri^3 + Rj^3)/(Ri^2 + Rj^2),
 * eps_ij = 4 ei ej / (sqrt(ei) + sqrt(ej))^2, no hydrogen reduction.
 * LJ: e = 4 eps_ij [(s/r)^12 - (s/r)^6], s = (si+sj)/2, eps_ij = sqrt(ei ej).
 * Both: pairs with equal molid are skipped; the energy is multiplied by the
 * taper S(x) = 1 - 10x^3 + 15x^4 - 6x^5, x = (r - ron)/(rc - ron),
 * ron = taper_frac * rc, for r > ron. */
#define OR_VDW_HAL 0
#define OR_VDW_LJ 1

static void or_vdw_pair(int form, double r, double ri, double rj, double ei, double ej,
                        double dhal, double ghal, double* e, double* dedr) {
  if (form == OR_VDW_HAL) {
    double rv = (ri * ri * ri + rj * rj * rj) / (ri * ri + rj * rj);
    double se = sqrt(ei) + sqrt(ej);
    double eps = se > 0.0 ? 4.0 * ei * ej / (se * se) : 0.0;
    double rv7 = pow(rv, 7.0);
    double rik7 = pow(r, 7.0);
    double invrho = 1.0 / (rik7 + ghal * rv7);
    double invtmp = 1.0 / (r + dhal * rv);
    double t7 = pow((1.0 + dhal) * rv * invtmp, 7.0);
    double w = (1.0 + ghal) * rv7 * invrho;
    *e = eps * t7 * (w - 2.0);
    /* d t7/dr = -7 t7 invtmp ; d w/dr = -7 r^6 w invrho */
    *dedr = eps * (-7.0 * t7 * invtmp * (w - 2.0) - t7 * 7.0 * pow(r, 6.0) * w * invrho);
  } else {
    double s = 0.5 * (ri + rj);
    double eps = sqrt(ei * ej);
    double sr6 = pow(s / r, 6.0);
    *e = 4.0 * eps * (sr6 * sr6 - sr6);
    *dedr = 4.0 * eps * (-12.0 * sr6 * sr6 + 6.0 * sr6) / r;
  }
}

int or_evdw(int n, const double* xyz, double box, const int32_t* molid, const int32_t* row_ptr,
            const int32_t* col, int form, const double* rad, const double* eps, double rc,
            double taper_frac, double dhal, double ghal, double* energy, double* force,
            double* virial) {
  int st = or_pair_args(n, box, rc);
  if (st) return st;
  if (form != OR_VDW_HAL && form != OR_VDW_LJ) return OR_E_ARG;
  double rc2 = rc * rc, ron = taper_frac * rc;
  *energy = 0.0;
  for (int k = 0; k < 9; ++k) virial[k] = 0.0;
  for (int k = 0; k < 3 * n; ++k) force[k] = 0.0;
  for (int i = 0; i < n; ++i) {
    for (int p = row_ptr[i]; p < row_ptr[i + 1]; ++p) {
      int j = col[p];
      if (molid[i] == molid[j]) continue;
      double d[3], r2;
      or_image(xyz + 3 * i, xyz + 3 * j, box, d, &r2);
      if (!(r2 <= rc2)) continue;
      double r = sqrt(r2), e, dedr;
      or_vdw_pair(form, r, rad[i], rad[j], eps[i], eps[j], dhal, ghal, &e, &dedr);
      if (r > ron) {
        double w = rc - ron, x = (r - ron) / w;
        double S = 1.0 - 10.0 * pow(x, 3) + 15.0 * pow(x, 4) - 6.0 * pow(x, 5);
        double dS = (-30.0 * x * x + 60.0 * pow(x, 3) - 30.0 * pow(x, 4)) / w;
        dedr = dedr * S + e * dS;
        e *= S;
      }
      *energy += e;
      for (int a = 0; a < 3; ++a) {
        double de = dedr * d[a] / r;
        force[3 * i + a] += de;
        force[3 * j + a] -= de;
        for (int b = 0; b < 3; ++b) virial[3 * a + b] += d[a] * dedr * d[b] / r;
      }
    }
  }
  return OR_OK;
}

/* ------------------------------------------------------------------------ */
/* Validation-only Ewald pieces (not on the GPU path).
 * Self energy: -C beta/sqrt(pi) sum_i [qi^2 + (2 beta^2/3)|mui|^2
 *                                      + (8 beta^4/5) Thi:Thi].
 * Reciprocal energy (tin-foil):
 *   (C/2V) sum_{k != 0} (4 pi/k^2) exp(-k^2/(4 beta^2)) |S(k)|^2,
 *   S(k) = sum_j (qj + i muj.k - Thj:kk) exp(i k.r_j), k = 2 pi m / L,
 * over integer vectors m with |m_a| <= kmax. */
double or_eself(int n, const double* mpole, double beta) {
  double s = 0.0;
  for (int i = 0; i < n; ++i) {
    double q, u[3], t[3][3];
    or_unpack(mpole + 10 * i, &q, u, t);
    double tt = 0.0;
    for (int a = 0; a < 3; ++a)
      for (int b = 0; b < 3; ++b) tt += t[a][b] * t[a][b];
    s += q * q + (2.0 * beta * beta / 3.0) * or_dot(u, u) + (8.0 * pow(beta, 4) / 5.0) * tt;
  }
  return -OR_COULOMB * beta / OR_SQRTPI * s;
}

double or_erecip(int n, const double* xyz, double box, const double* mpole, double beta,
                 int kmax) {
  const double twopi = 6.283185307179586477;
  double vol = box * box * box, sum = 0.0;
  for (int mx = -kmax; mx <= kmax; ++mx)
    for (int my = -kmax; my <= kmax; ++my)
      for (int mz = -kmax; mz <= kmax; ++mz) {
        if (!mx && !my && !mz) continue;
        double k[3] = {twopi * mx / box, twopi * my / box, twopi * mz / box};
        double k2 = or_dot(k, k);
        double damp = exp(-k2 / (4.0 * beta * beta)) * 4.0 * M_PI / k2;
        if (damp < 1e-300) continue;
        double sr = 0.0, si = 0.0;
        for (int j = 0; j < n; ++j) {
          double q, u[3], t[3][3], tk[3];
          or_unpack(mpole + 10 * j, &q, u, t);
          or_matvec3(t, k, tk);
          double re = q - or_dot(k, tk), im = or_dot(u, k);
          double ph = or_dot(k, xyz + 3 * j);
          double c = cos(ph), s = sin(ph);
          sr += re * c - im * s;
          si += re * s + im * c;
        }
        sum += damp * (sr * sr + si * si);
      }
  return OR_COULOMB * sum / (2.0 * vol);
}

/* Reciprocal-space forces and field by the same k-sum (validation only).
 * With a_j = qj - Thj:kk + i muj.k and S(k) = sum_j a_j exp(i k.r_j):
 *   potential phi(y) = (1/V) sum_k G(k) Re[exp(i k.y) conj S(k)],
 *   G(k) = (4 pi/k^2) exp(-k^2/(4 beta^2));
 *   field_i = -grad phi(r_i) (no Coulomb constant; it includes the site's
 *   own contribution, which the Ewald self field removes);
 *   force_j = -dE/dr_j = (C/V) sum_k G(k) k Im[a_j exp(i k.r_j) conj S(k)]. */
int or_erecip_grad(int n, const double* xyz, double box, const double* mpole, double beta,
                   int kmax, double* force, double* field) {
  if (n < 0 || !(box > 0.0) || !(beta > 0.0) || kmax < 0) return OR_E_ARG;
  const double twopi = 6.283185307179586477;
  double vol = box * box * box;
  double* ar = (double*)malloc(sizeof(double) * (size_t)(n > 0 ? n : 1));
  double* ai = (double*)malloc(sizeof(double) * (size_t)(n > 0 ? n : 1));
  double* cr = (double*)malloc(sizeof(double) * (size_t)(n > 0 ? n : 1));
  double* ci = (double*)malloc(sizeof(double) * (size_t)(n > 0 ? n : 1));
  for (int k = 0; k < 3 * n; ++k) force[k] = field[k] = 0.0;
  for (int mx = -kmax; mx <= kmax; ++mx)
    for (int my = -kmax; my <= kmax; ++my)
      for (int mz = -kmax; mz <= kmax; ++mz) {
        if (!mx && !my && !mz) continue;
        double k[3] = {twopi * mx / box, twopi * my / box, twopi * mz / box};
        double k2 = or_dot(k, k);
        double G = exp(-k2 / (4.0 * beta * beta)) * 4.0 * M_PI / k2;
        if (G < 1e-300) continue;
        double sr = 0.0, si = 0.0;
        for (int j = 0; j < n; ++j) {
          double q, u[3], t[3][3], tk[3];
          or_unpack(mpole + 10 * j, &q, u, t);
          or_matvec3(t, k, tk);
          ar[j] = q - or_dot(k, tk);
          ai[j] = or_dot(u, k);
          double ph = or_dot(k, xyz + 3 * j);
          cr[j] = cos(ph);
          ci[j] = sin(ph);
          sr += ar[j] * cr[j] - ai[j] * ci[j];
          si += ar[j] * ci[j] + ai[j] * cr[j];
        }
        for (int j = 0; j < n; ++j) {
          /* a_j e^{ik.r_j} conj(S) and e^{ik.r_j} conj(S): imaginary parts */
          double tr = ar[j] * cr[j] - ai[j] * ci[j], ti = ar[j] * ci[j] + ai[j] * cr[j];
          double im_f = ti * sr - tr * si;
          double im_e = ci[j] * sr - cr[j] * si;
          for (int a = 0; a < 3; ++a) {
            force[3 * j + a] += OR_COULOMB / vol * G * k[a] * im_f;
            field[3 * j + a] += G * k[a] * im_e / vol;
          }
        }
      }
  free(ar); free(ai); free(cr); free(ci);
  return OR_OK;
}

/* ------------------------------------------------------------------------ */
/* Smooth particle-mesh Ewald for the reciprocal-space multipole energy (the
 * reciprocal multipole routine that section "Hotspots" names beside the
 * real-space one; the paper leaves it unvectorized).  Reading: the textbook
 * smooth PME of Essmann et al. (1995) with cardinal B-splines, extended to
 * dipoles and quadrupoles by differentiating the spline (as in Sagui,
 * Pedersen and Darden, 2004); no further correction of the spline moduli.
 *
 * Cardinal B-spline of order p on (0, p):
 *   M_2(x) = 1 - |x - 1|,  M_p(x) = [x M_(p-1)(x) + (p - x) M_(p-1)(x - 1)] / (p - 1),
 *   M_p'(x) = M_(p-1)(x) - M_(p-1)(x - 1)   (deriv <= p - 2). */
double or_bspline(int p, double x, int deriv) {
  if (deriv > 0) return or_bspline(p - 1, x, deriv - 1) - or_bspline(p - 1, x - 1.0, deriv - 1);
  if (!(x > 0.0) || !(x < p)) return 0.0;
  if (p == 2) return 1.0 - fabs(x - 1.0);
  return (x * or_bspline(p - 1, x, 0) + (p - x) * or_bspline(p - 1, x - 1.0, 0)) / (p - 1);
}

/* Spline modulus D(m) = |sum_{k=0}^{p-2} M_p(k+1) exp(2 pi i m k/K)|^2, so that
 * |b(m)|^2 = 1/D(m).  Reading: where D vanishes (m = K/2 for odd p) it is
 * replaced by the mean of its two neighbours. */
static double or_spline_mod_raw(int p, int K, int m) {
  double sr = 0.0, si = 0.0;
  for (int k = 0; k <= p - 2; ++k) {
    double w = or_bspline(p, k + 1.0, 0), ang = 6.283185307179586477 * m * k / K;
    sr += w * cos(ang);
    si += w * sin(ang);
  }
  return sr * sr + si * si;
}

double or_spline_mod(int p, int K, int m) {
  double d = or_spline_mod_raw(p, K, m);
  if (d < 1e-10)
    d = 0.5 * (or_spline_mod_raw(p, K, (m + K - 1) % K) + or_spline_mod_raw(p, K, (m + 1) % K));
  return d;
}

/* Reciprocal-space multipole energy, forces and field by smooth PME on a
 * K x K x K grid with splines of order p, 5 <= p <= 8 (quadrupole forces need
 * the third derivative of the spline), K >= 2p.  In the order of the method:
 *  1. u_j = K frac(x_j / L) per axis; the weights of grid point g are the
 *     tensor product of M_p(u_j - g) (g = floor(u_j) - t, t = 0..p-1, taken
 *     mod K), and d/dx of a weight is (K/L) M_p'.
 *  2. Spread: Q(g) = sum_j [qj M + muj.grad M + Thj:grad grad M](u_j - g),
 *     which interpolates S(k) as b(m) sum_g Q(g) exp(2 pi i m.g/K).
 *  3. F(m) = sum_g Q(g) exp(+2 pi i m.g/K) (plain separable DFT).
 *  4. W(m) = (4 pi/k^2) exp(-k^2/(4 beta^2)) / (V D(m1) D(m2) D(m3)), k = 2 pi m'/L
 *     with m' the signed frequency (m' = m for m <= K/2, else m - K); W(0) = 0.
 *  5. phi(g) = sum_m W(m) F(m) exp(-2 pi i m.g/K): the potential on the grid
 *     (e/A), E = (C/2) sum_g Q(g) phi(g).
 *  6. Interpolate phi and its derivatives up to third order at each site:
 *     phi^(abc)(r_j) = sum_g phi(g) d^abc M(u_j - g).
 * Then energy = (C/2) sum_j [qj phi + muj.grad phi + Thj:grad grad phi],
 * force_j = -C [qj grad phi + (grad grad phi) muj + (grad grad grad phi):Thj],
 * field_j = -grad phi(r_j) (includes the site's own contribution, as the
 * k-sum field does).  field may be NULL. */
int or_pme_mpole(int n, const double* xyz, double box, const double* mpole, double beta, int K,
                 int p, double* energy, double* force, double* field) {
  if (n < 0 || !(box > 0.0) || !(beta > 0.0) || K < 2 * p || p < 5 || p > 8) return OR_E_ARG;
  const double twopi = 6.283185307179586477;
  size_t KK = (size_t)K * K * K;
  double* Q = (double*)calloc(KK, sizeof(double));
  double* Fr = (double*)malloc(sizeof(double) * KK);
  double* Fi = (double*)malloc(sizeof(double) * KK);
  double* Tr = (double*)malloc(sizeof(double) * KK);
  double* Ti = (double*)malloc(sizeof(double) * KK);
  double* phi = (double*)malloc(sizeof(double) * KK);
  double* cs = (double*)malloc(sizeof(double) * (size_t)K * K);
  double* sn = (double*)malloc(sizeof(double) * (size_t)K * K);
  double* th = (double*)malloc(sizeof(double) * (size_t)(n > 0 ? n : 1) * 3 * p * 4);
  int* g0 = (int*)malloc(sizeof(int) * (size_t)(n > 0 ? n : 1) * 3);
  double kl = K / box;
  /* 1. spline weights and derivatives, th[j][axis][t][d] */
  for (int j = 0; j < n; ++j)
    for (int a = 0; a < 3; ++a) {
      double x = xyz[3 * j + a] / box;
      double u = K * (x - floor(x));
      int i0 = (int)floor(u);
      double w = u - i0;
      g0[3 * j + a] = i0;
      for (int t = 0; t < p; ++t)
        for (int d = 0; d < 4; ++d)
          th[(((size_t)j * 3 + a) * p + t) * 4 + d] =
              or_bspline(p, w + t, d) * pow(kl, d);
    }
#define TH(j, a, t, d) th[((((size_t)(j)) * 3 + (a)) * p + (t)) * 4 + (d)]
#define GIX(j, a, t) ((((g0[3 * (j) + (a)] - (t)) % K) + K) % K)
  /* 2. spread */
  for (int j = 0; j < n; ++j) {
    double q, u[3], T[3][3];
    or_unpack(mpole + 10 * j, &q, u, T);
    for (int t1 = 0; t1 < p; ++t1)
      for (int t2 = 0; t2 < p; ++t2)
        for (int t3 = 0; t3 < p; ++t3) {
          int tt[3] = {t1, t2, t3};
          double v = 0.0;
          /* derivative orders (dx, dy, dz) with dx + dy + dz <= 2 */
          for (int dx = 0; dx <= 2; ++dx)
            for (int dy = 0; dy <= 2 - dx; ++dy)
              for (int dz = 0; dz <= 2 - dx - dy; ++dz) {
                double wgt = TH(j, 0, tt[0], dx) * TH(j, 1, tt[1], dy) * TH(j, 2, tt[2], dz);
                int ord = dx + dy + dz;
                double c = 0.0;
                if (ord == 0) c = q;
                else if (ord == 1) c = dx ? u[0] : (dy ? u[1] : u[2]);
                else {
                  /* Theta : grad grad, full symmetric sum */
                  int ia = dx ? 0 : (dy ? 1 : 2);
                  int ib = dx == 2 ? 0 : (dy == 2 ? 1 : (dz == 2 ? 2 : -1));
                  if (ib >= 0) c = T[ia][ia];
                  else {
                    int i1 = dx ? 0 : 1, i2 = dz ? 2 : 1;
                    c = 2.0 * T[i1][i2];
                  }
                }
                v += c * wgt;
              }
          size_t g = ((size_t)GIX(j, 0, t1) * K + GIX(j, 1, t2)) * K + GIX(j, 2, t3);
          Q[g] += v;
        }
  }
  /* 3. F(m) = sum_g Q(g) exp(+2 pi i m.g/K), one axis at a time */
  for (int m = 0; m < K; ++m)
    for (int g = 0; g < K; ++g) {
      cs[m * K + g] = cos(twopi * (double)((long)m * g % K) / K);
      sn[m * K + g] = sin(twopi * (double)((long)m * g % K) / K);
    }
  for (size_t k = 0; k < KK; ++k) { Fr[k] = Q[k]; Fi[k] = 0.0; }
  for (int axis = 0; axis < 3; ++axis) {
    for (int a = 0; a < K; ++a)
      for (int b = 0; b < K; ++b)
        for (int m = 0; m < K; ++m) {
          double sr = 0.0, si = 0.0;
          for (int g = 0; g < K; ++g) {
            size_t idx = axis == 0 ? ((size_t)g * K + a) * K + b
                       : axis == 1 ? ((size_t)a * K + g) * K + b : ((size_t)a * K + b) * K + g;
            sr += Fr[idx] * cs[m * K + g] - Fi[idx] * sn[m * K + g];
            si += Fr[idx] * sn[m * K + g] + Fi[idx] * cs[m * K + g];
          }
          size_t o = axis == 0 ? ((size_t)m * K + a) * K + b
                   : axis == 1 ? ((size_t)a * K + m) * K + b : ((size_t)a * K + b) * K + m;
          Tr[o] = sr;
          Ti[o] = si;
        }
    memcpy(Fr, Tr, sizeof(double) * KK);
    memcpy(Fi, Ti, sizeof(double) * KK);
  }
  /* 4. multiply by W(m) */
  double vol = box * box * box;
  for (int m1 = 0; m1 < K; ++m1)
    for (int m2 = 0; m2 < K; ++m2)
      for (int m3 = 0; m3 < K; ++m3) {
        size_t idx = ((size_t)m1 * K + m2) * K + m3;
        int s1 = m1 <= K / 2 ? m1 : m1 - K, s2 = m2 <= K / 2 ? m2 : m2 - K,
            s3 = m3 <= K / 2 ? m3 : m3 - K;
        double W = 0.0;
        if (s1 || s2 || s3) {
          double k[3] = {twopi * s1 / box, twopi * s2 / box, twopi * s3 / box};
          double k2 = or_dot(k, k);
          W = 4.0 * M_PI / k2 * exp(-k2 / (4.0 * beta * beta)) /
              (vol * or_spline_mod(p, K, m1) * or_spline_mod(p, K, m2) * or_spline_mod(p, K, m3));
        }
        Fr[idx] *= W;
        Fi[idx] *= W;
      }
  /* 5. phi(g) = sum_m W F(m) exp(-2 pi i m.g/K) */
  for (int axis = 0; axis < 3; ++axis) {
    for (int a = 0; a < K; ++a)
      for (int b = 0; b < K; ++b)
        for (int g = 0; g < K; ++g) {
          double sr = 0.0, si = 0.0;
          for (int m = 0; m < K; ++m) {
            size_t idx = axis == 0 ? ((size_t)m * K + a) * K + b
                       : axis == 1 ? ((size_t)a * K + m) * K + b : ((size_t)a * K + b) * K + m;
            sr += Fr[idx] * cs[m * K + g] + Fi[idx] * sn[m * K + g];
            si += Fi[idx] * cs[m * K + g] - Fr[idx] * sn[m * K + g];
          }
          size_t o = axis == 0 ? ((size_t)g * K + a) * K + b
                   : axis == 1 ? ((size_t)a * K + g) * K + b : ((size_t)a * K + b) * K + g;
          Tr[o] = sr;
          Ti[o] = si;
        }
    memcpy(Fr, Tr, sizeof(double) * KK);
    memcpy(Fi, Ti, sizeof(double) * KK);
  }
  for (size_t k = 0; k < KK; ++k) phi[k] = Fr[k];
  /* 6. interpolate derivatives up to third order; energy, forces, field */
  double esum = 0.0;
  for (int j = 0; j < n; ++j) {
    double D[4][4][4];
    for (int dx = 0; dx < 4; ++dx)
      for (int dy = 0; dy < 4; ++dy)
        for (int dz = 0; dz < 4; ++dz) D[dx][dy][dz] = 0.0;
    for (int t1 = 0; t1 < p; ++t1)
      for (int t2 = 0; t2 < p; ++t2)
        for (int t3 = 0; t3 < p; ++t3) {
          double ph = phi[((size_t)GIX(j, 0, t1) * K + GIX(j, 1, t2)) * K + GIX(j, 2, t3)];
          for (int dx = 0; dx < 4; ++dx)
            for (int dy = 0; dy < 4 - dx; ++dy)
              for (int dz = 0; dz < 4 - dx - dy; ++dz)
                D[dx][dy][dz] += ph * TH(j, 0, t1, dx) * TH(j, 1, t2, dy) * TH(j, 2, t3, dz);
        }
    double q, u[3], T[3][3];
    or_unpack(mpole + 10 * j, &q, u, T);
    /* derivative along axes (a, b, c): orders counted per axis */
#define DER1(a) D[(a) == 0][(a) == 1][(a) == 2]
#define DER2(a, b) D[((a) == 0) + ((b) == 0)][((a) == 1) + ((b) == 1)][((a) == 2) + ((b) == 2)]
#define DER3(a, b, c) D[((a) == 0) + ((b) == 0) + ((c) == 0)][((a) == 1) + ((b) == 1) + ((c) == 1)] \
                       [((a) == 2) + ((b) == 2) + ((c) == 2)]
    double e = q * D[0][0][0];
    for (int a = 0; a < 3; ++a) {
      e += u[a] * DER1(a);
      for (int b = 0; b < 3; ++b) e += T[a][b] * DER2(a, b);
    }
    esum += e;
    for (int a = 0; a < 3; ++a) {
      double g = q * DER1(a);
      for (int b = 0; b < 3; ++b) {
        g += u[b] * DER2(a, b);
        for (int c = 0; c < 3; ++c) g += T[b][c] * DER3(a, b, c);
      }
      force[3 * j + a] = -OR_COULOMB * g;
      if (field) field[3 * j + a] = -DER1(a);
    }
#undef DER1
#undef DER2
#undef DER3
  }
  *energy = 0.5 * OR_COULOMB * esum;
#undef TH
#undef GIX
  free(Q); free(Fr); free(Fi); free(Tr); free(Ti); free(phi); free(cs); free(sn); free(th);
  free(g0);
  return OR_OK;
}

/* ------------------------------------------------------------------------ */
/* Local-frame multipoles (the rotation and torque steps that section
 * "Hotspots" lists beside the multipole routines).  Reading (the paper gives
 * no frame definitions): the AMOEBA frames, with d_k = r_katom - r_i and
 * u_k = d_k/|d_k| for the z-, x- and y-atoms (minimum image).  Every type
 * takes z as below and a vector a, then x = unit(a - (a.z) z):
 *   type 0 (none):        R = I;
 *   type 1 (Z-then-X):    z = u_z,                 a = d_x;
 *   type 2 (bisector):    z = unit(u_z + u_x),     a = u_x;
 *   type 3 (Z-only):      z = u_z,                 a = the global x axis, or the
 *                         global y axis when |z_x| > 0.866 (z within 30 degrees
 *                         of +-x);
 *   type 4 (Z-bisector):  z = u_z,                 a = u_x + u_y;
 *   type 5 (3-fold):      z = unit(u_z + u_x + u_y), a = u_x;
 * y = z cross x.  With R = [x y z] (columns), the lab-frame multipoles are
 *   q = q_loc, mu = R mu_loc, Theta = R Theta_loc R^T.
 * Values are carried with their derivatives with respect to the twelve
 * coordinates of (r_i, r_zatom, r_xatom, r_yatom) (forward-mode dual
 * numbers), so the rotated multipoles come with their exact Jacobian. */
#define OR_ND 12
typedef struct {
  double v, d[OR_ND];
} or_dual;

static or_dual od_const(double v) {
  or_dual r;
  r.v = v;
  for (int k = 0; k < OR_ND; ++k) r.d[k] = 0.0;
  return r;
}
static or_dual od_add(or_dual a, or_dual b) {
  or_dual r;
  r.v = a.v + b.v;
  for (int k = 0; k < OR_ND; ++k) r.d[k] = a.d[k] + b.d[k];
  return r;
}
static or_dual od_sub(or_dual a, or_dual b) {
  or_dual r;
  r.v = a.v - b.v;
  for (int k = 0; k < OR_ND; ++k) r.d[k] = a.d[k] - b.d[k];
  return r;
}
static or_dual od_mul(or_dual a, or_dual b) {
  or_dual r;
  r.v = a.v * b.v;
  for (int k = 0; k < OR_ND; ++k) r.d[k] = a.d[k] * b.v + a.v * b.d[k];
  return r;
}
static or_dual od_div(or_dual a, or_dual b) {
  or_dual r;
  r.v = a.v / b.v;
  for (int k = 0; k < OR_ND; ++k) r.d[k] = (a.d[k] * b.v - a.v * b.d[k]) / (b.v * b.v);
  return r;
}
static or_dual od_sqrt(or_dual a) {
  or_dual r;
  r.v = sqrt(a.v);
  for (int k = 0; k < OR_ND; ++k) r.d[k] = a.d[k] / (2.0 * r.v);
  return r;
}
static or_dual od_dot3(const or_dual* a, const or_dual* b) {
  return od_add(od_add(od_mul(a[0], b[0]), od_mul(a[1], b[1])), od_mul(a[2], b[2]));
}
static void od_unit3(const or_dual* a, or_dual* out) {
  or_dual nrm = od_sqrt(od_dot3(a, a));
  for (int c = 0; c < 3; ++c) out[c] = od_div(a[c], nrm);
}

/* d_k = r_katom - r_i (minimum image) as duals; slot s (1 z, 2 x, 3 y) of the partials. */
static void or_frame_vec(const double* xyz, double box, int i, int k, int slot, or_dual* d) {
  for (int c = 0; c < 3; ++c) {
    double t = xyz[3 * k + c] - xyz[3 * i + c];
    d[c] = od_const(t - box * rint(t / box));
    d[c].d[c] = -1.0;              /* d/dr_i */
    d[c].d[3 * slot + c] = 1.0;    /* d/dr_katom */
  }
}

/* Frame vectors of site i (as duals over r_i, r_zatom, r_xatom, r_yatom). */
static void or_frame_axes(const double* xyz, double box, int i, int type, int iz, int ix,
                          int iy, or_dual ax[3][3]) {
  for (int a = 0; a < 3; ++a)
    for (int b = 0; b < 3; ++b) ax[a][b] = od_const(a == b ? 1.0 : 0.0);
  if (type == 0) return;
  or_dual dz[3], uz[3], dx[3], ux[3], dy[3], uy[3], z[3], a[3], x[3];
  or_frame_vec(xyz, box, i, iz, 1, dz);
  od_unit3(dz, uz);
  if (type != 3) {
    or_frame_vec(xyz, box, i, ix, 2, dx);
    od_unit3(dx, ux);
  }
  if (type == 4 || type == 5) {
    or_frame_vec(xyz, box, i, iy, 3, dy);
    od_unit3(dy, uy);
  }
  if (type == 2) {
    or_dual s[3];
    for (int c = 0; c < 3; ++c) s[c] = od_add(uz[c], ux[c]);
    od_unit3(s, z);
  } else if (type == 5) {
    or_dual s[3];
    for (int c = 0; c < 3; ++c) s[c] = od_add(od_add(uz[c], ux[c]), uy[c]);
    od_unit3(s, z);
  } else {
    for (int c = 0; c < 3; ++c) z[c] = uz[c];
  }
  for (int c = 0; c < 3; ++c) {
    if (type == 1) a[c] = dx[c];
    else if (type == 3) {
      int near_x = fabs(z[0].v) > 0.866;
      a[c] = od_const(c == (near_x ? 1 : 0) ? 1.0 : 0.0);
    } else if (type == 4) a[c] = od_add(ux[c], uy[c]);
    else a[c] = ux[c];
  }
  or_dual p = od_dot3(a, z), w[3];
  for (int c = 0; c < 3; ++c) w[c] = od_sub(a[c], od_mul(p, z[c]));
  od_unit3(w, x);
  or_dual y[3];
  y[0] = od_sub(od_mul(z[1], x[2]), od_mul(z[2], x[1]));
  y[1] = od_sub(od_mul(z[2], x[0]), od_mul(z[0], x[2]));
  y[2] = od_sub(od_mul(z[0], x[1]), od_mul(z[1], x[0]));
  for (int c = 0; c < 3; ++c) {   /* columns x, y, z */
    ax[c][0] = x[c];
    ax[c][1] = y[c];
    ax[c][2] = z[c];
  }
}

/* Lab-frame multipoles of site i as duals (10 components, stored layout). */
static void or_rotate_site(const double* xyz, double box, int i, int type, const int32_t* fa,
                           const double* loc, or_dual out[10]) {
  or_dual R[3][3];
  or_frame_axes(xyz, box, i, type, fa[0], fa[1], fa[2], R);
  double tl[3][3];
  tl[0][0] = loc[4]; tl[0][1] = tl[1][0] = loc[5]; tl[0][2] = tl[2][0] = loc[6];
  tl[1][1] = loc[7]; tl[1][2] = tl[2][1] = loc[8]; tl[2][2] = loc[9];
  out[0] = od_const(loc[0]);
  for (int a = 0; a < 3; ++a) {
    or_dual s = od_const(0.0);
    for (int b = 0; b < 3; ++b) s = od_add(s, od_mul(R[a][b], od_const(loc[1 + b])));
    out[1 + a] = s;
  }
  const int ia[6] = {0, 0, 0, 1, 1, 2}, ib[6] = {0, 1, 2, 1, 2, 2};
  for (int k = 0; k < 6; ++k) {
    or_dual s = od_const(0.0);
    for (int c = 0; c < 3; ++c)
      for (int d = 0; d < 3; ++d)
        s = od_add(s, od_mul(od_mul(R[ia[k]][c], od_const(tl[c][d])), R[ib[k]][d]));
    out[4 + k] = s;
  }
}

/* Frame atoms per type: z (types 1-5), x (1, 2, 4, 5), y (4, 5); each in
 * [0, n), none the site itself, all distinct. */
static int or_frame_natoms(int t) { return t == 0 ? 0 : t == 3 ? 1 : t <= 2 ? 2 : 3; }

static int or_frames_args(int n, const int32_t* ftype, const int32_t* fatoms) {
  for (int i = 0; i < n; ++i) {
    int t = ftype[i];
    if (t < 0 || t > 5) return OR_E_ARG;
    int m = or_frame_natoms(t);
    for (int k = 0; k < m; ++k) {
      int a = fatoms[3 * i + k];
      if (a < 0 || a >= n || a == i) return OR_E_ARG;
      for (int l = 0; l < k; ++l)
        if (fatoms[3 * i + l] == a) return OR_E_ARG;
    }
  }
  return OR_OK;
}

/* force_k -= sum over sites i with k in their frame of sum_c G_i,c dM_i,c/dx_k.
 * virial (nullable): M_i depends on positions only through the frame vectors
 * d_k = r_katom - r_i, and dM/dd_k = dM/dr_katom, so the frame part of
 * W_ab = sum over relative vectors v of v_a dE/dv_b is
 * sum_i sum_k d_k,a (sum_c G_i,c dM_i,c/dr_katom,b). */
static void or_frames_chain(int n, const double* xyz, double box, const int32_t* ftype,
                            const int32_t* fatoms, const or_dual* M, const double* G,
                            double* force, double* virial) {
  for (int i = 0; i < n; ++i) {
    if (ftype[i] == 0) continue;
    int m = or_frame_natoms(ftype[i]);
    int who[4] = {i, fatoms[3 * i], fatoms[3 * i + 1], fatoms[3 * i + 2]};
    for (int s = 0; s <= m; ++s) {
      double g[3];
      for (int a = 0; a < 3; ++a) {
        g[a] = 0.0;
        for (int c = 0; c < 10; ++c) g[a] += G[10 * i + c] * M[10 * i + c].d[3 * s + a];
        force[3 * who[s] + a] -= g[a];
      }
      if (virial && s > 0) {
        double d[3], r2;
        or_image(xyz + 3 * i, xyz + 3 * who[s], box, d, &r2);
        for (int a = 0; a < 3; ++a)
          for (int b = 0; b < 3; ++b) virial[3 * a + b] += d[a] * g[b];
      }
    }
  }
}

int or_rotate_mpole(int n, const double* xyz, double box, const int32_t* ftype,
                    const int32_t* fatoms, const double* local, double* global) {
  if (n < 0 || !(box > 0.0)) return OR_E_ARG;
  int st = or_frames_args(n, ftype, fatoms);
  if (st) return st;
  for (int i = 0; i < n; ++i) {
    or_dual m[10];
    or_rotate_site(xyz, box, i, ftype[i], fatoms + 3 * i, local + 10 * i, m);
    for (int k = 0; k < 10; ++k) global[10 * i + k] = m[k].v;
  }
  return OR_OK;
}

/* Permanent-multipole real-space energy and forces with local frames.  The
 * energy is that of or_empole_real at the rotated multipoles M(x).  Its
 * gradient has the direct part (or_empole_real's forces at fixed M) and the
 * frame part: with G_i,c = dE/dM_i,c, which is the pair energy with a unit
 * multipole in component c of site i (E is linear in each site's
 * multipoles), the force on atom k gains -sum_i sum_c G_i,c dM_i,c/dx_k over
 * the sites i whose frame contains k.  energy[3] as or_empole_real; virial
 * (nullable) [9]: or_empole_real's pair virial at M plus the frame part. */
int or_empole_frames(int n, const double* xyz, double box, const int32_t* molid,
                     const int32_t* row_ptr, const int32_t* col, const int32_t* ftype,
                     const int32_t* fatoms, const double* local, double beta, double rc,
                     double* energy, double* force, double* virial) {
  int st = or_pair_args(n, box, rc);
  if (st) return st;
  if ((st = or_frames_args(n, ftype, fatoms))) return st;
  size_t nn = (size_t)(n > 0 ? n : 1);
  or_dual* M = (or_dual*)malloc(sizeof(or_dual) * 10 * nn);
  double* Mg = (double*)calloc(10 * nn, sizeof(double));
  double* G = (double*)calloc(10 * nn, sizeof(double));
  double vir[9];
  for (int i = 0; i < n; ++i) {
    or_rotate_site(xyz, box, i, ftype[i], fatoms + 3 * i, local + 10 * i,
                   M + 10 * i);
    for (int k = 0; k < 10; ++k) Mg[10 * i + k] = M[10 * i + k].v;
  }
  or_empole_real(n, xyz, box, molid, row_ptr, col, Mg, beta, rc, energy, force, vir);
  double rc2 = rc * rc;
  for (int i = 0; i < n; ++i)
    for (int p = row_ptr[i]; p < row_ptr[i + 1]; ++p) {
      int j = col[p];
      double d[3], r2;
      or_image(xyz + 3 * i, xyz + 3 * j, box, d, &r2);
      if (!(r2 <= rc2)) continue;
      double r = sqrt(r2), B[6], R[6], g[6];
      or_radial(r, beta, 5, B, R);
      int excl = molid[i] == molid[j];
      for (int k = 0; k <= 5; ++k) g[k] = excl ? B[k] - R[k] : B[k];
      for (int c = 0; c < 10; ++c) {
        double unit[10] = {0.0}, e, de[3];
        unit[c] = 1.0;
        or_mpole_pair(d, unit, Mg + 10 * j, g, &e, de);
        G[10 * i + c] += e;
        or_mpole_pair(d, Mg + 10 * i, unit, g, &e, de);
        G[10 * j + c] += e;
      }
    }
  or_frames_chain(n, xyz, box, ftype, fatoms, M, G, force, virial ? vir : NULL);
  if (virial)
    for (int k = 0; k < 9; ++k) virial[k] = vir[k];
  free(M);
  free(Mg);
  free(G);
  return OR_OK;
}

/* Polarization energy at fixed induced dipoles with local-frame multipoles:
 * the pair energies of or_epolar_real at the rotated multipoles M(x), and
 * their full gradient.  Only the induced-permanent energy depends on M; its
 * G_i,c is the pair energy U(unit_c at i, mu_j; gp) over the partners j
 * (and U(mu_i, unit_c at j; gp) from the other side), gp the damped family
 * of or_epolar_real.  energy[3] as or_epolar_real; virial (nullable) [9]:
 * or_epolar_real's pair virial at M plus the frame part. */
int or_epolar_frames(int n, const double* xyz, double box, const int32_t* molid,
                     const int32_t* row_ptr, const int32_t* col, const int32_t* ftype,
                     const int32_t* fatoms, const double* local, const double* polarity,
                     const double* thole, const double* mu, double beta, double rc,
                     double* energy, double* force, double* virial) {
  int st = or_pair_args(n, box, rc);
  if (st) return st;
  if ((st = or_frames_args(n, ftype, fatoms))) return st;
  size_t nn = (size_t)(n > 0 ? n : 1);
  or_dual* M = (or_dual*)malloc(sizeof(or_dual) * 10 * nn);
  double* Mg = (double*)calloc(10 * nn, sizeof(double));
  double* G = (double*)calloc(10 * nn, sizeof(double));
  double vir[9];
  for (int i = 0; i < n; ++i) {
    or_rotate_site(xyz, box, i, ftype[i], fatoms + 3 * i, local + 10 * i,
                   M + 10 * i);
    for (int k = 0; k < 10; ++k) Mg[10 * i + k] = M[10 * i + k].v;
  }
  or_epolar_real(n, xyz, box, molid, row_ptr, col, Mg, polarity, thole, mu, beta, rc, energy,
                 force, vir);
  double rc2 = rc * rc;
  for (int i = 0; i < n; ++i)
    for (int p = row_ptr[i]; p < row_ptr[i + 1]; ++p) {
      int j = col[p];
      double d[3], r2;
      or_image(xyz + 3 * i, xyz + 3 * j, box, d, &r2);
      if (!(r2 <= rc2)) continue;
      double r = sqrt(r2), B[6], R[6], l[5], gp[6] = {0.0};
      or_radial(r, beta, 5, B, R);
      or_thole(r, polarity[i], polarity[j], thole[i], thole[j], &l[1], &l[2], &l[3]);
      l[4] = or_thole_l9(r, polarity[i], polarity[j], thole[i], thole[j]);
      double s = molid[i] == molid[j] ? 0.0 : 1.0;
      for (int k = 1; k <= 4; ++k) gp[k] = B[k] - (1.0 - s * l[k]) * R[k];
      double ind_i[10] = {0.0}, ind_j[10] = {0.0};
      for (int a = 0; a < 3; ++a) {
        ind_i[1 + a] = mu[3 * i + a];
        ind_j[1 + a] = mu[3 * j + a];
      }
      for (int c = 0; c < 10; ++c) {
        double unit[10] = {0.0}, e, de[3];
        unit[c] = 1.0;
        or_mpole_pair(d, unit, ind_j, gp, &e, de);
        G[10 * i + c] += e;
        or_mpole_pair(d, ind_i, unit, gp, &e, de);
        G[10 * j + c] += e;
      }
    }
  or_frames_chain(n, xyz, box, ftype, fatoms, M, G, force, virial ? vir : NULL);
  if (virial)
    for (int k = 0; k < 9; ++k) virial[k] = vir[k];
  free(M);
  free(Mg);
  free(G);
  return OR_OK;
}

/* ------------------------------------------------------------------------ */
/* vdW hydrogen reduction (the "vdW hydrogen reduction" of AMOEBA's Halgren
 * term).  Reading: a site with parent p >= 0 sits at r_p + red_i (r_i - r_p)
 * (minimum image of r_i - r_p); other sites at their atoms.  Site forces go
 * back by the chain rule: atom i receives red_i f_i, its parent
 * (1 - red_i) f_i. */
int or_vdw_sites(int n, const double* xyz, double box, const int32_t* parent, const double* red,
                 double* sites) {
  if (n < 0 || !(box > 0.0)) return OR_E_ARG;
  for (int i = 0; i < n; ++i) {
    int p = parent[i];
    if (p >= n || p == i) return OR_E_ARG;
    for (int a = 0; a < 3; ++a) {
      if (p < 0) {
        sites[3 * i + a] = xyz[3 * i + a];
      } else {
        double d = xyz[3 * i + a] - xyz[3 * p + a];
        d -= box * rint(d / box);
        sites[3 * i + a] = xyz[3 * p + a] + red[i] * d;
      }
    }
  }
  return OR_OK;
}

int or_vdw_forces_to_atoms(int n, const int32_t* parent, const double* red, const double* fsite,
                           double* fatom) {
  for (int i = 0; i < n; ++i)
    if (parent[i] >= n || parent[i] == i) return OR_E_ARG;
  for (int k = 0; k < 3 * n; ++k) fatom[k] = 0.0;
  for (int i = 0; i < n; ++i) {
    int p = parent[i];
    for (int a = 0; a < 3; ++a) {
      if (p < 0) {
        fatom[3 * i + a] += fsite[3 * i + a];
      } else {
        fatom[3 * i + a] += red[i] * fsite[3 * i + a];
        fatom[3 * p + a] += (1.0 - red[i]) * fsite[3 * i + a];
      }
    }
  }
  return OR_OK;
}

/* ------------------------------------------------------------------------ */
/* Truncated conjugate gradient, one step (TCG1; the fixed-cost polarization
 * solvers that the paper's later versions use).  Reading: diagonal
 * preconditioner alpha, direct guess, no "peek" step:
 *   mu0 = alpha E,  r0 = E - A mu0,  p0 = alpha r0,
 *   gamma = r0.p0,  delta = p0.A p0,  a = gamma/delta,  mu1 = mu0 + a p0,
 *   U = -1/2 C mu1.E,
 * with E the permanent field and A the operator of or_tmatvec (rows of
 * alpha = 0 zero).  U is not variational in mu, so its force is the total
 * derivative through every step.  Writing s = p0.E,
 *   w = 2 p0/delta - 2 gamma alpha A p0/delta^2,  v = s w + a mu0,
 *   u = mu0 + mu1 + v - alpha A v,
 * the gradient is  dU = -1/2 C [u.dE + v.dT mu0 + s gamma/delta^2 p0.dT p0]
 * (dA = -dT), i.e. the force is
 *   F = 1/2 F_ip(u) + 1/2 F_bil(v, mu0) + 1/2 s gamma/delta^2 F_bil(p0, p0),
 * where, from the pair forces F(mu) of or_epolar_real at dipoles mu,
 *   F_ip(u) = [F(u) - F(-u)]/2           (the part linear in the dipoles)
 *   F_ii(w) = [F(w) + F(-w)]/2           (the part quadratic in them)
 *   F_bil(b, c) = F_ii(b + c) - F_ii(b) - F_ii(c). */
static double or_dot3n(int n, const double* a, const double* b) {
  double s = 0.0;
  for (int k = 0; k < 3 * n; ++k) s += a[k] * b[k];
  return s;
}

static void or_epolar_parts(int n, const double* xyz, double box, const int32_t* molid,
                            const int32_t* row_ptr, const int32_t* col, const double* mpole,
                            const double* polarity, const double* thole, double beta, double rc,
                            const double* mu, double* Fplus, double* Fminus) {
  size_t m = 3 * (size_t)(n > 0 ? n : 1);
  double* neg = (double*)malloc(sizeof(double) * m);
  double e[3], w[9];
  for (int k = 0; k < 3 * n; ++k) neg[k] = -mu[k];
  or_epolar_real(n, xyz, box, molid, row_ptr, col, mpole, polarity, thole, mu, beta, rc, e, Fplus,
                 w);
  or_epolar_real(n, xyz, box, molid, row_ptr, col, mpole, polarity, thole, neg, beta, rc, e,
                 Fminus, w);
  free(neg);
}

int or_polarize_tcg1(int n, const double* xyz, double box, const int32_t* molid,
                     const int32_t* row_ptr, const int32_t* col, const double* mpole,
                     const double* polarity, const double* thole, double beta, double rc,
                     double* mu_out, double* epol, double* force) {
  int st = or_pair_args(n, box, rc);
  if (st) return st;
  for (int i = 0; i < n; ++i)
    if (!(polarity[i] >= 0.0)) return OR_E_ARG;
  size_t m = 3 * (size_t)(n > 0 ? n : 1);
  double *E = (double*)malloc(sizeof(double) * m), *mu0 = (double*)malloc(sizeof(double) * m),
         *r0 = (double*)malloc(sizeof(double) * m), *p0 = (double*)malloc(sizeof(double) * m),
         *P = (double*)malloc(sizeof(double) * m), *q = (double*)malloc(sizeof(double) * m);
  or_efield_direct(n, xyz, box, molid, row_ptr, col, mpole, polarity, thole, beta, rc, E);
  for (int i = 0; i < n; ++i)
    for (int a = 0; a < 3; ++a) mu0[3 * i + a] = polarity[i] * E[3 * i + a];
  or_tmatvec(n, xyz, box, row_ptr, col, polarity, thole, beta, rc, 1, mu0, q);
  for (int i = 0; i < n; ++i)
    for (int a = 0; a < 3; ++a) {
      int k = 3 * i + a;
      r0[k] = polarity[i] > 0.0 ? E[k] - q[k] : 0.0;
      p0[k] = polarity[i] * r0[k];
    }
  or_tmatvec(n, xyz, box, row_ptr, col, polarity, thole, beta, rc, 1, p0, P);
  double gamma = or_dot3n(n, r0, p0), delta = or_dot3n(n, p0, P);
  double a = delta != 0.0 ? gamma / delta : 0.0;
  for (int k = 0; k < 3 * n; ++k) mu_out[k] = mu0[k] + a * p0[k];
  *epol = -0.5 * OR_COULOMB * or_dot3n(n, mu_out, E);
  if (force) {
    double s = or_dot3n(n, p0, E);
    double *v = (double*)malloc(sizeof(double) * m), *u = (double*)malloc(sizeof(double) * m),
           *Av = (double*)malloc(sizeof(double) * m), *t = (double*)malloc(sizeof(double) * m),
           *Fp = (double*)malloc(sizeof(double) * m), *Fm = (double*)malloc(sizeof(double) * m);
    for (int i = 0; i < n; ++i)
      for (int c = 0; c < 3; ++c) {
        int k = 3 * i + c;
        double w = delta != 0.0 ? 2.0 * p0[k] / delta - 2.0 * gamma * polarity[i] * P[k] /
                                                            (delta * delta)
                                : 0.0;
        v[k] = s * w + a * mu0[k];
      }
    or_tmatvec(n, xyz, box, row_ptr, col, polarity, thole, beta, rc, 1, v, Av);
    for (int i = 0; i < n; ++i)
      for (int c = 0; c < 3; ++c) {
        int k = 3 * i + c;
        u[k] = mu0[k] + mu_out[k] + v[k] - polarity[i] * Av[k];
      }
    double cb = delta != 0.0 ? s * gamma / (delta * delta) : 0.0;
    for (int k = 0; k < 3 * n; ++k) force[k] = 0.0;
    /* 1/2 F_ip(u) = 1/4 [F(u) - F(-u)] */
    or_epolar_parts(n, xyz, box, molid, row_ptr, col, mpole, polarity, thole, beta, rc, u, Fp, Fm);
    for (int k = 0; k < 3 * n; ++k) force[k] += 0.25 * (Fp[k] - Fm[k]);
    /* 1/2 F_bil(v, mu0) = 1/2 [F_ii(v + mu0) - F_ii(v) - F_ii(mu0)] */
    for (int k = 0; k < 3 * n; ++k) t[k] = v[k] + mu0[k];
    or_epolar_parts(n, xyz, box, molid, row_ptr, col, mpole, polarity, thole, beta, rc, t, Fp, Fm);
    for (int k = 0; k < 3 * n; ++k) force[k] += 0.25 * (Fp[k] + Fm[k]);
    or_epolar_parts(n, xyz, box, molid, row_ptr, col, mpole, polarity, thole, beta, rc, v, Fp, Fm);
    for (int k = 0; k < 3 * n; ++k) force[k] -= 0.25 * (Fp[k] + Fm[k]);
    or_epolar_parts(n, xyz, box, molid, row_ptr, col, mpole, polarity, thole, beta, rc, mu0, Fp,
                    Fm);
    for (int k = 0; k < 3 * n; ++k) force[k] -= 0.25 * (Fp[k] + Fm[k]);
    /* 1/2 cb F_bil(p0, p0) = cb F_ii(p0) = cb/2 [F(p0) + F(-p0)] */
    or_epolar_parts(n, xyz, box, molid, row_ptr, col, mpole, polarity, thole, beta, rc, p0, Fp,
                    Fm);
    for (int k = 0; k < 3 * n; ++k) force[k] += 0.5 * cb * (Fp[k] + Fm[k]);
    free(v); free(u); free(Av); free(t); free(Fp); free(Fm);
  }
  free(E); free(mu0); free(r0); free(p0); free(P); free(q);
  return OR_OK;
}
