// Reciprocal-space multipole energy, forces and field by smooth particle-mesh
// Ewald (the reciprocal multipole routine named beside the real-space one in
// section "Hotspots"; the paper leaves it unvectorized).  Textbook smooth PME
// with cardinal B-splines of order P, extended to dipoles and quadrupoles by
// differentiating the spline.
//
// One call: bin sites by x -> spread by mesh tiles -> FFT along z, y -> [FFT along x, multiply by the
// influence function, inverse FFT along x] -> inverse FFT along y, z ->
// gather (potential derivatives up to third order at every site) -> energy.
//
// The spread grid is accumulated in 64-bit fixed point (2^-40 units) with
// LDS integer atomics: integer addition is associative, so the grid, and
// every result after it, is bitwise the same run to run.  A single contribution of
// magnitude 2^17 or more is refused (the energy comes back NaN); below that
// the sums of up to 2^6 such contributions at one point stay exact.
//
// The FFTs are radix-2 in LDS, one workgroup per batch of grid lines: lines of
// length K (a power of two, 16..128) along one axis, 256 threads, K/2
// butterflies per line and stage.  Forward transforms take bit-reversed input
// (decimation in time), inverse ones natural input (decimation in frequency),
// so no transform needs a separate permutation pass.
#include <cmath>

#include "tk_internal.hpp"

namespace tk {

namespace {

constexpr double kPi = 3.14159265358979323846;
constexpr double kFix = 1099511627776.0;   // 2^40
constexpr double kFixMax = 131072.0;       // 2^17

// The sites of a PME call: caller-order multipoles ([n][3] coordinates,
// [n][10] multipoles), or dipoles in a solver's sorted order (coordinates as
// SoA rows with a stride, [n][3] dipoles; charges and quadrupoles zero at
// compile time).
struct SrcMpole {
  const double* xyz;
  const double* mpole;
  __device__ void pos(int j, double x[3]) const {
#pragma unroll
    for (int a = 0; a < 3; ++a) x[a] = xyz[3 * j + a];
  }
  __device__ void mp(int j, double m[10]) const {
#pragma unroll
    for (int k = 0; k < 10; ++k) m[k] = mpole[10 * j + k];
  }
};

struct SrcDipole {
  const double* p;   // p[a * ps + j]
  long ps;
  const double* v;   // v[3 j + a]
  __device__ void pos(int j, double x[3]) const {
#pragma unroll
    for (int a = 0; a < 3; ++a) x[a] = p[a * ps + j];
  }
  __device__ void mp(int j, double m[10]) const {
#pragma unroll
    for (int k = 0; k < 10; ++k) m[k] = 0.0;
#pragma unroll
    for (int a = 0; a < 3; ++a) m[1 + a] = v[3 * j + a];
  }
};

// Launches queued ahead by the iterative solver read its state: with done
// set, a launch returns at once while *done != 0 (when = 0: the solve has
// stopped) or while *done == 0 (when = 1: work for the stopped solve only).
// done2 (two packed right-hand sides): open while either side is open
struct Gate {
  const int32_t* done = nullptr;
  int when = 0;
  const int32_t* done2 = nullptr;
  __device__ bool closed() const {
    if (!done) return false;
    const bool c1 = when ? *done == 0 : *done != 0;
    if (!done2) return c1;
    return c1 && (when ? *done2 == 0 : *done2 != 0);
  }
};

// Cardinal B-spline weights th[t][d] = M_P^(d)(w + t) (t = 0..P-1, d = 0..3)
// for a fractional offset w in [0, 1), by the recursion
//   M_k(x) = [x M_(k-1)(x) + (k - x) M_(k-1)(x - 1)] / (k - 1),  M_2 on (0, 2),
// and the derivatives as differences of lower orders,
//   M_P'(x) = M_(P-1)(x) - M_(P-1)(x - 1).
template <int P>
__device__ __forceinline__ void bspline_table(double w, double th[P][4]) {
  double A[P + 1][P];   // A[k][t] = M_k(w + t), zero outside t < k
#pragma unroll
  for (int k = 0; k <= P; ++k)
#pragma unroll
    for (int t = 0; t < P; ++t) A[k][t] = 0.0;
  A[2][0] = w;
  A[2][1] = 1.0 - w;
#pragma unroll
  for (int k = 3; k <= P; ++k)
#pragma unroll
    for (int t = 0; t < k; ++t) {
      const double x = w + t;
      const double lo = t < k - 1 ? A[k - 1][t] : 0.0;
      const double hi = t > 0 ? A[k - 1][t - 1] : 0.0;
      A[k][t] = (x * lo + (k - x) * hi) * (1.0 / (k - 1));
    }
#pragma unroll
  for (int t = 0; t < P; ++t) {
    auto at = [&](int k, int s) { return s >= 0 ? A[k][s] : 0.0; };
    th[t][0] = A[P][t];
    th[t][1] = at(P - 1, t) - at(P - 1, t - 1);
    th[t][2] = at(P - 2, t) - 2.0 * at(P - 2, t - 1) + at(P - 2, t - 2);
    th[t][3] = at(P - 3, t) - 3.0 * at(P - 3, t - 1) + 3.0 * at(P - 3, t - 2) - at(P - 3, t - 3);
  }
}

// Per axis: grid origin i0 = floor(u), weights scaled to d/dx = (K/L) d/du.
// Axes y and z keep all P rows; along x only row t1 (the lane's plane) is
// kept, selected by an unrolled compare so that every table stays in
// registers.
template <int P>
__device__ __forceinline__ void site_splines(const double* x, double box, int K, int t1,
                                             double X[4], double th[2][P][4], int i0[3]) {
  const double kl = K / box;
  const double sc[4] = {1.0, kl, kl * kl, kl * kl * kl};
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    const double s = x[a] / box;
    const double u = K * (s - floor(s));
    const double fl = floor(u);
    i0[a] = fl >= 0.0 && fl <= K ? (int)fl : 0;   // NaN: any in-range index (weights NaN)
    double t4[P][4];
    bspline_table<P>(u - fl, t4);
    if (a == 0) {
#pragma unroll
      for (int d = 0; d < 4; ++d) X[d] = 0.0;
#pragma unroll
      for (int t = 0; t < P; ++t)
        if (t == t1)
#pragma unroll
          for (int d = 0; d < 4; ++d) X[d] = t4[t][d] * sc[d];
    } else {
#pragma unroll
      for (int t = 0; t < P; ++t)
#pragma unroll
        for (int d = 0; d < 4; ++d) th[a - 1][t][d] = t4[t][d] * sc[d];
    }
  }
}

__device__ __forceinline__ int wrap(int g, int K) { return ((g % K) + K) % K; }

// The spread is owned by mesh tiles: sites are binned by their x grid index
// (a counting sort; the order inside a bin does not matter, integer sums being
// exact), and one workgroup per tile (a whole x-plane; half a plane at
// K = 128, to fit the LDS) adds, in LDS,
// the contributions of the sites whose x-row reaches its plane (bins gx..gx+P-1),
// then stores the tile.  No global atomics, and every mesh point is written
// once, so the mesh needs no clearing.
// One workgroup per spread tile: 1024 threads, 512 for orders 7 and 8 (their
// larger spline tables need more than the 128 registers of a 1024-thread
// workgroup).
template <int P>
constexpr int spread_threads() { return P <= 6 ? 1024 : 512; }

// The x grid index of the spline code, mod K (a fraction that rounds up to
// 1 gives K, i.e. 0).  A non-finite coordinate maps to bin 0: its weights are
// NaN, which the spread refuses (the energy comes back NaN).
__device__ __forceinline__ int xbin(const double* x, double box, int K) {
  const double s = x[0] / box;
  const double f = floor(K * (s - floor(s)));
  return f >= 0.0 && f < K ? (int)f : 0;
}

// Counting sort by x-bin without global atomics: each block of 256 sites
// counts its bins in LDS (slot = rank inside its block and bin) and stores its
// counts; block 0 also clears the refusal flag.
template <class Src>
__global__ __launch_bounds__(256) void k_pme_bin(int n, Src src, double box, int K,
                                                 int* __restrict__ bcnt, int* __restrict__ bin,
                                                 int* __restrict__ slot, int* __restrict__ flag,
                                                 Gate gate) {
  if (gate.closed()) return;
  __shared__ int h[128];
  if ((int)threadIdx.x < K) h[threadIdx.x] = 0;
  if (blockIdx.x == 0 && threadIdx.x == 0) flag[0] = 0;
  __syncthreads();
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j < n) {
    double x[3];
    src.pos(j, x);
    const int b = xbin(x, box, K);
    bin[j] = b;
    slot[j] = atomicAdd(&h[b], 1);
  }
  __syncthreads();
  if ((int)threadIdx.x < K) bcnt[blockIdx.x * K + threadIdx.x] = h[threadIdx.x];
}

// Same blocks as k_pme_bin: per bin, the total over all blocks and the count
// in the blocks before this one; the exclusive prefix of the totals gives the
// bin starts (stored by block 0, start[0..K]).
__global__ __launch_bounds__(256) void k_pme_scatter(int n, int K, int nblk,
                                                     const int* __restrict__ bcnt,
                                                     const int* __restrict__ bin,
                                                     const int* __restrict__ slot,
                                                     int* __restrict__ start,
                                                     int* __restrict__ list, Gate gate) {
  if (gate.closed()) return;
  __shared__ int tot[256], off[256], pre[129];
  {
    // thread (r, b): bin b = tid % K, blocks q = r, r + R, ... (R = 256 / K)
    const int R = (int)blockDim.x / K, b = threadIdx.x % K, r = threadIdx.x / K;
    int t = 0, o = 0;
#pragma unroll 4
    for (int q = r; q < nblk; q += R) {
      const int c = bcnt[q * K + b];
      t += c;
      o += q < (int)blockIdx.x ? c : 0;
    }
    tot[threadIdx.x] = t;
    off[threadIdx.x] = o;
    __syncthreads();
    if (r == 0) {
      for (int k = 1; k < R; ++k) {
        t += tot[k * K + b];
        o += off[k * K + b];
      }
    }
    __syncthreads();
    if (r == 0) {
      tot[b] = t;
      off[b] = o;
    }
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    int acc = 0;
    for (int b = 0; b < K; ++b) {
      pre[b] = acc;
      acc += tot[b];
    }
    pre[K] = acc;
  }
  __syncthreads();
  if (blockIdx.x == 0 && (int)threadIdx.x <= K) start[threadIdx.x] = pre[threadIdx.x];
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j < n) {
    const int b = bin[j];
    list[pre[b] + off[b] + slot[j]] = j;
  }
}

//   Q(g) += q M + mu.grad M + Theta:grad grad M   at M = M(u - g)
template <int K>
constexpr int spread_rows() { return K <= 64 ? K : K / 2; }

template <int P, int K, class Src>
__global__ __launch_bounds__(spread_threads<P>()) void k_pme_spread(Src src, double box,
                                                    const int* __restrict__ start,
                                                    const int* __restrict__ list,
                                                    unsigned long long* __restrict__ grid,
                                                    int* __restrict__ flag, Gate gate) {
  if (gate.closed()) return;
  constexpr int YB = spread_rows<K>();
  constexpr int NYB = K / YB;
  __shared__ unsigned long long tile[YB * K];
  const int gx = blockIdx.x / NYB, y0 = (blockIdx.x % NYB) * YB;
  for (int i = threadIdx.x; i < YB * K; i += blockDim.x) tile[i] = 0ull;
  __syncthreads();
  bool bad = false;
#pragma unroll 1
  for (int t1 = 0; t1 < P; ++t1) {
    const int b = (gx + t1) % K;
    const int s1 = start[b + 1];
#pragma unroll 1
    for (int s = start[b] + threadIdx.x; s < s1; s += blockDim.x) {
      const int j = list[s];
      double xj[3];
      src.pos(j, xj);
      if (NYB > 1) {   // rows i0y - t2 (t2 < P) miss this tile: skip the spline work
        const double sy = xj[1] / box;
        const double fy = floor(K * (sy - floor(sy)));
        const int iy = fy >= 0.0 && fy <= K ? (int)fy : 0;
        if (wrap(iy - y0, K) >= YB + P - 1) continue;
      }
      double X[4], th[2][P][4];
      int i0[3];
      site_splines<P>(xj, box, K, t1, X, th, i0);
      double m[10];
      src.mp(j, m);
      const double q = m[0], ux = m[1], uy = m[2], uz = m[3];
      const double txx = m[4], txy = m[5], txz = m[6], tyy = m[7], tyz = m[8], tzz = m[9];
#pragma unroll
      for (int t2 = 0; t2 < P; ++t2) {
        const int ly = wrap(i0[1] - t2 - y0, K);
        if (ly >= YB) continue;
        const double* Y = th[0][t2];
#pragma unroll
        for (int t3 = 0; t3 < P; ++t3) {
          const double* Z = th[1][t3];
          const double v =
              q * X[0] * Y[0] * Z[0] +
              ux * X[1] * Y[0] * Z[0] + uy * X[0] * Y[1] * Z[0] + uz * X[0] * Y[0] * Z[1] +
              txx * X[2] * Y[0] * Z[0] + tyy * X[0] * Y[2] * Z[0] + tzz * X[0] * Y[0] * Z[2] +
              2.0 * (txy * X[1] * Y[1] * Z[0] + txz * X[1] * Y[0] * Z[1] + tyz * X[0] * Y[1] * Z[1]);
          bad |= !(fabs(v) < kFixMax);
          const long long iv = bad ? 0ll : llrint(v * kFix);
          atomicAdd(&tile[ly * K + wrap(i0[2] - t3, K)], (unsigned long long)iv);
        }
      }
    }
  }
  if (bad) atomicOr(flag, 1);
  __syncthreads();
  for (int i = threadIdx.x; i < YB * K; i += blockDim.x)
    grid[((long)gx * K + y0 + i / K) * K + i % K] = tile[i];
}

// ---------------------------------------------------------------- FFT
template <int K>
struct Fft {
  static constexpr int H = K / 2;     // butterflies per line and stage
  static constexpr int L = 256 / H;   // lines per workgroup
  static constexpr int LOG = K == 16 ? 4 : K == 32 ? 5 : K == 64 ? 6 : 7;
  static_assert(K == 16 || K == 32 || K == 64 || K == 128, "grid edge");
};

__device__ __forceinline__ int bitrev(int x, int bits) { return (int)(__brev((unsigned)x) >> (32 - bits)); }

// tw[k] = exp(2 pi i k / K), k < K/2
template <int K>
__device__ __forceinline__ void twiddles(double2* tw) {
  for (int k = threadIdx.x; k < K / 2; k += blockDim.x) {
    double s, c;
    sincospi(2.0 * k / K, &s, &c);
    tw[k] = make_double2(c, s);
  }
}

// Decimation in time on bit-reversed input, natural output:
// X(m) = sum_g x(g) exp(sign 2 pi i m g / K).
template <int K>
__device__ __forceinline__ void fft_dit(double2* sh, const double2* tw, double sign) {
  constexpr int H = Fft<K>::H;
  const int t = threadIdx.x, line = t / H, b = t % H;
  double2* x = sh + line * K;
#pragma unroll
  for (int half = 1; half < K; half <<= 1) {
    const int grp = b / half, pos = b % half;
    const int i = grp * 2 * half + pos, j = i + half;
    const double2 w = tw[pos * (H / half)];
    const double wr = w.x, wi = sign * w.y;
    const double2 a = x[i], c = x[j];
    const double tr = wr * c.x - wi * c.y, ti = wr * c.y + wi * c.x;
    x[i] = make_double2(a.x + tr, a.y + ti);
    x[j] = make_double2(a.x - tr, a.y - ti);
    __syncthreads();
  }
}

// Decimation in frequency on natural input, bit-reversed output (same sum).
template <int K>
__device__ __forceinline__ void fft_dif(double2* sh, const double2* tw, double sign) {
  constexpr int H = Fft<K>::H;
  const int t = threadIdx.x, line = t / H, b = t % H;
  double2* x = sh + line * K;
#pragma unroll
  for (int half = H; half >= 1; half >>= 1) {
    const int grp = b / half, pos = b % half;
    const int i = grp * 2 * half + pos, j = i + half;
    const double2 w = tw[pos * (H / half)];
    const double wr = w.x, wi = sign * w.y;
    const double2 a = x[i], c = x[j];
    const double dr = a.x - c.x, di = a.y - c.y;
    x[i] = make_double2(a.x + c.x, a.y + c.y);
    x[j] = make_double2(wr * dr - wi * di, wr * di + wi * dr);
    __syncthreads();
  }
}

// Grid line geometry: line gl of axis ax (0: x, 1: y, 2: z) starts at base
// and steps by stride; index = (gx K + gy) K + gz.
template <int K>
__device__ __forceinline__ void line_geom(int ax, int gl, long& base, long& stride) {
  const int a = gl / K, b = gl % K;
  if (ax == 2) { base = ((long)a * K + b) * K; stride = 1; }
  else if (ax == 1) { base = (long)a * K * K + b; stride = K; }
  else { base = (long)a * K + b; stride = (long)K * K; }
}

// Element (line, k) handled by thread t in load/store slot s (two slots):
// along z (contiguous) consecutive threads take consecutive k of one line;
// along x, y consecutive threads take consecutive lines (consecutive z).
template <int K>
__device__ __forceinline__ void slot(int ax, int t, int s, int& line, int& k) {
  constexpr int H = Fft<K>::H, L = Fft<K>::L;
  if (ax == 2) { line = t / H; k = t % H + s * H; }
  else { line = t % L; k = t / L + s * H; }
}

// Forward pass along axis ax (z: from the fixed-point grid; y: in place).
template <int K>
// fix2 (nullable): a second real mesh, packed as the imaginary part
__global__ __launch_bounds__(256) void k_pme_fft_fwd(int ax, const unsigned long long* __restrict__ fix,
                                                     const unsigned long long* __restrict__ fix2,
                                                     double2* __restrict__ cg, Gate gate) {
  if (gate.closed()) return;
  constexpr int L = Fft<K>::L, LOG = Fft<K>::LOG;
  __shared__ double2 sh[L * K];
  __shared__ double2 tw[K / 2];
  twiddles<K>(tw);
  const int t = threadIdx.x;
#pragma unroll
  for (int s = 0; s < 2; ++s) {
    int line, k;
    slot<K>(ax, t, s, line, k);
    long base, stride;
    line_geom<K>(ax, blockIdx.x * L + line, base, stride);
    const long g = base + k * stride;
    const double2 v =
        fix ? make_double2((double)(long long)fix[g] * (1.0 / kFix),
                           fix2 ? (double)(long long)fix2[g] * (1.0 / kFix) : 0.0)
            : cg[g];
    sh[line * K + bitrev(k, LOG)] = v;
  }
  __syncthreads();
  fft_dit<K>(sh, tw, 1.0);
#pragma unroll
  for (int s = 0; s < 2; ++s) {
    int line, k;
    slot<K>(ax, t, s, line, k);
    long base, stride;
    line_geom<K>(ax, blockIdx.x * L + line, base, stride);
    cg[base + k * stride] = sh[line * K + k];
  }
}

// Spline modulus D(m) = |sum_{k=0}^{P-2} M_P(k+1) exp(2 pi i m k / K)|^2 for
// m = 0..K-1 into D; where it vanishes (m = K/2, odd P) the mean of the
// neighbours.
template <int P, int K>
__device__ __forceinline__ void spline_moduli(double* D) {
  double mk[P];   // M_P(k + 1), k = 0..P-2: the table at w = 0 read backwards
  {
    double th[P][4];
    bspline_table<P>(0.0, th);
#pragma unroll
    for (int k = 0; k < P - 1; ++k) mk[k] = th[k + 1][0];
  }
  for (int m = threadIdx.x; m < K; m += blockDim.x) {
    double sr = 0.0, si = 0.0;
#pragma unroll
    for (int k = 0; k < P - 1; ++k) {
      double s, c;
      sincospi(2.0 * ((long)m * k % K) / K, &s, &c);
      sr += mk[k] * c;
      si += mk[k] * s;
    }
    D[m] = sr * sr + si * si;
  }
  __syncthreads();
  double fixv = 0.0;
  const int m = threadIdx.x;
  if (m < K && D[m] < 1e-10) fixv = 0.5 * (D[(m + K - 1) % K] + D[(m + 1) % K]);
  __syncthreads();
  if (m < K && fixv != 0.0) D[m] = fixv;
  __syncthreads();
}

// Along x: forward transform (the grid is then fully transformed), multiply
// by W(m) = (4 pi/k^2) exp(-k^2/(4 beta^2)) / (V D(m1) D(m2) D(m3)), W(0) = 0,
// inverse transform, in place.
template <int P, int K>
__global__ __launch_bounds__(256) void k_pme_fft_conv(double2* __restrict__ cg, double box,
                                                      double beta, Gate gate) {
  if (gate.closed()) return;
  constexpr int H = Fft<K>::H, L = Fft<K>::L, LOG = Fft<K>::LOG;
  __shared__ double2 sh[L * K];
  __shared__ double2 tw[K / 2];
  __shared__ double D[K];
  twiddles<K>(tw);
  spline_moduli<P, K>(D);
  const int t = threadIdx.x;
#pragma unroll
  for (int s = 0; s < 2; ++s) {
    int line, k;
    slot<K>(0, t, s, line, k);
    long base, stride;
    line_geom<K>(0, blockIdx.x * L + line, base, stride);
    sh[line * K + bitrev(k, LOG)] = cg[base + k * stride];
  }
  __syncthreads();
  fft_dit<K>(sh, tw, 1.0);
  {
    const int line = t / H, b = t % H;
    const int gl = blockIdx.x * L + line, m2 = gl / K, m3 = gl % K;
    const double vol = box * box * box, f = 2.0 * kPi / box;
    const int s2 = m2 <= K / 2 ? m2 : m2 - K, s3 = m3 <= K / 2 ? m3 : m3 - K;
#pragma unroll
    for (int s = 0; s < 2; ++s) {
      const int m1 = b + s * H;
      const int s1 = m1 <= K / 2 ? m1 : m1 - K;
      double W = 0.0;
      if (s1 || s2 || s3) {
        const double k2 = f * f * (double)(s1 * s1 + s2 * s2 + s3 * s3);
        W = 4.0 * kPi / k2 * exp(-k2 / (4.0 * beta * beta)) / (vol * D[m1] * D[m2] * D[m3]);
      }
      double2& e = sh[line * K + m1];
      e = make_double2(e.x * W, e.y * W);
    }
  }
  __syncthreads();
  fft_dif<K>(sh, tw, -1.0);
#pragma unroll
  for (int s = 0; s < 2; ++s) {
    int line, k;
    slot<K>(0, t, s, line, k);
    long base, stride;
    line_geom<K>(0, blockIdx.x * L + line, base, stride);
    cg[base + k * stride] = sh[line * K + bitrev(k, LOG)];
  }
}

// Inverse pass along axis ax (y: in place; z: real part to phi).
template <int K>
// phi2 (nullable): the imaginary part, the potential of a packed second mesh
__global__ __launch_bounds__(256) void k_pme_fft_inv(int ax, double2* __restrict__ cg,
                                                     double* __restrict__ phi,
                                                     double* __restrict__ phi2, Gate gate) {
  if (gate.closed()) return;
  constexpr int L = Fft<K>::L, LOG = Fft<K>::LOG;
  __shared__ double2 sh[L * K];
  __shared__ double2 tw[K / 2];
  twiddles<K>(tw);
  const int t = threadIdx.x;
#pragma unroll
  for (int s = 0; s < 2; ++s) {
    int line, k;
    slot<K>(ax, t, s, line, k);
    long base, stride;
    line_geom<K>(ax, blockIdx.x * L + line, base, stride);
    sh[line * K + k] = cg[base + k * stride];
  }
  __syncthreads();
  fft_dif<K>(sh, tw, -1.0);
#pragma unroll
  for (int s = 0; s < 2; ++s) {
    int line, k;
    slot<K>(ax, t, s, line, k);
    long base, stride;
    line_geom<K>(ax, blockIdx.x * L + line, base, stride);
    const double2 v = sh[line * K + bitrev(k, LOG)];
    if (phi) {
      phi[base + k * stride] = v.x;
      if (phi2) phi2[base + k * stride] = v.y;
    } else {
      cg[base + k * stride] = v;
    }
  }
}

// ---------------------------------------------------------------- gather
// 8 lanes per site; lane t1 < P sums its plane of the P^3 points.  The
// derivatives of the interpolated potential, D[dx][dy][dz] (dx+dy+dz <= 3),
// are combined across the 8 lanes by three butterfly steps (fixed order).
// Lane 0 of the group writes the force -C [q grad phi + (grad grad phi) mu +
// (grad grad grad phi):Theta], the field -grad phi, and its site's energy
// term q phi + mu.grad phi + Theta:grad grad phi into the block's partial.
template <int P>
__global__ __launch_bounds__(256) void k_pme_gather(int n, const double* __restrict__ xyz,
                                                    const double* __restrict__ mpole, double box,
                                                    int K, const double* __restrict__ phi,
                                                    double* __restrict__ force,
                                                    double* __restrict__ field,
                                                    double* __restrict__ epart) {
  __shared__ double we[4];
  const int gid = blockIdx.x * blockDim.x + threadIdx.x;
  const int j0 = gid >> 3, t1 = gid & 7;
  const bool site = j0 < n;
  const int j = site ? j0 : n - 1;
  double X[4], th[2][P][4];
  int i0[3];
  site_splines<P>(xyz + 3 * j, box, K, t1, X, th, i0);
  // S[dy][dz] over this lane's plane
  double S[4][4];
#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int b = 0; b < 4; ++b) S[a][b] = 0.0;
  if (site && t1 < P) {
    const int gx = wrap(i0[0] - t1, K);
#pragma unroll
    for (int t2 = 0; t2 < P; ++t2) {
      const long row = ((long)gx * K + wrap(i0[1] - t2, K)) * K;
      double z[4] = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
      for (int t3 = 0; t3 < P; ++t3) {
        const double v = phi[row + wrap(i0[2] - t3, K)];
#pragma unroll
        for (int dz = 0; dz < 4; ++dz) z[dz] += v * th[1][t3][dz];
      }
#pragma unroll
      for (int dy = 0; dy < 4; ++dy)
#pragma unroll
        for (int dz = 0; dz < 4 - dy; ++dz) S[dy][dz] += th[0][t2][dy] * z[dz];
    }
  }
  double Dv[4][4][4];
#pragma unroll
  for (int dx = 0; dx < 4; ++dx)
#pragma unroll
    for (int dy = 0; dy < 4; ++dy)
#pragma unroll
      for (int dz = 0; dz < 4; ++dz) {
        if (dx + dy + dz > 3) {   // resolved at compile time (unrolled)
          Dv[dx][dy][dz] = 0.0;
          continue;
        }
        double v = site && t1 < P ? X[dx] * S[dy][dz] : 0.0;
        v += __shfl_xor(v, 1);
        v += __shfl_xor(v, 2);
        v += __shfl_xor(v, 4);
        Dv[dx][dy][dz] = v;
      }
  double e = 0.0;
  if (site && t1 == 0) {
    const double* m = mpole + 10 * j;
    const double q = m[0], u[3] = {m[1], m[2], m[3]};
    const double T[3][3] = {{m[4], m[5], m[6]}, {m[5], m[7], m[8]}, {m[6], m[8], m[9]}};
    auto d1 = [&](int a) { return Dv[a == 0][a == 1][a == 2]; };
    auto d2 = [&](int a, int b) {
      return Dv[(a == 0) + (b == 0)][(a == 1) + (b == 1)][(a == 2) + (b == 2)];
    };
    auto d3 = [&](int a, int b, int c) {
      return Dv[(a == 0) + (b == 0) + (c == 0)][(a == 1) + (b == 1) + (c == 1)]
               [(a == 2) + (b == 2) + (c == 2)];
    };
    e = q * Dv[0][0][0];
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      e += u[a] * d1(a);
#pragma unroll
      for (int b = 0; b < 3; ++b) e += T[a][b] * d2(a, b);
    }
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      double g = q * d1(a);
#pragma unroll
      for (int b = 0; b < 3; ++b) {
        g += u[b] * d2(a, b);
#pragma unroll
        for (int c = 0; c < 3; ++c) g += T[b][c] * d3(a, b, c);
      }
      force[3 * j + a] = -kCoulomb * g;
      if (field) field[3 * j + a] = -d1(a);
    }
  }
  // block partial of the site energies: wave sums in lane order, then waves
  for (int o = 32; o > 0; o >>= 1) e += __shfl_xor(e, o);
  if ((threadIdx.x & 63) == 0) we[threadIdx.x >> 6] = e;
  __syncthreads();
  if (threadIdx.x == 0) epart[blockIdx.x] = ((we[0] + we[1]) + we[2]) + we[3];
}

// ---------------------------------------------------------------- prepared sites
// While a solver iterates, the sites do not move: their x-bin order and
// spline weights (value and first derivative per axis, scaled to d/dx) are
// computed once per solve and read by every iteration's spread and field.
// Tables are indexed by sorted position s (SoA rows of n), so that a tile's
// sites are read with coalesced loads.
template <int P>
__global__ __launch_bounds__(256) void k_pme_tables(int n, SrcDipole src, double box, int K,
                                                    const int* __restrict__ list,
                                                    int* __restrict__ I0,
                                                    double* __restrict__ TB) {
  const int s = blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= n) return;
  const int j = list[s];
  double x[3];
  src.pos(j, x);
  const double kl = K / box;
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    const double f = x[a] / box;
    const double u = K * (f - floor(f));
    const double fl = floor(u);
    I0[a * n + s] = fl >= 0.0 && fl <= K ? (int)fl : 0;
    double t4[P][4];
    bspline_table<P>(u - fl, t4);
#pragma unroll
    for (int t = 0; t < P; ++t) {
      TB[(long)((a * P + t) * 2) * n + s] = t4[t][0];
      TB[(long)((a * P + t) * 2 + 1) * n + s] = t4[t][1] * kl;
    }
  }
}

// Dipole spread from the tables: one workgroup per x-plane (as k_pme_spread).
template <int P, int K>
__global__ __launch_bounds__(spread_threads<P>()) void k_pme_spread_tab(
    int n, const int* __restrict__ start, const int* __restrict__ list,
    const int* __restrict__ I0, const double* __restrict__ TB, const double* __restrict__ v,
    unsigned long long* __restrict__ grid, int* __restrict__ flag, Gate gate,
    Gate partner = Gate{}, int packed = 0) {
  constexpr int YB = spread_rows<K>();
  constexpr int NYB = K / YB;
  const int gx = blockIdx.x / NYB, y0 = (blockIdx.x % NYB) * YB;
  if (gate.closed()) {
    // Packed with a second set that still runs: this set's part of the
    // shared FFT must be an empty mesh, not the previous iteration's.
    if (packed && !partner.closed())
      for (int i = threadIdx.x; i < YB * K; i += blockDim.x)
        grid[((long)gx * K + y0 + i / K) * K + i % K] = 0ull;
    return;
  }
  __shared__ unsigned long long tile[YB * K];
  for (int i = threadIdx.x; i < YB * K; i += blockDim.x) tile[i] = 0ull;
  __syncthreads();   // flag: cleared once per solve, by the preparation
  bool bad = false;
#pragma unroll 1
  for (int t1 = 0; t1 < P; ++t1) {
    const int b = (gx + t1) % K;
    const int s1 = start[b + 1];
#pragma unroll 1
    for (int s = start[b] + threadIdx.x; s < s1; s += blockDim.x) {
      const int iy = I0[n + s];
      if (NYB > 1 && wrap(iy - y0, K) >= YB + P - 1) continue;
      const int iz = I0[2 * n + s];
      const int j = list[s];
      const double vx = v[3 * j], vy = v[3 * j + 1], vz = v[3 * j + 2];
      const double X0 = TB[(long)(t1 * 2) * n + s], X1 = TB[(long)(t1 * 2 + 1) * n + s];
      double Y[P][2], Z[P][2];
#pragma unroll
      for (int t = 0; t < P; ++t) {
        Y[t][0] = TB[(long)((P + t) * 2) * n + s];
        Y[t][1] = TB[(long)((P + t) * 2 + 1) * n + s];
        Z[t][0] = TB[(long)((2 * P + t) * 2) * n + s];
        Z[t][1] = TB[(long)((2 * P + t) * 2 + 1) * n + s];
      }
      const double ax = vx * X1, a0 = X0;
#pragma unroll
      for (int t2 = 0; t2 < P; ++t2) {
        const int ly = wrap(iy - t2 - y0, K);
        if (ly >= YB) continue;
        const double c0 = ax * Y[t2][0] + a0 * vy * Y[t2][1];   // times Z0
        const double c1 = a0 * vz * Y[t2][0];                    // times Z1
#pragma unroll
        for (int t3 = 0; t3 < P; ++t3) {
          const double val = c0 * Z[t3][0] + c1 * Z[t3][1];
          bad |= !(fabs(val) < kFixMax);
          const long long iv = bad ? 0ll : llrint(val * kFix);
          atomicAdd(&tile[ly * K + wrap(iz - t3, K)], (unsigned long long)iv);
        }
      }
    }
  }
  if (bad) atomicOr(flag, 1);
  __syncthreads();
  for (int i = threadIdx.x; i < YB * K; i += blockDim.x)
    grid[((long)gx * K + y0 + i / K) * K + i % K] = tile[i];
}

// Field from the tables, 8 lanes per sorted site (lane t1 its plane);
// out in the sites' own order (out[3 list[s] + a]).
template <int P>
__global__ __launch_bounds__(256) void k_pme_field_tab(int n, int K, const int* __restrict__ list,
                                                       const int* __restrict__ I0,
                                                       const double* __restrict__ TB,
                                                       const double* __restrict__ phi,
                                                       const int* __restrict__ flag,
                                                       double* __restrict__ out, Gate gate) {
  if (gate.closed()) return;
  const int gid = blockIdx.x * blockDim.x + threadIdx.x;
  const int s0 = gid >> 3, t1 = gid & 7;
  const bool site = s0 < n;
  const int s = site ? s0 : n - 1;
  double g[3] = {0.0, 0.0, 0.0};
  if (site && t1 < P) {
    const int gx = wrap(I0[s] - t1, K), iy = I0[n + s], iz = I0[2 * n + s];
    const double X0 = TB[(long)(t1 * 2) * n + s], X1 = TB[(long)(t1 * 2 + 1) * n + s];
    double S00 = 0.0, S10 = 0.0, S01 = 0.0;
#pragma unroll
    for (int t2 = 0; t2 < P; ++t2) {
      const long row = ((long)gx * K + wrap(iy - t2, K)) * K;
      double z0 = 0.0, z1 = 0.0;
#pragma unroll
      for (int t3 = 0; t3 < P; ++t3) {
        const double val = phi[row + wrap(iz - t3, K)];
        z0 += val * TB[(long)((2 * P + t3) * 2) * n + s];
        z1 += val * TB[(long)((2 * P + t3) * 2 + 1) * n + s];
      }
      S00 += TB[(long)((P + t2) * 2) * n + s] * z0;
      S10 += TB[(long)((P + t2) * 2 + 1) * n + s] * z0;
      S01 += TB[(long)((P + t2) * 2) * n + s] * z1;
    }
    g[0] = X1 * S00;
    g[1] = X0 * S10;
    g[2] = X0 * S01;
  }
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    g[a] += __shfl_xor(g[a], 1);
    g[a] += __shfl_xor(g[a], 2);
    g[a] += __shfl_xor(g[a], 4);
  }
  const bool refused = flag[0] != 0;
  if (site && t1 == 0) {
    const int j = list[s];
#pragma unroll
    for (int a = 0; a < 3; ++a) out[3 * j + a] = refused ? __builtin_nan("") : -g[a];
  }
}

// energy = (C/2) sum of the partials in block order; NaN if the spread refused
// a contribution.
__global__ __launch_bounds__(256) void k_pme_energy(const double* __restrict__ epart, int nb,
                                                    const int* __restrict__ flag,
                                                    double* __restrict__ energy) {
  __shared__ double we[4];
  double s = 0.0;
  for (int b = threadIdx.x; b < nb; b += blockDim.x) s += epart[b];
  for (int o = 32; o > 0; o >>= 1) s += __shfl_xor(s, o);
  if ((threadIdx.x & 63) == 0) we[threadIdx.x >> 6] = s;
  __syncthreads();
  if (threadIdx.x == 0) {
    const double t = ((we[0] + we[1]) + we[2]) + we[3];
    energy[0] = flag[0] ? __builtin_nan("") : 0.5 * kCoulomb * t;
  }
}

// Five mesh passes: forward along z, y; forward x, influence function,
// inverse x; inverse along y, z (real part into phi).  With fx2 the second
// real mesh rides in the imaginary part: the influence function is real and
// even, so the inverse returns its potential as the imaginary part (phi2).
template <int P, int K>
void mesh_fft(tk_ctx* ctx, hipStream_t st, const unsigned long long* fx, double2* c2, double* phi,
              double box, double beta, Gate gate, const unsigned long long* fx2 = nullptr,
              double* phi2 = nullptr) {
  const int nlines = K * K / Fft<K>::L;
  ProfScope ps(ctx, st, "pme_fft");
  k_pme_fft_fwd<K><<<nlines, 256, 0, st>>>(2, fx, fx2, c2, gate);
  k_pme_fft_fwd<K><<<nlines, 256, 0, st>>>(1, nullptr, nullptr, c2, gate);
  k_pme_fft_conv<P, K><<<nlines, 256, 0, st>>>(c2, box, beta, gate);
  k_pme_fft_inv<K><<<nlines, 256, 0, st>>>(1, c2, nullptr, nullptr, gate);
  k_pme_fft_inv<K><<<nlines, 256, 0, st>>>(2, c2, phi, phi2, gate);
}

// Bin, spread and convolve: the potential phi on the mesh (scratch of this
// stream), and the spread's refusal flag.
template <int P, int K, class Src>
tk_status mesh_potential(tk_ctx* ctx, hipStream_t st, int n, Src src, double box, double beta,
                         Gate gate, double** phi_out, int** flag_out, const Src* src2 = nullptr,
                         double** phi2_out = nullptr) {
  const long KK = (long)K * K * K;
  const size_t nn = n > 0 ? n : 1;
  const int na = n > 0 ? ceil_div(n, 256) : 1;   // sort blocks (one even when empty)
  void *fix, *cg, *phi, *flag, *bins;
  tk_status s;
  if ((s = scratch(ctx, per_stream("pme_fix", st).c_str(), sizeof(unsigned long long) * KK, &fix)) ||
      (s = scratch(ctx, per_stream("pme_bins", st).c_str(),
                   sizeof(int) * (3 * nn + (size_t)(na + 1) * K + K + 2), &bins)) ||
      (s = scratch(ctx, per_stream("pme_c", st).c_str(), sizeof(double2) * KK, &cg)) ||
      (s = scratch(ctx, per_stream("pme_phi", st).c_str(), sizeof(double) * KK, &phi)) ||
      (s = scratch(ctx, per_stream("pme_flag", st).c_str(), sizeof(int) * 64, &flag)))
    return s;
  void *fix2 = nullptr, *phi2 = nullptr;   // a second source rides in the imaginary part
  if (src2 && ((s = scratch(ctx, per_stream("pme_fix2", st).c_str(),
                            sizeof(unsigned long long) * KK, &fix2)) ||
               (s = scratch(ctx, per_stream("pme_phi2", st).c_str(), sizeof(double) * KK, &phi2))))
    return s;
  auto* fx = (unsigned long long*)fix;
  auto* c2 = (double2*)cg;
  int* bcnt = (int*)bins;
  int* start = bcnt + (size_t)na * K;
  int* bin = start + K + 1;
  int* slot = bin + nn;
  int* list = slot + nn;
  {
    ProfScope ps(ctx, st, "pme_spread");
    k_pme_bin<Src><<<na, 256, 0, st>>>(n, src, box, K, bcnt, bin, slot, (int*)flag, gate);
    k_pme_scatter<<<na, 256, 0, st>>>(n, K, na, bcnt, bin, slot, start, list, gate);
    k_pme_spread<P, K, Src><<<K * (K / spread_rows<K>()), spread_threads<P>(), 0, st>>>(
        src, box, start, list, fx, (int*)flag, gate);
    if (src2)   // the same sites, so the same bins
      k_pme_spread<P, K, Src><<<K * (K / spread_rows<K>()), spread_threads<P>(), 0, st>>>(
          *src2, box, start, list, (unsigned long long*)fix2, (int*)flag, gate);
  }
  mesh_fft<P, K>(ctx, st, fx, c2, (double*)phi, box, beta, gate,
                 (const unsigned long long*)fix2, (double*)phi2);
  if (phi2_out) *phi2_out = (double*)phi2;
  *phi_out = (double*)phi;
  *flag_out = (int*)flag;
  return TK_OK;
}

// Prepared sites of a solve (see k_pme_tables): sort buffers, then I0 [3][n],
// then the weight table [6 P][n].
struct Sites {
  int* bcnt;
  int* start;
  int* bin;
  int* slot;
  int* list;
  int* I0;
  double* TB;
  int* flag;
};

template <int P, int K>
tk_status sites_layout(tk_ctx* ctx, hipStream_t st, int n, Sites& S) {
  const size_t nn = n > 0 ? n : 1;
  const int na = n > 0 ? ceil_div(n, 256) : 1;
  void *ints, *tb, *flag;
  tk_status s;
  if ((s = scratch(ctx, per_stream("pme_sites_i", st).c_str(),
                   sizeof(int) * ((size_t)na * K + K + 1 + 6 * nn), &ints)) ||
      (s = scratch(ctx, per_stream("pme_sites_tb", st).c_str(), sizeof(double) * 6 * P * nn,
                   &tb)) ||
      (s = scratch(ctx, per_stream("pme_flag", st).c_str(), sizeof(int) * 64, &flag)))
    return s;
  S.bcnt = (int*)ints;
  S.start = S.bcnt + (size_t)na * K;
  S.bin = S.start + K + 1;
  S.slot = S.bin + nn;
  S.list = S.slot + nn;
  S.I0 = S.list + nn;
  S.TB = (double*)tb;
  S.flag = (int*)flag;
  return TK_OK;
}

template <int P, int K>
tk_status prepare_sites(tk_ctx* ctx, hipStream_t st, int n, double box, const double* pos,
                        long ps) {
  Sites S;
  tk_status s;
  if ((s = sites_layout<P, K>(ctx, st, n, S))) return s;
  const int na = n > 0 ? ceil_div(n, 256) : 1;
  const SrcDipole src{pos, ps, nullptr};
  ProfScope ps_(ctx, st, "pme_prepare");
  k_pme_bin<SrcDipole><<<na, 256, 0, st>>>(n, src, box, K, S.bcnt, S.bin, S.slot, S.flag, Gate{});
  k_pme_scatter<<<na, 256, 0, st>>>(n, K, na, S.bcnt, S.bin, S.slot, S.start, S.list, Gate{});
  if (n > 0) k_pme_tables<P><<<na, 256, 0, st>>>(n, src, box, K, S.list, S.I0, S.TB);
  TK_HIP(hipGetLastError());
  return TK_OK;
}

// The dipole field of v (and, with v2, of v2 in the same FFT passes: the two
// meshes packed as one complex mesh), each spread and gathered under its own
// gate.
template <int P, int K>
tk_status field_prepared(tk_ctx* ctx, hipStream_t st, int n, double box, const double* v,
                         double beta, double* out, Gate gate, const double* v2 = nullptr,
                         double* out2 = nullptr, Gate gate2 = Gate{}) {
  Sites S;
  tk_status s;
  if ((s = sites_layout<P, K>(ctx, st, n, S))) return s;
  const long KK = (long)K * K * K;
  void *fix, *cg, *phi, *fix2 = nullptr, *phi2 = nullptr;
  if ((s = scratch(ctx, per_stream("pme_fix", st).c_str(), sizeof(unsigned long long) * KK, &fix)) ||
      (s = scratch(ctx, per_stream("pme_c", st).c_str(), sizeof(double2) * KK, &cg)) ||
      (s = scratch(ctx, per_stream("pme_phi", st).c_str(), sizeof(double) * KK, &phi)))
    return s;
  if (v2 && ((s = scratch(ctx, per_stream("pme_fix2", st).c_str(),
                          sizeof(unsigned long long) * KK, &fix2)) ||
             (s = scratch(ctx, per_stream("pme_phi2", st).c_str(), sizeof(double) * KK, &phi2))))
    return s;
  auto* fx = (unsigned long long*)fix;
  auto* fx2 = (unsigned long long*)fix2;
  {
    ProfScope ps(ctx, st, "pme_spread");
    const int packed = v2 ? 1 : 0;
    k_pme_spread_tab<P, K><<<K * (K / spread_rows<K>()), spread_threads<P>(), 0, st>>>(
        n, S.start, S.list, S.I0, S.TB, v, fx, S.flag, gate, gate2, packed);
    if (v2)
      k_pme_spread_tab<P, K><<<K * (K / spread_rows<K>()), spread_threads<P>(), 0, st>>>(
          n, S.start, S.list, S.I0, S.TB, v2, fx2, S.flag, gate2, gate, packed);
  }
  // the passes run while either right-hand side is open
  const Gate both{gate.done, gate.when, v2 ? gate2.done : nullptr};
  mesh_fft<P, K>(ctx, st, fx, (double2*)cg, (double*)phi, box, beta, v2 ? both : gate, fx2,
                 (double*)phi2);
  {
    ProfScope ps(ctx, st, "pme_field");
    if (n > 0) {
      k_pme_field_tab<P><<<ceil_div((long)n * 8, 256), 256, 0, st>>>(
          n, K, S.list, S.I0, S.TB, (const double*)phi, S.flag, out, gate);
      if (v2)
        k_pme_field_tab<P><<<ceil_div((long)n * 8, 256), 256, 0, st>>>(
            n, K, S.list, S.I0, S.TB, (const double*)phi2, S.flag, out2, gate2);
    }
  }
  TK_HIP(hipGetLastError());
  return TK_OK;
}

template <int P, int K>
tk_status run_pme(tk_ctx* ctx, hipStream_t st, const tk_system* sys, const double* mpole,
                  double beta, double* energy, double* force, double* field,
                  const double* m2 = nullptr, double* energy2 = nullptr,
                  double* force2 = nullptr) {
  const int n = sys->n;
  const int nb = ceil_div((long)n * 8, 256);
  double *phi, *phi2 = nullptr;
  int* flag;
  void* epart;
  tk_status s;
  const size_t nbp = nb > 0 ? nb : 1;
  if ((s = scratch(ctx, per_stream("pme_part", st).c_str(), sizeof(double) * 2 * nbp, &epart)))
    return s;
  const SrcMpole src1{sys->xyz, mpole}, src2{sys->xyz, m2};
  if ((s = mesh_potential<P, K>(ctx, st, n, src1, sys->box, beta, Gate{}, &phi, &flag,
                                m2 ? &src2 : nullptr, m2 ? &phi2 : nullptr)))
    return s;
  {
    ProfScope ps(ctx, st, "pme_gather");
    if (n > 0) {
      k_pme_gather<P><<<nb, 256, 0, st>>>(n, sys->xyz, mpole, sys->box, K, phi, force, field,
                                           (double*)epart);
      if (m2)
        k_pme_gather<P><<<nb, 256, 0, st>>>(n, sys->xyz, m2, sys->box, K, phi2, force2, nullptr,
                                             (double*)epart + nbp);
    }
    k_pme_energy<<<1, 256, 0, st>>>((const double*)epart, n > 0 ? nb : 0, flag, energy);
    if (m2)
      k_pme_energy<<<1, 256, 0, st>>>((const double*)epart + nbp, n > 0 ? nb : 0, flag, energy2);
  }
  TK_HIP(hipGetLastError());
  return TK_OK;
}

// b[3 s + a] += f[3 perm[s] + a]
__global__ __launch_bounds__(256) void k_add_permuted(int n, const int32_t* __restrict__ perm,
                                                      const double* __restrict__ f,
                                                      double* __restrict__ b) {
  const int s = blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= n) return;
  const int i = perm[s];
#pragma unroll
  for (int a = 0; a < 3; ++a) b[3 * s + a] += f[3 * i + a];
}

template <int P>
tk_status run_pme_k(tk_ctx* ctx, hipStream_t st, const tk_system* sys, const double* mpole,
                    double beta, int K, double* energy, double* force, double* field,
                    const double* m2, double* energy2, double* force2) {
  switch (K) {
    case 16: return run_pme<P, 16>(ctx, st, sys, mpole, beta, energy, force, field, m2, energy2, force2);
    case 32: return run_pme<P, 32>(ctx, st, sys, mpole, beta, energy, force, field, m2, energy2, force2);
    case 64: return run_pme<P, 64>(ctx, st, sys, mpole, beta, energy, force, field, m2, energy2, force2);
    case 128:
      return run_pme<P, 128>(ctx, st, sys, mpole, beta, energy, force, field, m2, energy2, force2);
    default: return TK_E_ARG;
  }
}

tk_status pme_dispatch(tk_ctx* ctx, hipStream_t st, const tk_system* sys, const double* mpole,
                       double beta, int K, int order, double* energy, double* force,
                       double* field, const double* m2 = nullptr, double* energy2 = nullptr,
                       double* force2 = nullptr) {
  switch (order) {
    case 5: return run_pme_k<5>(ctx, st, sys, mpole, beta, K, energy, force, field, m2, energy2, force2);
    case 6: return run_pme_k<6>(ctx, st, sys, mpole, beta, K, energy, force, field, m2, energy2, force2);
    case 7: return run_pme_k<7>(ctx, st, sys, mpole, beta, K, energy, force, field, m2, energy2, force2);
    case 8: return run_pme_k<8>(ctx, st, sys, mpole, beta, K, energy, force, field, m2, energy2, force2);
    default: return TK_E_ARG;
  }
}

}  // namespace

bool pme_args_ok(int grid, int order) {
  return (grid == 16 || grid == 32 || grid == 64 || grid == 128) && order >= 5 && order <= 8 &&
         grid >= 2 * order;
}

namespace {
template <int P>
tk_status prepare_k(tk_ctx* ctx, hipStream_t st, int n, double box, const double* pos, long ps,
                    int K) {
  switch (K) {
    case 16: return prepare_sites<P, 16>(ctx, st, n, box, pos, ps);
    case 32: return prepare_sites<P, 32>(ctx, st, n, box, pos, ps);
    case 64: return prepare_sites<P, 64>(ctx, st, n, box, pos, ps);
    case 128: return prepare_sites<P, 128>(ctx, st, n, box, pos, ps);
    default: return TK_E_ARG;
  }
}
template <int P>
tk_status field_k(tk_ctx* ctx, hipStream_t st, int n, double box, const double* v, double beta,
                  int K, double* out, Gate gate, const double* v2, double* out2, Gate gate2) {
  switch (K) {
    case 16: return field_prepared<P, 16>(ctx, st, n, box, v, beta, out, gate, v2, out2, gate2);
    case 32: return field_prepared<P, 32>(ctx, st, n, box, v, beta, out, gate, v2, out2, gate2);
    case 64: return field_prepared<P, 64>(ctx, st, n, box, v, beta, out, gate, v2, out2, gate2);
    case 128: return field_prepared<P, 128>(ctx, st, n, box, v, beta, out, gate, v2, out2, gate2);
    default: return TK_E_ARG;
  }
}
}  // namespace

tk_status pme_prepare_sites(tk_ctx* ctx, hipStream_t st, int n, double box, const double* pos,
                            long ps, int grid, int order) {
  if (!pme_args_ok(grid, order)) return TK_E_ARG;
  switch (order) {
    case 5: return prepare_k<5>(ctx, st, n, box, pos, ps, grid);
    case 6: return prepare_k<6>(ctx, st, n, box, pos, ps, grid);
    case 7: return prepare_k<7>(ctx, st, n, box, pos, ps, grid);
    default: return prepare_k<8>(ctx, st, n, box, pos, ps, grid);
  }
}

tk_status pme_prepared_dipole_field(tk_ctx* ctx, hipStream_t st, int n, double box,
                                    const double* v, double beta, int grid, int order,
                                    double* out, const int32_t* done, int run_when_done) {
  if (!pme_args_ok(grid, order)) return TK_E_ARG;
  Gate gate;
  gate.done = done;
  gate.when = run_when_done;
  switch (order) {
    case 5: return field_k<5>(ctx, st, n, box, v, beta, grid, out, gate, nullptr, nullptr, Gate{});
    case 6: return field_k<6>(ctx, st, n, box, v, beta, grid, out, gate, nullptr, nullptr, Gate{});
    case 7: return field_k<7>(ctx, st, n, box, v, beta, grid, out, gate, nullptr, nullptr, Gate{});
    default: return field_k<8>(ctx, st, n, box, v, beta, grid, out, gate, nullptr, nullptr, Gate{});
  }
}

tk_status pme_prepared_dipole_field2(tk_ctx* ctx, hipStream_t st, int n, double box,
                                     const double* v, const double* v2, double beta, int grid,
                                     int order, double* out, double* out2, const int32_t* done,
                                     const int32_t* done2, int run_when_done) {
  if (!pme_args_ok(grid, order)) return TK_E_ARG;
  const Gate g1{done, run_when_done, nullptr}, g2{done2, run_when_done, nullptr};
  switch (order) {
    case 5: return field_k<5>(ctx, st, n, box, v, beta, grid, out, g1, v2, out2, g2);
    case 6: return field_k<6>(ctx, st, n, box, v, beta, grid, out, g1, v2, out2, g2);
    case 7: return field_k<7>(ctx, st, n, box, v, beta, grid, out, g1, v2, out2, g2);
    default: return field_k<8>(ctx, st, n, box, v, beta, grid, out, g1, v2, out2, g2);
  }
}

tk_status pme_mpole_pair(tk_ctx* ctx, hipStream_t st, const tk_system* sys, const double* m1,
                         const double* m2, double beta, int grid, int order, double* e1,
                         double* f1, double* e2, double* f2) {
  if (!pme_args_ok(grid, order)) return TK_E_ARG;
  return pme_dispatch(ctx, st, sys, m1, beta, grid, order, e1, f1, nullptr, m2, e2, f2);
}

tk_status pme_perm_field_add(tk_ctx* ctx, hipStream_t st, const tk_system* sys,
                             const double* mpole, double beta, int grid, int order,
                             const int32_t* perm, double* b_sorted) {
  if (!pme_args_ok(grid, order)) return TK_E_ARG;
  const int n = sys->n;
  if (n == 0) return TK_OK;
  void *tmp;
  tk_status s;
  if ((s = scratch(ctx, per_stream("pme_perm", st).c_str(), sizeof(double) * (7 * (size_t)n + 1),
                   &tmp)))
    return s;
  double* e = (double*)tmp;
  double* f = e + 1;
  double* fld = f + 3 * (size_t)n;
  if ((s = pme_dispatch(ctx, st, sys, mpole, beta, grid, order, e, f, fld))) return s;
  k_add_permuted<<<ceil_div(n, 256), 256, 0, st>>>(n, perm, fld, b_sorted);
  TK_HIP(hipGetLastError());
  return TK_OK;
}

}  // namespace tk

using namespace tk;

extern "C" {

tk_status tk_pme_mpole(tk_ctx* ctx, void* stream, const tk_system* sys, const double* mpole,
                       double ewald_beta, int32_t grid, int32_t order, double* energy,
                       double* force, double* field) {
  if (!ctx) return TK_E_ARG;
  tk_status s = check_system(sys);
  if (s) return s;
  if (!(ewald_beta > 0.0) || !std::isfinite(ewald_beta) || !energy) return TK_E_ARG;
  if (!pme_args_ok(grid, order)) return TK_E_ARG;
  if (sys->n > 0 && (!mpole || !force)) return TK_E_ARG;
  return pme_dispatch(ctx, (hipStream_t)stream, sys, mpole, ewald_beta, grid, order, energy, force,
                      field);
}

}  // extern "C"
