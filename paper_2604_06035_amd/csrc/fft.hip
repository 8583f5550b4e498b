// Direct FFT solve of a periodic level (section "FFTW3 CPU Direct Poisson
// Solver": on a fully uniform periodic level the V-cycles are replaced by one
// forward FFT, a multiplication by the Green's function and an inverse FFT).
//
// The Green's function here is that of the discrete 7-point operator itself:
// its eigenvectors are the Fourier modes, with eigenvalues
//   lambda(k) = sum_d (2 cos(2 pi k_d / n) - 2) / h^2,
// so phi = F^-1[ F[f] / lambda ] (the k = 0 mode set to 0, i.e. mean(phi) = 0)
// is the exact solution of the same discrete system the multigrid solves, up
// to rounding.
//
// Layout and passes (FP64 complex work array W[z][y][kx], kx fastest, rows of
// R = row_len(n) entries of 16 B: the n/2 + 1 frequencies a real row has, padded
// to whole 4-column tiles; every 1-D transform runs in LDS, radix 4):
//   X forward  one oct row per workgroup: the 4 cell rows of n/2 consecutive
//              octs of f (oct-major, one contiguous 32 n-byte run).  A real
//              row of n is transformed as the complex row of n/2 formed by
//              its (even, odd) cell pairs -- exactly an oct's 16-byte pairs --
//              and unpacked into frequencies 0..n/2 (real-to-complex FFT)
//   Y forward  4 consecutive kx (64-byte row pieces) x all y, at one z
//   Z          4 consecutive kx x all z, at one y: forward, Green multiply
//              (and the 1/n^3 of the inverse), inverse
//   Y inverse  as Y forward
//   X inverse  the reverse of X forward: repack, n/2-point inverse, and the
//              real and imaginary parts are the (even, odd) cell pairs of phi
// Forward y and z transforms are decimation in frequency (natural order in,
// bit-reversed frequencies out), inverse ones decimation in time (bit-reversed
// in, natural out), so these passes reorder nothing; the Green multiply
// indexes its y/z eigenvalue table by position (bit-reversed) and its x table
// by frequency.
#include "mg_internal.h"

namespace mg {
namespace {

constexpr int kFThreads = 256;
constexpr int kFW = 4;   // lines per workgroup in the y and z passes (consecutive x; 4 of 8 measured
                          // fastest at 512^3: 40 KB of LDS lets four workgroups share a CU)
// entries per row of W: the n/2 + 1 frequencies of a real row, rounded up to whole tiles
__host__ __device__ constexpr int row_len(int n) { return ((n / 2 + 1 + kFW - 1) / kFW) * kFW; }

__device__ __forceinline__ double2 cmul(double2 a, double2 b) {
  return double2{a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x};
}
__device__ __forceinline__ double2 cmulc(double2 a, double2 b) {   // a * conj(b)
  return double2{a.x * b.x + a.y * b.y, a.y * b.x - a.x * b.y};
}

// Transforms of L lines of n = 2^lg points in LDS, radix 4 (each radix-4
// step is two radix-2 steps merged, so the ordering is still bit-reversed),
// plus one radix-2 step when lg is odd.  LINES_FAST: point p of line l at
// s[p * L + l] (y and z passes); else at s[l * n + p].
// tw[j] = exp(-2 pi i j / n), j < n.
template <int L, bool LINES_FAST>
__device__ __forceinline__ int fidx(int l, int p, int lg) {
  return LINES_FAST ? p * L + l : (l << lg) + p;
}
__device__ __forceinline__ double2 cadd(double2 a, double2 b) { return double2{a.x + b.x, a.y + b.y}; }
__device__ __forceinline__ double2 csub(double2 a, double2 b) { return double2{a.x - b.x, a.y - b.y}; }
__device__ __forceinline__ double2 mul_mi(double2 a) { return double2{a.y, -a.x}; }   // a * (-i)
__device__ __forceinline__ double2 mul_pi(double2 a) { return double2{-a.y, a.x}; }   // a * (+i)

// forward, decimation in frequency: natural order in, bit-reversed out
// tw holds exp(-2 pi i j / (n << tws)); a transform of n points reads every
// (1 << tws)-th entry.
template <int L, bool LINES_FAST>
__device__ void fft_dif(double2* __restrict__ s, const double2* __restrict__ tw, int lg, int tws = 0) {
  int lh = lg - 1;   // log2 of the current radix-2 half span
  for (; lh >= 1; lh -= 2) {
    // radix-2 spans 2q and q merged, q = 2^(lh-1): for offset j < q in a block of 4q,
    // (x0, x1, x2, x3) = x[i + {0, q, 2q, 3q}], W = exp(-2 pi i / 4q):
    //   x[i] = (x0 + x2) + (x1 + x3)          x[i + q]  = ((x0 + x2) - (x1 + x3)) W^2j
    //   x[i + 2q] = ((x0 - x2) - i (x1 - x3)) W^j   x[i + 3q] = ((x0 - x2) + i (x1 - x3)) W^3j
    const int lq = lh - 1, q = 1 << lq, ts = lg - 2 - lq + tws;   // W^j = tw[j << ts]
    const int nb = L << (lg - 2);
    for (int u = threadIdx.x; u < nb; u += blockDim.x) {
      const int l = LINES_FAST ? u % L : u >> (lg - 2);
      const int jg = LINES_FAST ? u / L : u & ((1 << (lg - 2)) - 1);
      const int j = jg & (q - 1);
      const int i = ((jg >> lq) << (lq + 2)) + j;
      const int a0 = fidx<L, LINES_FAST>(l, i, lg), a1 = fidx<L, LINES_FAST>(l, i + q, lg);
      const int a2 = fidx<L, LINES_FAST>(l, i + 2 * q, lg), a3 = fidx<L, LINES_FAST>(l, i + 3 * q, lg);
      const double2 x0 = s[a0], x1 = s[a1], x2 = s[a2], x3 = s[a3];
      const double2 e0 = cadd(x0, x2), e1 = cadd(x1, x3), d0 = csub(x0, x2), d1 = mul_mi(csub(x1, x3));
      s[a0] = cadd(e0, e1);
      s[a1] = cmul(csub(e0, e1), tw[(2 * j) << ts]);
      s[a2] = cmul(cadd(d0, d1), tw[j << ts]);
      s[a3] = cmul(csub(d0, d1), tw[(3 * j) << ts]);
    }
    __syncthreads();
  }
  if (lh == 0) {   // odd lg: the last radix-2 step (span 2, twiddle 1)
    const int nb = L << (lg - 1);
    for (int u = threadIdx.x; u < nb; u += blockDim.x) {
      const int l = LINES_FAST ? u % L : u >> (lg - 1);
      const int jg = LINES_FAST ? u / L : u & ((1 << (lg - 1)) - 1);
      const int a0 = fidx<L, LINES_FAST>(l, 2 * jg, lg), a1 = fidx<L, LINES_FAST>(l, 2 * jg + 1, lg);
      const double2 x0 = s[a0], x1 = s[a1];
      s[a0] = cadd(x0, x1);
      s[a1] = csub(x0, x1);
    }
    __syncthreads();
  }
}
// inverse (unnormalised), decimation in time: bit-reversed in, natural out
template <int L, bool LINES_FAST>
__device__ void fft_dit_inv(double2* __restrict__ s, const double2* __restrict__ tw, int lg, int tws = 0) {
  int lh = 0;
  if (lg & 1) {   // odd lg: the first radix-2 step (span 2, twiddle 1)
    const int nb = L << (lg - 1);
    for (int u = threadIdx.x; u < nb; u += blockDim.x) {
      const int l = LINES_FAST ? u % L : u >> (lg - 1);
      const int jg = LINES_FAST ? u / L : u & ((1 << (lg - 1)) - 1);
      const int a0 = fidx<L, LINES_FAST>(l, 2 * jg, lg), a1 = fidx<L, LINES_FAST>(l, 2 * jg + 1, lg);
      const double2 x0 = s[a0], x1 = s[a1];
      s[a0] = cadd(x0, x1);
      s[a1] = csub(x0, x1);
    }
    __syncthreads();
    lh = 1;
  }
  for (; lh < lg; lh += 2) {
    // radix-2 spans q and 2q merged (q = 2^lh), conjugate twiddles c = conj(W^j), W = exp(-2 pi i / 4q):
    //   b0 = x0 + x1 conj(W^2j), b1 = x0 - x1 conj(W^2j), b2 = x2 + x3 conj(W^2j), b3 = x2 - x3 conj(W^2j)
    //   x[i] = b0 + b2 c, x[i + 2q] = b0 - b2 c, x[i + q] = b1 + i b3 c, x[i + 3q] = b1 - i b3 c
    const int lq = lh, q = 1 << lq, ts = lg - 2 - lq + tws;
    const int nb = L << (lg - 2);
    for (int u = threadIdx.x; u < nb; u += blockDim.x) {
      const int l = LINES_FAST ? u % L : u >> (lg - 2);
      const int jg = LINES_FAST ? u / L : u & ((1 << (lg - 2)) - 1);
      const int j = jg & (q - 1);
      const int i = ((jg >> lq) << (lq + 2)) + j;
      const int a0 = fidx<L, LINES_FAST>(l, i, lg), a1 = fidx<L, LINES_FAST>(l, i + q, lg);
      const int a2 = fidx<L, LINES_FAST>(l, i + 2 * q, lg), a3 = fidx<L, LINES_FAST>(l, i + 3 * q, lg);
      const double2 w2 = tw[(2 * j) << ts], w1 = tw[j << ts];
      const double2 x0 = s[a0], x1 = cmulc(s[a1], w2), x2 = s[a2], x3 = cmulc(s[a3], w2);
      const double2 b0 = cadd(x0, x1), b1 = csub(x0, x1), b2 = cmulc(cadd(x2, x3), w1),
                    b3 = mul_pi(cmulc(csub(x2, x3), w1));
      s[a0] = cadd(b0, b2);
      s[a2] = csub(b0, b2);
      s[a1] = cadd(b1, b3);
      s[a3] = csub(b1, b3);
    }
    __syncthreads();
  }
}

__device__ __forceinline__ void stage_twiddles(double2* __restrict__ stw, const double2* __restrict__ tw, int n) {
  for (int j = threadIdx.x; j < n; j += blockDim.x) stw[j] = tw[j];
}

__device__ __forceinline__ int brev(int v, int lg) { return (int)(__brev((unsigned)v) >> (32 - lg)); }

// X forward: f (oct-major, n^3 cells) -> W (frequencies 0..n/2 of each real
// row, zero padding up to R).  Block b = oy + (n/2) oz.
//   z[m] = f[2m] + i f[2m+1],  Z = FFT_{n/2}(z)  (bit-reversed in LDS),
//   F[k] = (Z[k] + conj Z[n/2-k]) / 2 - i W^k (Z[k] - conj Z[n/2-k]) / 2,
//   W = exp(-2 pi i / n), Z[n/2] = Z[0].
__global__ __launch_bounds__(kFThreads) void k_fft_x_fwd(int lg, const double* __restrict__ f,
                                                         double2* __restrict__ W, const double2* __restrict__ tw,
                                                         double* __restrict__ partials) {
  extern __shared__ double2 sm[];
  const int n = 1 << lg, no = n >> 1, R = row_len(n);
  double2* s = sm;              // 4 lines of n/2
  double2* stw = sm + 4 * no;   // n twiddles
  const int oy = blockIdx.x % no, oz = blockIdx.x / no;
  stage_twiddles(stw, tw, n);
  // the oct row: n/2 octs x 4 cell pairs (part = cell row cy + 2 cz)
  const double2* src = reinterpret_cast<const double2*>(f + ((int64_t)oz * no + oy) * no * 8);
  double acc = 0.0;
  for (int q = threadIdx.x; q < 4 * no; q += blockDim.x) {
    const double2 v = src[q];
    s[(q & 3) * no + (q >> 2)] = v;
    acc += v.x + v.y;
  }
  if (partials) {   // (uniform branch) sum of the oct row, for the mean
    const double tot = block_sum(acc);
    if (threadIdx.x == 0) partials[blockIdx.x] = tot;
  }
  __syncthreads();
  fft_dif<4, false>(s, stw, lg - 1, 1);
  for (int q = threadIdx.x; q < 4 * R; q += blockDim.x) {
    const int l = q / R, k = q - l * R;
    const int y = 2 * oy + (l & 1), z = 2 * oz + (l >> 1);
    double2 out{0.0, 0.0};
    if (k <= no) {
      const double2 zk = s[l * no + brev(k & (no - 1), lg - 1)];
      const double2 zm = s[l * no + brev((no - k) & (no - 1), lg - 1)];
      const double2 e{0.5 * (zk.x + zm.x), 0.5 * (zk.y - zm.y)};    // (Z[k] + conj Z[n/2-k]) / 2
      const double2 o{0.5 * (zk.y + zm.y), -0.5 * (zk.x - zm.x)};   // (Z[k] - conj Z[n/2-k]) / 2i
      out = cadd(e, cmul(o, stw[k]));
    }
    W[((int64_t)z * n + y) * R + k] = out;
  }
}

// X inverse: frequencies 0..n/2 of each row -> phi (oct-major).  With
// A[k] the row's spectrum (A[k + n/2] = conj A[n/2 - k] for a real row),
//   Z[k] = (A[k] + conj A[n/2-k]) + i W^-k (A[k] - conj A[n/2-k]),  k < n/2,
// is the spectrum of the packed row, and the n/2-point inverse gives
// n (phi[2m] + i phi[2m+1]) (the same scale as an n-point inverse).
__global__ __launch_bounds__(kFThreads) void k_fft_x_inv(int lg, const double2* __restrict__ W,
                                                         double* __restrict__ phi, const double2* __restrict__ tw) {
  extern __shared__ double2 sm[];
  const int n = 1 << lg, no = n >> 1, R = row_len(n);
  double2* s = sm;                   // 4 lines of n/2
  double2* stw = sm + 4 * no;        // n twiddles
  double2* sa = stw + n;             // 4 rows of n/2 + 1 frequencies
  const int oy = blockIdx.x % no, oz = blockIdx.x / no;
  stage_twiddles(stw, tw, n);
  for (int q = threadIdx.x; q < 4 * (no + 1); q += blockDim.x) {
    const int l = q / (no + 1), k = q - l * (no + 1);
    const int y = 2 * oy + (l & 1), z = 2 * oz + (l >> 1);
    sa[q] = W[((int64_t)z * n + y) * R + k];
  }
  __syncthreads();
  for (int q = threadIdx.x; q < 4 * no; q += blockDim.x) {
    const int l = q / no, k = q - l * no;
    const double2 ak = sa[l * (no + 1) + k], am = sa[l * (no + 1) + no - k];
    const double2 e{ak.x + am.x, ak.y - am.y};                 // A[k] + conj A[n/2-k]
    const double2 d = cmulc(double2{ak.x - am.x, ak.y + am.y}, stw[k]);   // W^-k (A[k] - conj A[n/2-k])
    s[l * no + brev(k, lg - 1)] = double2{e.x - d.y, e.y + d.x};          // e + i d
  }
  __syncthreads();
  fft_dit_inv<4, false>(s, stw, lg - 1, 1);
  double2* dst = reinterpret_cast<double2*>(phi + ((int64_t)oz * no + oy) * no * 8);
  for (int q = threadIdx.x; q < 4 * no; q += blockDim.x) dst[q] = s[(q & 3) * no + (q >> 2)];
}

// Y pass (forward or inverse) in place on W.  Block b = xt + (R/kFW) z, numbered
// XCD by XCD so that the workgroups reading the other half of each 128-byte
// row segment share an L2.
template <bool INVERSE>
__global__ __launch_bounds__(kFThreads) void k_fft_y(int lg, double2* __restrict__ W, const double2* __restrict__ tw) {
  extern __shared__ double2 sm[];
  const int n = 1 << lg, R = row_len(n), nt = R / kFW;
  double2* s = sm;              // n points x kFW lines, lines fastest
  double2* stw = sm + kFW * n;
  const int xt = xcd_block() % nt, z = xcd_block() / nt;
  double2* base = W + (int64_t)z * n * R + xt * kFW;
  stage_twiddles(stw, tw, n);
  for (int q = threadIdx.x; q < kFW * n; q += blockDim.x) s[q] = base[(int64_t)(q / kFW) * R + (q % kFW)];
  __syncthreads();
  if (INVERSE) fft_dit_inv<kFW, true>(s, stw, lg);
  else fft_dif<kFW, true>(s, stw, lg);
  for (int q = threadIdx.x; q < kFW * n; q += blockDim.x) base[(int64_t)(q / kFW) * R + (q % kFW)] = s[q];
}

// Z pass: forward, multiply by g = gscale / (lamx[kx] + lam[y] + lam[z]) / n^3
// (y and z positions are bit-reversed frequencies and lam is stored by
// position; lamx is by frequency; the zero mode gets 0), inverse.
// Block b = xt + (R/kFW) y, numbered XCD by XCD.
__global__ __launch_bounds__(kFThreads) void k_fft_z(int lg, double2* __restrict__ W, const double2* __restrict__ tw,
                                                     const double* __restrict__ lam, const double* __restrict__ lamx,
                                                     double gscale) {
  extern __shared__ double2 sm[];
  const int n = 1 << lg, R = row_len(n), nt = R / kFW;
  double2* s = sm;
  double2* stw = sm + kFW * n;
  const int xt = xcd_block() % nt, y = xcd_block() / nt;
  const int64_t plane = (int64_t)n * R;
  double2* base = W + (int64_t)y * R + xt * kFW;
  stage_twiddles(stw, tw, n);
  for (int q = threadIdx.x; q < kFW * n; q += blockDim.x) s[q] = base[(q / kFW) * plane + (q % kFW)];
  __syncthreads();
  fft_dif<kFW, true>(s, stw, lg);
  const double ly = lam[y];
  for (int q = threadIdx.x; q < kFW * n; q += blockDim.x) {
    const int x = xt * kFW + (q % kFW), z = q / kFW;
    const double l = lamx[x] + ly + lam[z];
    const double g = (x == 0 && y == 0 && z == 0) ? 0.0 : gscale / l;
    s[q] = double2{s[q].x * g, s[q].y * g};
  }
  __syncthreads();
  fft_dit_inv<kFW, true>(s, stw, lg);
  for (int q = threadIdx.x; q < kFW * n; q += blockDim.x) base[(q / kFW) * plane + (q % kFW)] = s[q];
}

int bitrev(int v, int lg) {
  int r = 0;
  for (int b = 0; b < lg; ++b) r |= ((v >> b) & 1) << (lg - 1 - b);
  return r;
}

}  // namespace

int fft_max_n() { return 1024; }

size_t fft_work_bytes(int n) { return (size_t)n * n * row_len(n) * sizeof(double2); }

void fft_tables(int n, double h, DevBuf& tw, DevBuf& lam, hipStream_t s) {
  const int lg = ilog2(n);
  const int R = row_len(n);
  std::vector<double> t(2 * n), l(n + R);   // t: n complex twiddles; l: n by bit-reversed position, then R by frequency
  const double two_pi = 2.0 * std::acos(-1.0);
  for (int j = 0; j < n; ++j) {
    t[2 * j] = std::cos(two_pi * j / n);
    t[2 * j + 1] = -std::sin(two_pi * j / n);
  }
  for (int p = 0; p < n; ++p) l[p] = (2.0 * std::cos(two_pi * bitrev(p, lg) / n) - 2.0) / (h * h);
  for (int k = 0; k < R; ++k) l[n + k] = (2.0 * std::cos(two_pi * k / n) - 2.0) / (h * h);
  tw.alloc((size_t)n * sizeof(double2));
  lam.alloc((size_t)(n + R) * sizeof(double));
  MG_HIP(hipMemcpyAsync(tw.p, t.data(), (size_t)n * sizeof(double2), hipMemcpyHostToDevice, s));
  MG_HIP(hipMemcpyAsync(lam.p, l.data(), (size_t)(n + R) * sizeof(double), hipMemcpyHostToDevice, s));
  MG_HIP(hipStreamSynchronize(s));   // the host vectors go out of scope
}

void fft_solve(int n, const double* src, double gscale, double* phi, void* work, const void* tw, const double* lam,
               double* partials, hipStream_t s) {
  const int lg = ilog2(n);
  const int no = n / 2;
  double2* W = static_cast<double2*>(work);
  const double2* t = static_cast<const double2*>(tw);
  const size_t lds_x = (size_t)(4 * no + n + 4 * (no + 1)) * sizeof(double2);
  const size_t lds_yz = (size_t)(kFW * n + n) * sizeof(double2);
  static bool attr_set = false;
  if (!attr_set) {   // allow more than the default dynamic LDS (n = 1024: 144 KB in the y and z passes)
    const int m = fft_max_n();
    const int cap_x = (int)((4 * (m / 2) + m + 4 * (m / 2 + 1)) * sizeof(double2));
    const int cap_yz = (int)((kFW * m + m) * sizeof(double2));
    MG_HIP(hipFuncSetAttribute((const void*)k_fft_x_fwd, hipFuncAttributeMaxDynamicSharedMemorySize, cap_x));
    MG_HIP(hipFuncSetAttribute((const void*)k_fft_x_inv, hipFuncAttributeMaxDynamicSharedMemorySize, cap_x));
    MG_HIP(hipFuncSetAttribute((const void*)k_fft_y<false>, hipFuncAttributeMaxDynamicSharedMemorySize, cap_yz));
    MG_HIP(hipFuncSetAttribute((const void*)k_fft_y<true>, hipFuncAttributeMaxDynamicSharedMemorySize, cap_yz));
    MG_HIP(hipFuncSetAttribute((const void*)k_fft_z, hipFuncAttributeMaxDynamicSharedMemorySize, cap_yz));
    attr_set = true;
  }
  const int R = row_len(n);
  const unsigned bx = (unsigned)(no * no), byz = (unsigned)((R / kFW) * n);
  const double g = gscale / ((double)n * n * n);
  hipLaunchKernelGGL(k_fft_x_fwd, dim3(bx), dim3(kFThreads), lds_x, s, lg, src, W, t, partials);
  hipLaunchKernelGGL(k_fft_y<false>, dim3(byz), dim3(kFThreads), lds_yz, s, lg, W, t);
  hipLaunchKernelGGL(k_fft_z, dim3(byz), dim3(kFThreads), lds_yz, s, lg, W, t, lam, lam + n, g);
  hipLaunchKernelGGL(k_fft_y<true>, dim3(byz), dim3(kFThreads), lds_yz, s, lg, W, t);
  hipLaunchKernelGGL(k_fft_x_inv, dim3(bx), dim3(kFThreads), lds_x, s, lg, W, phi, t);
  check_launch();
}

}  // namespace mg
