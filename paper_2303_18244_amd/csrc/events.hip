// Event-level steps after the matrix element (see events.h).  All of them
// stream per-event rows of device memory once or twice: they are bound by
// HBM bandwidth and launch latency, not by arithmetic.
#include "events.h"

namespace mgme {
namespace {

constexpr int kBlock = 256;
constexpr int kWaves = kBlock / 64;
constexpr int kPerThread = 8;                 // events per thread in one unweighting tile
constexpr int kTile = kBlock * kPerThread;    // events per unweighting tile
constexpr int kMaxPartials = 1024;

// Butterfly reductions: every lane ends with the same value, formed in the
// same order whatever the scheduling.
__device__ __forceinline__ double wave_sum(double x) {
  for (int d = 32; d >= 1; d >>= 1) x += __shfl_xor(x, d);
  return x;
}
__device__ __forceinline__ double wave_max(double x) {
  for (int d = 32; d >= 1; d >>= 1) x = fmax(x, __shfl_xor(x, d));
  return x;
}

__global__ void __launch_bounds__(kBlock) weights_kernel(long long n, const double* __restrict__ wgt,
                                                        const double* __restrict__ me, double k,
                                                        double* __restrict__ w, double* __restrict__ part) {
  double s = 0.0, s2 = 0.0, mx = 0.0;
  const long long stride = (long long)gridDim.x * kBlock;
  for (long long e = (long long)blockIdx.x * kBlock + threadIdx.x; e < n; e += stride) {
    const double x = (wgt[e] * me[e]) * k;
    if (w) w[e] = x;
    s += x;
    s2 += x * x;
    mx = fmax(mx, x);
  }
  s = wave_sum(s);
  s2 = wave_sum(s2);
  mx = wave_max(mx);
  __shared__ double red[3][kWaves];
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  if (lane == 0) {
    red[0][wv] = s;
    red[1][wv] = s2;
    red[2][wv] = mx;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    double a = 0.0, b = 0.0, c = 0.0;
    for (int i = 0; i < kWaves; ++i) {
      a += red[0][i];
      b += red[1][i];
      c = fmax(c, red[2][i]);
    }
    part[3 * blockIdx.x + 0] = a;
    part[3 * blockIdx.x + 1] = b;
    part[3 * blockIdx.x + 2] = c;
  }
}

__global__ void __launch_bounds__(kBlock) weights_finish_kernel(int nparts, const double* __restrict__ part,
                                                               double* __restrict__ stats) {
  double s = 0.0, s2 = 0.0, mx = 0.0;
  for (int b = threadIdx.x; b < nparts; b += kBlock) {
    s += part[3 * b + 0];
    s2 += part[3 * b + 1];
    mx = fmax(mx, part[3 * b + 2]);
  }
  s = wave_sum(s);
  s2 = wave_sum(s2);
  mx = wave_max(mx);
  __shared__ double red[3][kWaves];
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  if (lane == 0) {
    red[0][wv] = s;
    red[1][wv] = s2;
    red[2][wv] = mx;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    double a = 0.0, b = 0.0, c = 0.0;
    for (int i = 0; i < kWaves; ++i) {
      a += red[0][i];
      b += red[1][i];
      c = fmax(c, red[2][i]);
    }
    stats[0] = a;
    stats[1] = b;
    stats[2] = c;
  }
}

// ------------------------------------------------------------ unweighting
__device__ __forceinline__ bool survives(const double* __restrict__ w, const double* __restrict__ r, long long e,
                                         long long n, double ref) {
  return e < n && r[e] * ref < w[e];
}

// Kept events of each tile of kTile consecutive events.
__global__ void __launch_bounds__(kBlock) unweight_count_kernel(long long n, const double* __restrict__ w,
                                                               const double* __restrict__ r,
                                                               const double* __restrict__ wref,
                                                               long long* __restrict__ counts) {
  const double ref = *wref;
  const long long base = (long long)blockIdx.x * kTile;
  int c = 0;
  for (int j = 0; j < kPerThread; ++j) c += survives(w, r, base + j * kBlock + threadIdx.x, n, ref) ? 1 : 0;
  for (int d = 32; d >= 1; d >>= 1) c += __shfl_xor(c, d);
  __shared__ int red[kWaves];
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = c;
  __syncthreads();
  if (threadIdx.x == 0) {
    long long t = 0;
    for (int i = 0; i < kWaves; ++i) t += red[i];
    counts[blockIdx.x] = t;
  }
}

// Exclusive prefix sum of the tile counts by one block; the total is the
// number of kept events.
__global__ void __launch_bounds__(1024) unweight_scan_kernel(long long ntiles, const long long* __restrict__ counts,
                                                            long long* __restrict__ offs,
                                                            long long* __restrict__ nkept) {
  __shared__ long long wsum[16];
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  long long carry = 0;
  for (long long b0 = 0; b0 < ntiles; b0 += 1024) {
    const long long b = b0 + threadIdx.x;
    const long long v = b < ntiles ? counts[b] : 0;
    long long x = v;
    for (int d = 1; d < 64; d <<= 1) {
      const long long y = __shfl_up(x, d);
      if (lane >= d) x += y;
    }
    if (lane == 63) wsum[wv] = x;
    __syncthreads();
    long long pre = 0, tot = 0;
    for (int i = 0; i < 16; ++i) {
      if (i < wv) pre += wsum[i];
      tot += wsum[i];
    }
    if (b < ntiles) offs[b] = carry + pre + x - v;
    carry += tot;
    __syncthreads();
  }
  if (threadIdx.x == 0) *nkept = carry;
}

// Writes the kept indices of each tile, in order, from the tile's offset.
__global__ void __launch_bounds__(kBlock) unweight_scatter_kernel(long long n, const double* __restrict__ w,
                                                                 const double* __restrict__ r,
                                                                 const double* __restrict__ wref,
                                                                 const long long* __restrict__ offs,
                                                                 long long* __restrict__ idx) {
  const double ref = *wref;
  const long long base = (long long)blockIdx.x * kTile;
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  __shared__ int wcount[kWaves];
  long long run = offs[blockIdx.x];
  for (int j = 0; j < kPerThread; ++j) {
    const long long e = base + j * kBlock + threadIdx.x;
    const bool keep = survives(w, r, e, n, ref);
    const unsigned long long m = __ballot(keep);
    const int before = __popcll(m & ((1ull << lane) - 1ull));
    if (lane == 0) wcount[wv] = __popcll(m);
    __syncthreads();
    int wpre = 0, tot = 0;
    for (int i = 0; i < kWaves; ++i) {
      if (i < wv) wpre += wcount[i];
      tot += wcount[i];
    }
    if (keep) idx[run + wpre + before] = e;
    run += tot;
    __syncthreads();
  }
}

// ------------------------------------------------------- helicity and colour
template <typename T>
__global__ void __launch_bounds__(kBlock) jamp2_kernel(long long n, int nhel, int ncol, const T* __restrict__ J,
                                                      long long ldj, double* __restrict__ jamp2, long long ldo) {
  const long long e = (long long)blockIdx.x * kBlock + threadIdx.x;
  const int s = blockIdx.y;
  if (e >= n) return;
  double acc = 0.0;
  for (int h = 0; h < nhel; ++h) {
    const T* p = J + 2 * (((long long)h * ncol + s) * ldj + e);
    acc += (double)p[0] * (double)p[0] + (double)p[1] * (double)p[1];
  }
  jamp2[(long long)s * ldo + e] = acc;
}

// Inverse-CDF choice among `m` non-negative weights row[i*ld]: index of the
// first running sum above r times the total, else the last non-zero weight,
// else -1.
__device__ __forceinline__ int choose(const double* __restrict__ row, long long ld, int m, double r) {
  double total = 0.0;
  for (int i = 0; i < m; ++i) total += row[(long long)i * ld];
  const double t = r * total;
  double run = 0.0;
  int pick = -1, last = -1;
  for (int i = 0; i < m; ++i) {
    const double x = row[(long long)i * ld];
    run += x;
    if (x != 0.0) last = i;
    if (pick < 0 && run > t) pick = i;
  }
  return pick >= 0 ? pick : last;
}

__global__ void __launch_bounds__(kBlock) select_kernel(long long n, const MeArgs args,
                                                       const double* __restrict__ meh, long long ldh, int ncol,
                                                       const double* __restrict__ jamp2, long long ldj,
                                                       const double* __restrict__ r_hel,
                                                       const double* __restrict__ r_col, int* __restrict__ hel,
                                                       int* __restrict__ col) {
  const long long e = (long long)blockIdx.x * kBlock + threadIdx.x;
  if (e >= n) return;
  const int ih = choose(meh + e, ldh, args.nhel, r_hel[e]);
  hel[e] = ih >= 0 ? args.hel[ih] : 0;
  const int s = choose(jamp2 + e, ldj, ncol, r_col[e]);
  col[e] = s >= 0 ? s : 0;
}

}  // namespace

int weights_partials(long long n) {
  long long nb = (n + (long long)kBlock * 16 - 1) / ((long long)kBlock * 16);
  if (nb < 1) nb = 1;
  if (nb > kMaxPartials) nb = kMaxPartials;
  return (int)nb;
}

hipError_t launch_event_weights(long long n, const double* wgt, const double* me, double k, double* w, double* part,
                                double* stats, hipStream_t stream) {
  const int nb = weights_partials(n);
  weights_kernel<<<nb, kBlock, 0, stream>>>(n, wgt, me, k, w, part);
  hipError_t err = hipGetLastError();
  if (err != hipSuccess) return err;
  weights_finish_kernel<<<1, kBlock, 0, stream>>>(nb, part, stats);
  return hipGetLastError();
}

long long unweight_tiles(long long n) { return (n + kTile - 1) / kTile; }

hipError_t launch_unweight(long long n, const double* w, const double* r, const double* wref, long long* idx,
                           long long* nkept, long long* tiles, hipStream_t stream) {
  const long long nt = unweight_tiles(n);
  if (nt > 0x7fffffffLL) return hipErrorInvalidValue;
  long long* counts = tiles;
  long long* offs = tiles + nt;
  if (nt > 0) {
    unweight_count_kernel<<<(unsigned)nt, kBlock, 0, stream>>>(n, w, r, wref, counts);
    hipError_t err = hipGetLastError();
    if (err != hipSuccess) return err;
  }
  unweight_scan_kernel<<<1, 1024, 0, stream>>>(nt, counts, offs, nkept);
  hipError_t err = hipGetLastError();
  if (err != hipSuccess || nt == 0) return err;
  unweight_scatter_kernel<<<(unsigned)nt, kBlock, 0, stream>>>(n, w, r, wref, offs, idx);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_jamp2(long long n, int nhel, int ncol, const T* J, long long ldj, double* jamp2, long long ldo,
                        hipStream_t stream) {
  if (n <= 0) return hipSuccess;
  const dim3 grid((unsigned)((n + kBlock - 1) / kBlock), (unsigned)ncol);
  jamp2_kernel<T><<<grid, kBlock, 0, stream>>>(n, nhel, ncol, J, ldj, jamp2, ldo);
  return hipGetLastError();
}
template hipError_t launch_jamp2<float>(long long, int, int, const float*, long long, double*, long long,
                                        hipStream_t);
template hipError_t launch_jamp2<double>(long long, int, int, const double*, long long, double*, long long,
                                         hipStream_t);

hipError_t launch_select(long long n, const MeArgs* args, const double* meh, long long ldh, int ncol,
                         const double* jamp2, long long ldj, const SelectArgs* sel, long long offset,
                         hipStream_t stream) {
  if (n <= 0) return hipSuccess;
  select_kernel<<<(unsigned)((n + kBlock - 1) / kBlock), kBlock, 0, stream>>>(
      n, *args, meh, ldh, ncol, jamp2, ldj, sel->r_hel + offset, sel->r_col + offset, sel->hel + offset,
      sel->col + offset);
  return hipGetLastError();
}

}  // namespace mgme
