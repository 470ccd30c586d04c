// Spin-glass observables: Fourier components of the tensor overlap of two replicas,
//   Q^{mu nu}(k) = (1/N) sum_r a_r^mu b_r^nu exp(+i k.r),
// at k = 0 and at the three smallest wave-vectors k_d = (2 pi / L) e_d, from which the
// spin-glass susceptibility chi_SG(k) = N <sum |Q(k)|^2>, the second-moment correlation
// length and the Binder cumulant follow.  The paper's model (§2) is what is measured;
// the observables are the standard ones of vector spin glasses (the paper defines
// none).  One record is 65 doubles: Q(0) (9), then per axis d = x, y, z the real and
// imaginary parts of Q(k_d) (9 + 9), then q2(0) = sum |Q(0)|^2 and
// q2(k_min) = (1/3) sum_d sum |Q(k_d)|^2.
//
// Every site contributes 9 products a^mu b^nu, each weighted by 1, cos and sin of
// k_min x, k_min y and k_min z: 63 binary64 accumulators per thread, phase factors
// from an LDS table of (cos, sin)(2 pi j / L).  The wave reduces its 63 sums with a
// transposing butterfly (lane l ends with the total of sum l: 63 exchanges instead of
// 63 x 6), the workgroup adds its waves in order, and the single-lattice form adds
// the workgroups in order in a second launch, so a record is the same bit for bit on
// every run.  The kernels are HBM-bound: 2 x 3 spin components per site.
#include "hsg.h"
#include "hsg_device.h"
#include "hsg_internal.h"

namespace hsg {

namespace {

constexpr int kFourierSums = 63;
constexpr int kThreads = 256;
constexpr int kWaves = kThreads / 64;

// Position of a colour-split element e = c*Nh + xh + Lh*(y + L*z) as mixed-radix
// digits, advanced by a fixed stride with carries (no division in the loop).
struct Cursor {
  int32_t xh, y, z, c;
};

__device__ __forceinline__ Cursor cursor_of(int64_t e, int32_t L, int32_t Lh, int64_t Nh) {
  Cursor p;
  p.c = (int32_t)(e / Nh);
  const int64_t ic = e - (int64_t)p.c * Nh;
  p.xh = (int32_t)(ic % Lh);
  const int64_t row = ic / Lh;
  p.y = (int32_t)(row % L);
  p.z = (int32_t)(row / L);
  return p;
}

__device__ __forceinline__ void advance(Cursor& p, const Cursor& s, int32_t L, int32_t Lh) {
  p.xh += s.xh;
  int32_t carry = p.xh >= Lh;
  p.xh -= carry ? Lh : 0;
  p.y += s.y + carry;
  carry = p.y >= L;
  p.y -= carry ? L : 0;
  p.z += s.z + carry;
  carry = p.z >= L;
  p.z -= carry ? L : 0;
  p.c += s.c + carry;
}

// (cos, sin)(2 pi j / L) for j < L, filled by the workgroup.
__device__ __forceinline__ void fill_phases(double2* tab, int32_t L) {
  for (int32_t j = threadIdx.x; j < L; j += blockDim.x) {
    double s, c;
    sincospi(2.0 * (double)j / (double)L, &s, &c);
    tab[j] = make_double2(c, s);
  }
  __syncthreads();
}

// Adds the sites e = e0, e0 + stride, ... < N of the pair (a, b) to acc.
template <typename R>
__device__ __forceinline__ void accumulate_sites(const R* __restrict__ a, const R* __restrict__ b,
                                                 int32_t L, int64_t e0, int64_t stride,
                                                 const double2* tab,
                                                 double (&acc)[kFourierSums]) {
  const int32_t Lh = L / 2;
  const int64_t Nh = (int64_t)Lh * L * L, N = 2 * Nh;
  if (e0 >= N) return;
  Cursor p = cursor_of(e0, L, Lh, Nh);
  const Cursor s = cursor_of(stride, L, Lh, Nh);
  for (int64_t e = e0; e < N; e += stride) {
    const int64_t base = e + 2 * (int64_t)p.c * Nh;  // plane 3c + mu, element ic
    double av[3], bv[3];
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      av[k] = (double)a[base + k * Nh];
      bv[k] = (double)b[base + k * Nh];
    }
    const int32_t x = 2 * p.xh + ((p.y + p.z + p.c) & 1);
    const double2 ph[3] = {tab[x], tab[p.y], tab[p.z]};
#pragma unroll
    for (int nu = 0; nu < 3; ++nu) {
      double bw[6];
#pragma unroll
      for (int d = 0; d < 3; ++d) {
        bw[2 * d] = bv[nu] * ph[d].x;
        bw[2 * d + 1] = bv[nu] * ph[d].y;
      }
#pragma unroll
      for (int mu = 0; mu < 3; ++mu) {
        const int m = 3 * mu + nu;
        acc[m] = fma(av[mu], bv[nu], acc[m]);
#pragma unroll
        for (int d = 0; d < 3; ++d) {
          acc[9 + 18 * d + m] = fma(av[mu], bw[2 * d], acc[9 + 18 * d + m]);
          acc[18 + 18 * d + m] = fma(av[mu], bw[2 * d + 1], acc[18 + 18 * d + m]);
        }
      }
    }
    advance(p, s, L, Lh);
  }
}

// Wave totals of the 63 sums: at step o = 32, 16, ..., 1 each lane keeps the half of
// its live values selected by lane bit o and receives the partner's copy of that half,
// so after six steps lane l holds the total of sum l (0 for l = 63).
__device__ __forceinline__ double wave_transpose_sum(const double (&acc)[kFourierSums]) {
  double v[64];
#pragma unroll
  for (int k = 0; k < kFourierSums; ++k) v[k] = acc[k];
  v[63] = 0.0;
  const int lane = threadIdx.x & 63;
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) {
    const bool upper = (lane & o) != 0;
#pragma unroll
    for (int j = 0; j < o; ++j) {
      const double keep = upper ? v[j + o] : v[j];
      const double send = upper ? v[j] : v[j + o];
      v[j] = keep + __shfl_xor(send, o);
    }
  }
  return v[0];
}

// Workgroup totals in sums[0..63) (shared memory), waves added in order.
__device__ __forceinline__ void block_totals(const double (&acc)[kFourierSums], double* part,
                                             double* sums) {
  const double w = wave_transpose_sum(acc);
  part[(threadIdx.x >> 6) * 64 + (threadIdx.x & 63)] = w;
  __syncthreads();
  if (threadIdx.x < 64) {
    double t = 0.0;
    for (int k = 0; k < kWaves; ++k) t += part[k * 64 + threadIdx.x];
    sums[threadIdx.x] = t;
  }
  __syncthreads();
}

// The 65-value record from the 63 totals (shared memory) and 1/N.
__device__ __forceinline__ void write_record(const double* sums, double inv_n, double* out) {
  if (threadIdx.x < kFourierSums) out[threadIdx.x] = sums[threadIdx.x] * inv_n;
  if (threadIdx.x == 64) {
    double q2 = 0.0;
    for (int k = 0; k < 9; ++k) q2 = fma(sums[k] * inv_n, sums[k] * inv_n, q2);
    out[63] = q2;
  }
  if (threadIdx.x == 128) {
    double q2 = 0.0;
    for (int k = 9; k < kFourierSums; ++k) q2 = fma(sums[k] * inv_n, sums[k] * inv_n, q2);
    out[64] = q2 / 3.0;
  }
}

__device__ __forceinline__ void write_nan_record(double* out) {
  if (threadIdx.x < HSG_FOURIER_VALUES) out[threadIdx.x] = __builtin_nan("");
}

// Single lattice, first stage: a grid-stride share of the sites per workgroup.
template <typename R>
__global__ __launch_bounds__(kThreads) void fourier_partials_kernel(int32_t L, const R* a,
                                                                    const R* b, double* partials) {
  __shared__ double2 tab[HSG_L_MAX];
  __shared__ double part[kWaves * 64];
  __shared__ double sums[64];
  fill_phases(tab, L);
  double acc[kFourierSums];
#pragma unroll
  for (int k = 0; k < kFourierSums; ++k) acc[k] = 0.0;
  accumulate_sites<R>(a, b, L, (int64_t)blockIdx.x * kThreads + threadIdx.x,
                      (int64_t)gridDim.x * kThreads, tab, acc);
  block_totals(acc, part, sums);
  if (threadIdx.x < 64) partials[(int64_t)blockIdx.x * 64 + threadIdx.x] = sums[threadIdx.x];
}

// Second stage: workgroup partials added in order (wave w takes sums w, w + 4, ...).
__global__ __launch_bounds__(kThreads) void fourier_finish_kernel(const double* partials,
                                                                  int32_t nblocks, double inv_n,
                                                                  double* out) {
  __shared__ double sums[64];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  for (int k = wave; k < 64; k += kWaves) {
    double t = 0.0;
    for (int32_t i = lane; i < nblocks; i += 64) t += partials[(int64_t)i * 64 + k];
    t = wave_sum(t);
    if (lane == 0) sums[k] = t;
  }
  __syncthreads();
  write_record(sums, inv_n, out);
}

// One workgroup per pair of chains; chains of different L (or indices out of range)
// give a record of NaNs.
template <typename R>
__device__ __forceinline__ void chain_pair_record(const hsg_chain* chains, int32_t n_chains,
                                                  int32_t ia, int32_t ib, const R* spins,
                                                  double* out) {
  __shared__ double2 tab[HSG_BATCH_L_MAX];
  __shared__ double part[kWaves * 64];
  __shared__ double sums[64];
  if (ia < 0 || ib < 0 || ia >= n_chains || ib >= n_chains || chains[ia].L != chains[ib].L) {
    write_nan_record(out);
    return;
  }
  const hsg_chain ca = chains[ia], cb = chains[ib];
  fill_phases(tab, ca.L);
  double acc[kFourierSums];
#pragma unroll
  for (int k = 0; k < kFourierSums; ++k) acc[k] = 0.0;
  accumulate_sites<R>(spins + ca.spin_offset, spins + cb.spin_offset, ca.L, threadIdx.x,
                      kThreads, tab, acc);
  block_totals(acc, part, sums);
  write_record(sums, 1.0 / ((double)ca.L * ca.L * ca.L), out);
}

template <typename R>
__global__ __launch_bounds__(kThreads) void chain_pairs_fourier_kernel(const hsg_chain* chains,
                                                                       int32_t n_chains,
                                                                       const R* spins,
                                                                       const int32_t* pairs,
                                                                       double* out) {
  const int32_t p = blockIdx.x;
  chain_pair_record<R>(chains, n_chains, pairs[2 * p], pairs[2 * p + 1], spins,
                       out + (int64_t)HSG_FOURIER_VALUES * p);
}

template <typename R>
__global__ __launch_bounds__(kThreads) void ladder_pairs_fourier_kernel(
    const hsg_chain* chains, int32_t n_chains, const R* spins, const int32_t* chain_at_slot,
    int32_t n_ladders, int32_t n_temps, const int32_t* ladder_pairs, double* out) {
  const int32_t p = blockIdx.x, t = blockIdx.y;
  double* rec = out + (int64_t)HSG_FOURIER_VALUES * ((int64_t)p * n_temps + t);
  const int32_t la = ladder_pairs[2 * p], lb = ladder_pairs[2 * p + 1];
  if (la < 0 || lb < 0 || la >= n_ladders || lb >= n_ladders) {
    write_nan_record(rec);
    return;
  }
  chain_pair_record<R>(chains, n_chains, chain_at_slot[(int64_t)la * n_temps + t],
                       chain_at_slot[(int64_t)lb * n_temps + t], spins, rec);
}

}  // namespace

static unsigned fourier_blocks(int32_t L) {
  const int64_t N = (int64_t)L * L * L;
  const int64_t b = (N + kThreads - 1) / kThreads;
  return (unsigned)(b < kFourierBlocks ? b : kFourierBlocks);
}

template <typename R>
hipError_t launch_overlap_fourier(int32_t L, const void* a, const void* b, double* partials,
                                  double* out, hipStream_t stream) {
  const unsigned nb = fourier_blocks(L);
  hipLaunchKernelGGL(fourier_partials_kernel<R>, dim3(nb), dim3(kThreads), 0, stream, L,
                     (const R*)a, (const R*)b, partials);
  hipLaunchKernelGGL(fourier_finish_kernel, dim3(1), dim3(kThreads), 0, stream,
                     (const double*)partials, (int32_t)nb, 1.0 / ((double)L * L * L), out);
  return hipGetLastError();
}

template <typename R>
hipError_t launch_batch_overlap_fourier(const hsg_batch* b, const int32_t* pairs, int32_t n_pairs,
                                        double* out, hipStream_t st) {
  hipLaunchKernelGGL(chain_pairs_fourier_kernel<R>, dim3((unsigned)n_pairs), dim3(kThreads), 0,
                     st, b->chains, b->n_chains, (const R*)b->spins, pairs, out);
  return hipGetLastError();
}

template <typename R>
hipError_t launch_pt_overlap_fourier(const hsg_pt* pt, const hsg_batch* b,
                                     const int32_t* ladder_pairs, int32_t n_pairs, double* out,
                                     hipStream_t st) {
  hipLaunchKernelGGL(ladder_pairs_fourier_kernel<R>,
                     dim3((unsigned)n_pairs, (unsigned)pt->n_temps), dim3(kThreads), 0, st,
                     b->chains, b->n_chains, (const R*)b->spins, pt->chain_at_slot,
                     pt->n_ladders, pt->n_temps, ladder_pairs, out);
  return hipGetLastError();
}

template hipError_t launch_overlap_fourier<float>(int32_t, const void*, const void*, double*,
                                                  double*, hipStream_t);
template hipError_t launch_overlap_fourier<double>(int32_t, const void*, const void*, double*,
                                                   double*, hipStream_t);
template hipError_t launch_batch_overlap_fourier<float>(const hsg_batch*, const int32_t*, int32_t,
                                                        double*, hipStream_t);
template hipError_t launch_batch_overlap_fourier<double>(const hsg_batch*, const int32_t*,
                                                         int32_t, double*, hipStream_t);
template hipError_t launch_pt_overlap_fourier<float>(const hsg_pt*, const hsg_batch*,
                                                     const int32_t*, int32_t, double*,
                                                     hipStream_t);
template hipError_t launch_pt_overlap_fourier<double>(const hsg_pt*, const hsg_batch*,
                                                      const int32_t*, int32_t, double*,
                                                      hipStream_t);

}  // namespace hsg
