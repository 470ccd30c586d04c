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
// Every site contributes its 9 products a^mu b^nu weighted by 1 and by cos and sin of
// k_min x, k_min y and k_min z: 63 binary64 sums per thread.  A thread takes items of
// four sites of one row (two for binary64 data or odd L/2) that share y and z, so
// the y, z and k = 0 weights multiply the item's summed products once: 45 binary64
// operations per site instead of 81, which leaves the kernel bound by HBM.  Phase
// factors come from an LDS table of (cos, sin)(2 pi j / L).  The wave reduces its 63
// sums with a transposing butterfly (lane l ends with the total of sum l: 63
// exchanges instead of 63 x 6), the workgroup adds its waves in order, and the
// single-lattice form adds the workgroups in order in a second launch, so a record is
// the same bit for bit on every run.
#include "hsg.h"
#include "hsg_device.h"
#include "hsg_internal.h"

namespace hsg {

namespace {

constexpr int kFourierSums = 63;
constexpr int kThreads = 256;
constexpr int kWaves = kThreads / 64;

// Work item: the sites (x, y, z) of one row (y, z) at xh = j and, when L/2 is even,
// xh = j + L/4, in both colours -- 2H sites that share their y and z phase factors,
// so those weights multiply the item's summed products once.  Items are numbered
// j + (L/(2H)) * (y + L*z) and enumerated as mixed-radix digits advanced by a fixed
// stride with carries (no division in the loop).
struct Cursor {
  int32_t j, y, z;
};

struct ItemShape {
  int32_t L, Lh, Lq;  // Lq = L / (2H): items per row
  int64_t Nh, n_items;
};

template <int H>
__device__ __forceinline__ ItemShape item_shape(int32_t L) {
  ItemShape sh;
  sh.L = L;
  sh.Lh = L / 2;
  sh.Lq = sh.Lh / H;
  sh.Nh = (int64_t)sh.Lh * L * L;
  sh.n_items = (int64_t)sh.Lq * L * L;
  return sh;
}

__device__ __forceinline__ Cursor cursor_of(int64_t w, const ItemShape& sh) {
  Cursor p;
  p.j = (int32_t)(w % sh.Lq);
  const int64_t row = w / sh.Lq;
  p.y = (int32_t)(row % sh.L);
  p.z = (int32_t)(row / sh.L);  // >= L once w is past the last item
  return p;
}

__device__ __forceinline__ void advance(Cursor& p, const Cursor& s, const ItemShape& sh) {
  p.j += s.j;
  int32_t carry = p.j >= sh.Lq;
  p.j -= carry ? sh.Lq : 0;
  p.y += s.y + carry;
  carry = p.y >= sh.L;
  p.y -= carry ? sh.L : 0;
  p.z += s.z + carry;
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

// One item's inputs, fetched one item ahead of its arithmetic.
template <typename R, int H>
struct ItemIn {
  R a[2 * H][3], b[2 * H][3];
  int32_t x[2 * H];
  int32_t y, z;
};

template <typename R, int H>
__device__ __forceinline__ ItemIn<R, H> fetch_item(const R* __restrict__ a,
                                                   const R* __restrict__ b, const Cursor& p,
                                                   const ItemShape& sh) {
  ItemIn<R, H> in;
  const int64_t row = (int64_t)sh.Lh * (p.y + (int64_t)sh.L * p.z);
  const int32_t par = (p.y + p.z) & 1;
#pragma unroll
  for (int h = 0; h < H; ++h) {
    const int32_t xh = p.j + h * sh.Lq;
#pragma unroll
    for (int c = 0; c < 2; ++c) {
      const int q = 2 * h + c;
      const int64_t base = 3 * c * sh.Nh + row + xh;  // plane 3c + mu
#pragma unroll
      for (int k = 0; k < 3; ++k) {
        in.a[q][k] = a[base + k * sh.Nh];
        in.b[q][k] = b[base + k * sh.Nh];
      }
      in.x[q] = 2 * xh + (par ^ c);
    }
  }
  in.y = p.y;
  in.z = p.z;
  return in;
}

// acc[0..9): sum of q; acc[9 + 18d ..): sum of q cos(k_min r_d); acc[18 + 18d ..): sin.
template <typename R, int H>
__device__ __forceinline__ void add_item(const ItemIn<R, H>& in, const double2* tab,
                                         double (&acc)[kFourierSums]) {
  double P[9];  // the item's summed products, for the phases it shares
#pragma unroll
  for (int q = 0; q < 2 * H; ++q) {
    double av[3], bv[3];
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      av[k] = (double)in.a[q][k];
      bv[k] = (double)in.b[q][k];
    }
    const double2 px = tab[in.x[q]];
#pragma unroll
    for (int m = 0; m < 9; ++m) {
      const double prod = av[m / 3] * bv[m % 3];
      P[m] = q == 0 ? prod : P[m] + prod;
      acc[9 + m] = fma(prod, px.x, acc[9 + m]);
      acc[18 + m] = fma(prod, px.y, acc[18 + m]);
    }
  }
  const double2 py = tab[in.y], pz = tab[in.z];
#pragma unroll
  for (int m = 0; m < 9; ++m) {
    acc[m] += P[m];
    acc[27 + m] = fma(P[m], py.x, acc[27 + m]);
    acc[36 + m] = fma(P[m], py.y, acc[36 + m]);
    acc[45 + m] = fma(P[m], pz.x, acc[45 + m]);
    acc[54 + m] = fma(P[m], pz.y, acc[54 + m]);
  }
}

// Adds the items w = w0, w0 + stride, ... of the pair (a, b) to acc, in that order,
// the loads of item i + 1 issued before the arithmetic of item i.
template <typename R, int H>
__device__ __forceinline__ void accumulate_items(const R* __restrict__ a,
                                                 const R* __restrict__ b, int32_t L, int64_t w0,
                                                 int64_t stride, const double2* tab,
                                                 double (&acc)[kFourierSums]) {
  const ItemShape sh = item_shape<H>(L);
  if (w0 >= sh.n_items) return;
  const Cursor s = cursor_of(stride, sh);
  Cursor p = cursor_of(w0, sh);
  ItemIn<R, H> cur = fetch_item<R, H>(a, b, p, sh);
  for (int64_t w = w0;;) {
    const int64_t wn = w + stride;
    advance(p, s, sh);
    const bool more = wn < sh.n_items;
    ItemIn<R, H> next;
    if (more) next = fetch_item<R, H>(a, b, p, sh);
    add_item<R, H>(cur, tab, acc);
    if (!more) break;
    cur = next;
    w = wn;
  }
}

// Items of four sites for binary32 data where L/2 is even, of two otherwise (four
// binary64 sites in flight twice over would not fit the register file).
template <typename R>
__device__ __forceinline__ bool quad_items(int32_t L) {
  return sizeof(R) == 4 && (L / 2) % 2 == 0;
}

template <typename R>
__device__ __forceinline__ void accumulate_pair(const R* a, const R* b, int32_t L, int64_t w0,
                                                int64_t stride, const double2* tab,
                                                double (&acc)[kFourierSums]) {
  if (quad_items<R>(L))
    accumulate_items<R, 2>(a, b, L, w0, stride, tab, acc);
  else
    accumulate_items<R, 1>(a, b, L, w0, stride, tab, acc);
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
  accumulate_pair<R>(a, b, L, (int64_t)blockIdx.x * kThreads + threadIdx.x,
                     (int64_t)gridDim.x * kThreads, tab, acc);
  block_totals(acc, part, sums);
  if (threadIdx.x < 64)
    partials[(int64_t)blockIdx.x * kFourierSlots + threadIdx.x] = sums[threadIdx.x];
}

// Second stage: workgroup partials added in order.  Wave w loads the rows of blocks
// w, w + 16, ... at once (lane = sum), then the 16 waves are added in order.
constexpr int kFinishThreads = 1024;
constexpr int kFinishWaves = kFinishThreads / 64;
constexpr int kRowsPerWave = kFourierBlocks / kFinishWaves;

__global__ __launch_bounds__(kFinishThreads) void fourier_finish_kernel(const double* partials,
                                                                        int32_t nblocks,
                                                                        double inv_n,
                                                                        double* out) {
  __shared__ double part[kFinishWaves * 64];
  __shared__ double sums[64];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  double v[kRowsPerWave];
#pragma unroll
  for (int r = 0; r < kRowsPerWave; ++r) {
    const int32_t i = wave + r * kFinishWaves;
    v[r] = i < nblocks ? partials[(int64_t)i * kFourierSlots + lane] : 0.0;
  }
  double t = 0.0;
#pragma unroll
  for (int r = 0; r < kRowsPerWave; ++r) t += v[r];
  part[wave * 64 + lane] = t;
  __syncthreads();
  if (threadIdx.x < 64) {
    double u = 0.0;
    for (int w = 0; w < kFinishWaves; ++w) u += part[w * 64 + threadIdx.x];
    sums[threadIdx.x] = u;
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
  accumulate_pair<R>(spins + ca.spin_offset, spins + cb.spin_offset, ca.L, threadIdx.x,
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

static unsigned fourier_blocks(int32_t L, size_t elem) {
  const int64_t Lh = L / 2;
  const int64_t items = (elem == 4 && Lh % 2 == 0 ? Lh / 2 : Lh) * L * L;
  const int64_t b = (items + kThreads - 1) / kThreads;
  return (unsigned)(b < kFourierBlocks ? b : kFourierBlocks);
}

template <typename R>
hipError_t launch_overlap_fourier(int32_t L, const void* a, const void* b, double* partials,
                                  double* out, hipStream_t stream) {
  const unsigned nb = fourier_blocks(L, sizeof(R));
  hipLaunchKernelGGL(fourier_partials_kernel<R>, dim3(nb), dim3(kThreads), 0, stream, L,
                     (const R*)a, (const R*)b, partials);
  hipLaunchKernelGGL(fourier_finish_kernel, dim3(1), dim3(kFinishThreads), 0, stream,
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
