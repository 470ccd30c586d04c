// Lattice-wide kernels: random initial state, canonical <-> colour-split layout
// conversion, renormalisation, and the binary64 energy and overlap reductions.
// None of these runs per sweep except renormalisation (every R sweeps), so they
// favour simple grid-stride loops over the tuned tiling of the colour passes.
#include "hsg_device.h"
#include "hsg_internal.h"
#include "hsg_site.h"

namespace hsg {

namespace {

inline unsigned grid_for(int64_t n, int threads) {
  const int64_t b = (n + threads - 1) / threads;
  return (unsigned)(b < 65536 ? (b < 1 ? 1 : b) : 65536);
}

template <typename R>
__global__ __launch_bounds__(256) void init_kernel(int32_t L, uint32_t k0, uint32_t k1, R* spins,
                                                   R* J) {
  const int64_t N = (int64_t)L * L * L;
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < N;
       e += (int64_t)gridDim.x * blockDim.x) {
    init_site<R>(L, e, k0, k1, spins, J, k0, k1);
  }
}

template <typename R>
__global__ __launch_bounds__(256) void import_kernel(int32_t L, const R* cs, const R* cj, R* spins,
                                                     R* J) {
  const int64_t N = (int64_t)L * L * L, Nh = N / 2;
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < N;
       e += (int64_t)gridDim.x * blockDim.x) {
    const SiteOf st = site_of(e, L);
    const int64_t base = (int64_t)3 * st.c * Nh + st.ic;
    for (int k = 0; k < 3; ++k) {
      spins[base + k * Nh] = cs[(int64_t)k * N + st.canon];
      if (cj) J[base + k * Nh] = cj[(int64_t)k * N + st.canon];
    }
  }
}

template <typename R>
__global__ __launch_bounds__(256) void export_kernel(int32_t L, const R* spins, const R* J, R* cs,
                                                     R* cj) {
  const int64_t N = (int64_t)L * L * L, Nh = N / 2;
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < N;
       e += (int64_t)gridDim.x * blockDim.x) {
    const SiteOf st = site_of(e, L);
    const int64_t base = (int64_t)3 * st.c * Nh + st.ic;
    for (int k = 0; k < 3; ++k) {
      if (cs) cs[(int64_t)k * N + st.canon] = spins[base + k * Nh];
      if (cj) cj[(int64_t)k * N + st.canon] = J[base + k * Nh];
    }
  }
}

// sigma <- sigma / |sigma| (length from a fused dot product, correctly rounded root
// and divisions).
template <typename R>
__global__ __launch_bounds__(256) void renormalise_kernel(int64_t Nh, int32_t colours,
                                                          R* spins) {
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < colours * Nh;
       e += (int64_t)gridDim.x * blockDim.x) {
    const int64_t c = e >= Nh ? 1 : 0;
    const int64_t base = 3 * c * Nh + (e - c * Nh);
    const Vec3<R> s{spins[base], spins[base + Nh], spins[base + 2 * Nh]};
    const R n = dev_sqrt(dot3(s, s));
    spins[base] = dev_div(s.x, n);
    spins[base + Nh] = dev_div(s.y, n);
    spins[base + 2 * Nh] = dev_div(s.z, n);
  }
}

// Writes the block's kReduceSlots partial sums (wave butterflies, then waves in order).
__device__ __forceinline__ void block_partials(double (&v)[kReduceSlots], int nslots,
                                               double* out) {
  __shared__ double part[kReduceThreads / 64][kReduceSlots];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  for (int k = 0; k < nslots; ++k) {
    const double s = wave_sum(v[k]);
    if (lane == 0) part[wave][k] = s;
  }
  __syncthreads();
  if (threadIdx.x < (unsigned)nslots) {
    double acc = 0.0;
    for (int w = 0; w < kReduceThreads / 64; ++w) acc += part[w][threadIdx.x];
    out[(int64_t)blockIdx.x * kReduceSlots + threadIdx.x] = acc;
  }
}

// Energy over the colour-0 sites: every bond has exactly one colour-0 end (L even),
// so H = -sum over colour-0 sites of sigma_i . h_i, all in binary64.
template <typename R>
__global__ __launch_bounds__(kReduceThreads) void energy_kernel(int32_t L, const R* spins,
                                                                const R* J, double* partials) {
  const int32_t Lh = L / 2;
  const int64_t Nh = (int64_t)Lh * L * L;
  double v[kReduceSlots] = {0.0};
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < Nh;
       e += (int64_t)gridDim.x * blockDim.x) {
    const SiteOf st = site_of(e, L);  // colour 0
    const double e_site = colour0_bond_sum(spins, J, Nh, L, Lh, st.xh, st.y, st.z);
    v[0] += e_site;
  }
  block_partials(v, 1, partials);
}

template <typename R>
__global__ __launch_bounds__(kReduceThreads) void overlap_kernel(int64_t N, const R* a,
                                                                 const R* b, double* partials) {
  const int64_t Nh = N / 2;
  double v[kReduceSlots] = {0.0};
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < N;
       e += (int64_t)gridDim.x * blockDim.x) {
    const int64_t c = e >= Nh ? 1 : 0;
    const int64_t base = 3 * c * Nh + (e - c * Nh);
    double av[3], bv[3];
    for (int k = 0; k < 3; ++k) {
      av[k] = (double)a[base + k * Nh];
      bv[k] = (double)b[base + k * Nh];
    }
    for (int m = 0; m < 3; ++m) {
      for (int n = 0; n < 3; ++n) v[3 * m + n] = fma(av[m], bv[n], v[3 * m + n]);
      v[9 + m] += av[m];
      v[12 + m] += bv[m];
    }
  }
  block_partials(v, 15, partials);
}

// out[k] = scale * sum over blocks of partials[block][k] (fixed order), k < nslots.
__global__ __launch_bounds__(kReduceThreads) void finish_reduce_kernel(const double* partials,
                                                                       int32_t nblocks,
                                                                       int32_t nslots,
                                                                       double scale, double* out) {
  __shared__ double part[kReduceThreads / 64];
  for (int k = 0; k < nslots; ++k) {
    double acc = 0.0;
    for (int32_t i = (int32_t)threadIdx.x; i < nblocks; i += kReduceThreads)
      acc += partials[(int64_t)i * kReduceSlots + k];
    const double s = wave_sum(acc);
    if ((threadIdx.x & 63) == 0) part[threadIdx.x >> 6] = s;
    __syncthreads();
    if (threadIdx.x == 0) {
      double tot = 0.0;
      for (int w = 0; w < kReduceThreads / 64; ++w) tot += part[w];
      out[k] = scale * tot;
    }
    __syncthreads();
  }
}

__global__ void zero_kernel(double* p, int64_t n) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    p[i] = 0.0;
}

__global__ void copy_double_kernel(const double* src, double* dst) { *dst = *src; }

}  // namespace

template <typename R>
hipError_t launch_init(int32_t L, uint64_t seed, void* spins, void* J, hipStream_t stream) {
  const int64_t N = (int64_t)L * L * L;
  hipLaunchKernelGGL(init_kernel<R>, dim3(grid_for(N, 256)), dim3(256), 0, stream, L,
                     (uint32_t)seed, (uint32_t)(seed >> 32), (R*)spins, (R*)J);
  return hipGetLastError();
}

template <typename R>
hipError_t launch_import(int32_t L, const R* canon_spins, const R* canon_J, void* spins, void* J,
                         hipStream_t stream) {
  const int64_t N = (int64_t)L * L * L;
  hipLaunchKernelGGL(import_kernel<R>, dim3(grid_for(N, 256)), dim3(256), 0, stream, L,
                     canon_spins, canon_J, (R*)spins, (R*)J);
  return hipGetLastError();
}

template <typename R>
hipError_t launch_export(int32_t L, const void* spins, const void* J, R* canon_spins, R* canon_J,
                         hipStream_t stream) {
  const int64_t N = (int64_t)L * L * L;
  hipLaunchKernelGGL(export_kernel<R>, dim3(grid_for(N, 256)), dim3(256), 0, stream, L,
                     (const R*)spins, (const R*)J, canon_spins, canon_J);
  return hipGetLastError();
}

template <typename R>
hipError_t launch_renormalise(int32_t L, void* spins, int32_t colours, hipStream_t stream) {
  const int64_t Nh = (int64_t)L * L * L / 2;
  hipLaunchKernelGGL(renormalise_kernel<R>, dim3(grid_for(colours * Nh, 256)), dim3(256), 0,
                     stream, Nh, colours, (R*)spins);
  return hipGetLastError();
}

static unsigned reduce_grid(int64_t n) {
  const int64_t b = (n + kReduceThreads - 1) / kReduceThreads;
  return (unsigned)(b < kReduceBlocks ? (b < 1 ? 1 : b) : kReduceBlocks);
}

template <typename R>
hipError_t launch_energy(int32_t L, const void* spins, const void* J, double* partials,
                         double* out, hipStream_t stream) {
  const int64_t Nh = (int64_t)L * L * L / 2;
  const unsigned nb = reduce_grid(Nh);
  hipLaunchKernelGGL(energy_kernel<R>, dim3(nb), dim3(kReduceThreads), 0, stream, L,
                     (const R*)spins, (const R*)J, partials);
  hipLaunchKernelGGL(finish_reduce_kernel, dim3(1), dim3(kReduceThreads), 0, stream,
                     (const double*)partials, (int32_t)nb, 1, -1.0, out);
  return hipGetLastError();
}

template <typename R>
hipError_t launch_overlap(int32_t L, const void* a, const void* b, double* partials, double* out,
                          hipStream_t stream) {
  const int64_t N = (int64_t)L * L * L;
  const unsigned nb = reduce_grid(N);
  hipLaunchKernelGGL(overlap_kernel<R>, dim3(nb), dim3(kReduceThreads), 0, stream, N,
                     (const R*)a, (const R*)b, partials);
  hipLaunchKernelGGL(finish_reduce_kernel, dim3(1), dim3(kReduceThreads), 0, stream,
                     (const double*)partials, (int32_t)nb, 15, 1.0 / (double)N, out);
  return hipGetLastError();
}

hipError_t launch_zero(double* p, int64_t n, hipStream_t stream) {
  hipLaunchKernelGGL(zero_kernel, dim3(grid_for(n, 256)), dim3(256), 0, stream, p, n);
  return hipGetLastError();
}

hipError_t launch_copy_double(const double* src, double* dst, hipStream_t stream) {
  hipLaunchKernelGGL(copy_double_kernel, dim3(1), dim3(1), 0, stream, src, dst);
  return hipGetLastError();
}

#define HSG_INSTANTIATE(R)                                                                     \
  template hipError_t launch_init<R>(int32_t, uint64_t, void*, void*, hipStream_t);           \
  template hipError_t launch_import<R>(int32_t, const R*, const R*, void*, void*, hipStream_t); \
  template hipError_t launch_export<R>(int32_t, const void*, const void*, R*, R*, hipStream_t); \
  template hipError_t launch_renormalise<R>(int32_t, void*, int32_t, hipStream_t);                     \
  template hipError_t launch_energy<R>(int32_t, const void*, const void*, double*, double*,   \
                                       hipStream_t);                                          \
  template hipError_t launch_overlap<R>(int32_t, const void*, const void*, double*, double*,  \
                                        hipStream_t);
HSG_INSTANTIATE(float)
HSG_INSTANTIATE(double)

}  // namespace hsg
