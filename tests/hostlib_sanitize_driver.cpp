// The host side of libhsg under AddressSanitizer and UndefinedBehaviorSanitizer (test
// infrastructure): every entry point with the arguments its checks must reject, the
// sizes of every lattice, the chain-table check and the tile table (host-only).  No call
// here reaches a kernel: lattices with placeholder device pointers are only passed with
// parameters the checks reject, and only when the machine has no GPU.  Exit status 0
// when every call returned what it should; 1 otherwise (the sanitizers abort on their
// own findings).
#include <hip/hip_runtime_api.h>

#include <cmath>
#include <cstdint>
#include <cstdio>
#include <limits>
#include <vector>

#include "hsg.h"

static int failures = 0;
#define EXPECT(cond)                                                                    \
  do {                                                                                  \
    if (!(cond)) {                                                                      \
      std::fprintf(stderr, "line %d: %s (last error: %s)\n", __LINE__, #cond,           \
                   hsg_last_error());                                                   \
      ++failures;                                                                       \
    }                                                                                   \
  } while (0)

static hsg_chain chain(int64_t s_off, int64_t j_off, int32_t L, int32_t k = 1, int32_t n_or = 0) {
  hsg_chain c{};
  c.spin_offset = s_off;
  c.J_offset = j_off;
  c.seed = 1;
  c.J_seed = 2;
  c.L = L;
  c.k_hits = k;
  c.n_or = n_or;
  return c;
}

static void sizes() {
  for (int32_t L : {-4, 0, 1, 2, 3, 8, 18, 64, 1024, 1290, 1291, 1292, 1 << 30,
                    std::numeric_limits<int32_t>::max()})
    for (int32_t dt : {HSG_F32, HSG_F64, 7, -1}) {
      size_t s = 1, j = 1, w = 1;
      const bool ok = L >= 2 && L <= HSG_L_MAX && L % 2 == 0 && (dt == HSG_F32 || dt == HSG_F64);
      EXPECT((hsg_lattice_bytes(L, dt, &s, &j, &w) == HSG_OK) == ok);
      if (ok) {
        const size_t n = (size_t)3 * L * L * L * (dt == HSG_F32 ? 4 : 8);
        EXPECT(s == n && j == n && w > 0);
      }
      EXPECT((hsg_lattice_bytes(L, dt, nullptr, nullptr, nullptr) == HSG_OK) == ok);
      EXPECT(hsg_last_error() != nullptr);
    }
}

static void lattice_calls(bool placeholders) {
  hsg_sweep_params good{0.5, 1, 1, 0, 0};
  EXPECT(hsg_init_lattice(nullptr, nullptr) == HSG_EINVAL);
  EXPECT(hsg_sweep(nullptr, &good, 1, nullptr) == HSG_EINVAL);
  EXPECT(hsg_energy(nullptr, 1, nullptr, nullptr) == HSG_EINVAL);
  EXPECT(hsg_overlap(nullptr, nullptr, nullptr, nullptr) == HSG_EINVAL);
  EXPECT(hsg_export(nullptr, nullptr, nullptr, nullptr) == HSG_EINVAL);
  EXPECT(hsg_import(nullptr, nullptr, nullptr, nullptr) == HSG_EINVAL);
  int32_t kinds[4];
  float ms[4];
  int32_t nrec = -1;
  EXPECT(hsg_sweep_timed(nullptr, &good, 1, nullptr, -1, kinds, ms, &nrec) == HSG_EINVAL);
  EXPECT(hsg_sweep_timed(nullptr, &good, 1, nullptr, 4, nullptr, ms, &nrec) == HSG_EINVAL);
  EXPECT(hsg_sweep_timed(nullptr, &good, 1, nullptr, 4, kinds, ms, &nrec) == HSG_EINVAL);
  EXPECT(hsg_sweep_noalloc(nullptr, &good, 1, nullptr) == HSG_EINVAL);
  // descriptors that fail their own checks (no device pointer is ever followed)
  hsg_lattice bad{};
  for (int32_t L : {0, 3, 1292}) {
    bad.L = L;
    bad.dtype = HSG_F32;
    EXPECT(hsg_init_lattice(&bad, nullptr) == HSG_EINVAL);
    EXPECT(hsg_sweep(&bad, &good, 1, nullptr) == HSG_EINVAL);
    EXPECT(hsg_sweep_noalloc(&bad, &good, 1, nullptr) == HSG_EINVAL);
  }
  bad.L = 8;
  bad.dtype = 5;
  EXPECT(hsg_sweep(&bad, &good, 1, nullptr) == HSG_EINVAL);
  bad.dtype = HSG_F32;  // spins, J, E still NULL
  EXPECT(hsg_sweep(&bad, &good, 1, nullptr) == HSG_EINVAL);
  EXPECT(hsg_energy(&bad, 0, nullptr, nullptr) == HSG_EINVAL);
  if (!placeholders) return;
  // a descriptor whose pointers are placeholders, only with parameters that are rejected
  hsg_lattice lat{};
  lat.L = 64;
  lat.dtype = HSG_F32;
  lat.spins = lat.J = (void*)0x1000;
  lat.E = (double*)0x2000;
  lat.work = (void*)0x4000;
  size_t s_b = 0, j_b = 0, w_b = 0;
  EXPECT(hsg_lattice_bytes(64, HSG_F32, &s_b, &j_b, &w_b) == HSG_OK);
  lat.work_bytes = w_b - s_b;  // the partials, not the second spin array of the phase launch
  const double inf = std::numeric_limits<double>::infinity();
  const double nan = std::numeric_limits<double>::quiet_NaN();
  std::vector<hsg_sweep_params> rejected = {
      {0.0, 1, 0, 0, 0},       {-1.0, 1, 0, 0, 0},      {nan, 1, 0, 0, 0},
      {0.5, 0, 0, 0, 0},       {0.5, -1, 1, 0, 0},      {0.5, 1, -1, 0, 0},
      {0.5, 70000, 0, 0, 0},   {0.5, 1, 40000, 0, 0},   {0.5, 1, 0, -1, 0},
      {0.5, 1, 0, 0, 1 << 20}, {0.5, 1, 0, 0, HSG_MARCH_PHASE},
      {inf, 1, 0, 0, HSG_FUSED | HSG_PHASE_MC}};
  for (const auto& p : rejected) {
    EXPECT(hsg_sweep(&lat, &p, 1, nullptr) == HSG_EINVAL);
    EXPECT(hsg_sweep_noalloc(&lat, &p, 1, nullptr) == HSG_EINVAL);
    EXPECT(hsg_sweep_timed(&lat, &p, 1, nullptr, 4, kinds, ms, &nrec) == HSG_EINVAL);
  }
  EXPECT(hsg_sweep(&lat, nullptr, 1, nullptr) == HSG_EINVAL);
  EXPECT(hsg_sweep(&lat, &good, -1, nullptr) == HSG_EINVAL);
  lat.sweep = 0xFFFFFFFFull;  // the 32-bit sweep counter would wrap
  EXPECT(hsg_sweep(&lat, &good, 2, nullptr) == HSG_EINVAL);
  lat.sweep = 0;
  hsg_lattice big = lat;
  big.L = 600;  // beyond HSG_NOALLOC_L_MAX
  EXPECT(hsg_sweep_noalloc(&big, &good, 1, nullptr) == HSG_EINVAL);
  hsg_sweep_params phase{0.5, 1, 1, 0, HSG_PHASE_MC};
  EXPECT(hsg_sweep_noalloc(&lat, &phase, 1, nullptr) == HSG_EINVAL);
  EXPECT(hsg_sweep(&lat, &phase, 1, nullptr) == HSG_EINVAL);  // no second spin array
  hsg_lattice other = lat;
  other.L = 32;
  EXPECT(hsg_overlap(&lat, &other, (double*)0x3000, nullptr) == HSG_EINVAL);
  EXPECT(hsg_overlap_fourier(&lat, &other, (double*)0x3000, nullptr) == HSG_EINVAL);
  EXPECT(hsg_energy(&lat, 1, nullptr, nullptr) == HSG_EINVAL);
  EXPECT(hsg_import(&lat, nullptr, nullptr, nullptr) == HSG_EINVAL);
  EXPECT(hsg_export(&lat, nullptr, nullptr, nullptr) == HSG_OK);  // nothing to do
}

static void chain_tables() {
  const int64_t big = std::numeric_limits<int64_t>::max();
  std::vector<hsg_chain> t = {chain(0, 0, 8), chain(3 * 512, 0, 8, 4, 1), chain(3 * 1024, 0, 16)};
  const int64_t s_el = 3 * 1024 + 3 * 4096, j_el = 3 * 4096;
  EXPECT(hsg_batch_check(t.data(), 3, s_el, j_el) == HSG_OK);
  EXPECT(hsg_batch_check(nullptr, 3, s_el, j_el) == HSG_EINVAL);
  EXPECT(hsg_batch_check(t.data(), 0, s_el, j_el) == HSG_EINVAL);
  EXPECT(hsg_batch_check(t.data(), 3, s_el - 1, j_el) == HSG_EINVAL);
  auto with = [&](int i, hsg_chain c) {
    std::vector<hsg_chain> u = t;
    u[i] = c;
    return hsg_batch_check(u.data(), 3, s_el, j_el);
  };
  EXPECT(with(1, chain(3 * 512 - 1, 0, 8)) == HSG_EINVAL);  // overlaps chain 0
  EXPECT(with(1, chain(-3, 0, 8)) == HSG_EINVAL);
  EXPECT(with(1, chain(big - 10, 0, 8)) == HSG_EINVAL);   // offset + size past int64
  EXPECT(with(1, chain(3 * 512, big - 10, 8)) == HSG_EINVAL);
  EXPECT(with(1, chain(3 * 512, 0, 7)) == HSG_EINVAL);
  EXPECT(with(1, chain(3 * 512, 0, HSG_BATCH_L_MAX + 2)) == HSG_EINVAL);
  EXPECT(with(1, chain(3 * 512, 0, 8, 0, 0)) == HSG_EINVAL);
  EXPECT(with(1, chain(3 * 512, 0, 8, 70000, 0)) == HSG_EINVAL);
  hsg_chain f = chain(3 * 512, 0, 8);
  f.flags = 1 << 20;
  EXPECT(with(1, f) == HSG_EINVAL);
  f = chain(3 * 512, 0, 8);
  f.reserved = 1;
  EXPECT(with(1, f) == HSG_EINVAL);
}

static void tiles() {
  std::vector<hsg_chain> t = {chain(0, 0, 8), chain(3 * 512, 0, 16), chain(0, 0, 24)};
  const int32_t active[3] = {0, 1, 2};
  // colour sites: 256, 2048, 6912; tiles of 256: 1 + 8 + 27 = 36
  std::vector<int32_t> out(2 * 64, -7);
  int32_t n = -1;
  EXPECT(hsg_batch_tiles(t.data(), 3, active, 3, 256, out.data(), 36, &n) == HSG_OK && n == 36);
  EXPECT(out[0] == 0 && out[1] == 0 && out[2] == 1 && out[3] == 0 && out[4] == 1 &&
         out[5] == 256 && out[2 * 35] == 2 && out[2 * 35 + 1] == 6912 - 256);
  EXPECT(hsg_batch_tiles(t.data(), 3, active, 3, 256, out.data(), 35, &n) == HSG_EINVAL);
  EXPECT(hsg_batch_tiles(t.data(), 3, active, 3, 1024, out.data(), 64, &n) == HSG_OK &&
         n == 1 + 2 + 7);
  EXPECT(hsg_batch_tiles(t.data(), 3, active, 0, 256, out.data(), 64, &n) == HSG_OK && n == 0);
  const int32_t out_of_range[1] = {3};
  EXPECT(hsg_batch_tiles(t.data(), 3, out_of_range, 1, 256, out.data(), 64, &n) == HSG_EINVAL);
  for (int32_t ts : {0, 32, 100, 2048})
    EXPECT(hsg_batch_tiles(t.data(), 3, active, 3, ts, out.data(), 64, &n) == HSG_EINVAL);
  EXPECT(hsg_batch_tiles(nullptr, 3, active, 3, 256, out.data(), 64, &n) == HSG_EINVAL);
  EXPECT(hsg_batch_tiles(t.data(), 3, active, 3, 256, out.data(), -1, &n) == HSG_EINVAL);
}

static void batch_calls() {
  hsg_batch b{};
  EXPECT(hsg_batch_init(nullptr, nullptr) == HSG_EINVAL);
  EXPECT(hsg_batch_init(&b, nullptr) == HSG_EINVAL);  // n_chains 0, buffers NULL
  b.n_chains = 4;
  b.dtype = HSG_F32;
  EXPECT(hsg_batch_sweep(&b, 1, nullptr) == HSG_EINVAL);
  EXPECT(hsg_batch_energy(&b, nullptr, nullptr) == HSG_EINVAL);
  EXPECT(hsg_batch_overlap(&b, nullptr, 1, nullptr, nullptr) == HSG_EINVAL);
  EXPECT(hsg_batch_pass_sweep(&b, nullptr, 1, 256, 0, 0, 1, nullptr) == HSG_EINVAL);
  hsg_pt pt{};
  EXPECT(hsg_pt_exchange(nullptr, &b, nullptr) == HSG_EINVAL);
  EXPECT(hsg_pt_exchange(&pt, &b, nullptr) == HSG_EINVAL);  // no ladders
  pt.n_ladders = 1;
  pt.n_temps = 70000;
  EXPECT(hsg_pt_overlap(&pt, &b, nullptr, 1, nullptr, nullptr) == HSG_EINVAL);
}

int main() {
  int devices = 0;
  const bool gpu = hipGetDeviceCount(&devices) == hipSuccess && devices > 0;
  sizes();
  lattice_calls(!gpu);
  chain_tables();
  tiles();
  batch_calls();
  std::printf("%d failed expectations%s\n", failures,
              gpu ? " (a GPU is present: placeholder-pointer calls skipped)" : "");
  return failures ? 1 : 0;
}
