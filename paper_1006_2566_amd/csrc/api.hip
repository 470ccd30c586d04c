// C interface of libhsg (declared and documented in include/hsg.h): argument
// validation, the sweep schedule, and error reporting.  Every entry point returns a
// status code and never throws; kernels are only enqueued on the caller's stream.
#include <math.h>
#include <stdarg.h>
#include <stdio.h>

#include <algorithm>
#include <mutex>
#include <utility>
#include <vector>

#include "hsg.h"
#include "hsg_internal.h"

namespace {

thread_local char g_last_error[512] = "";

int fail(int code, const char* fmt, ...) {
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(g_last_error, sizeof g_last_error, fmt, ap);
  va_end(ap);
  return code;
}

int device_status(hipError_t e, const char* what) {
  if (e == hipSuccess) return HSG_OK;
  return fail(HSG_EDEVICE, "%s: %s", what, hipGetErrorString(e));
}

int check_dims(int32_t L, int32_t dtype) {
  if (L < 2 || L > HSG_L_MAX || (L & 1))
    return fail(HSG_EINVAL, "L must be even with 2 <= L <= %d (got %d)", HSG_L_MAX, (int)L);
  if (dtype != HSG_F32 && dtype != HSG_F64)
    return fail(HSG_EINVAL, "dtype must be HSG_F32 or HSG_F64 (got %d)", (int)dtype);
  return HSG_OK;
}

int check_lattice(const hsg_lattice* lat) {
  if (!lat) return fail(HSG_EINVAL, "lattice descriptor is NULL");
  int rc = check_dims(lat->L, lat->dtype);
  if (rc) return rc;
  if (!lat->spins || !lat->J || !lat->E || !lat->work)
    return fail(HSG_EINVAL, "lattice buffers spins, J, E and work must all be set");
  const size_t need = hsg::work_bytes_for(lat->L);
  if (lat->work_bytes < need)
    return fail(HSG_EINVAL, "work buffer too small: %zu bytes, need %zu", lat->work_bytes, need);
  return HSG_OK;
}

hipStream_t as_stream(void* s) { return (hipStream_t)s; }

// Launch recorder of hsg_sweep_timed: while one is set (per calling thread), every
// launch of a sweep is bracketed by two events recorded on the launch stream, up to
// `capacity` launches; later launches run unrecorded.
struct LaunchRecorder {
  int32_t capacity = 0, count = 0;
  int32_t* kinds = nullptr;
  std::vector<hipEvent_t> events;  // 2 per recorded launch
  hipError_t err = hipSuccess;     // first event failure
};
thread_local LaunchRecorder* g_recorder = nullptr;

// Enqueues launch() (returning hipError_t), bracketed by events when a recorder is set.
template <class F>
hipError_t recorded(int32_t kind, hipStream_t st, F&& launch) {
  LaunchRecorder* r = g_recorder;
  if (!r || r->count >= r->capacity || r->err != hipSuccess) return launch();
  hipEvent_t ev[2] = {nullptr, nullptr};
  hipError_t e = hipEventCreate(&ev[0]);
  if (e == hipSuccess) e = hipEventCreate(&ev[1]);
  if (e == hipSuccess) e = hipEventRecord(ev[0], st);
  if (e != hipSuccess) {
    for (hipEvent_t x : ev)
      if (x) (void)hipEventDestroy(x);
    r->err = e;
    return launch();
  }
  const hipError_t le = launch();
  e = hipEventRecord(ev[1], st);
  r->events.push_back(ev[0]);
  r->events.push_back(ev[1]);
  r->kinds[r->count++] = kind;
  if (e != hipSuccess) r->err = e;
  return le;
}

int check_params(const hsg_sweep_params* p) {
  if (!p) return fail(HSG_EINVAL, "sweep parameters are NULL");
  if (!(p->T > 0.0)) return fail(HSG_EINVAL, "T must be > 0 (INFINITY for beta = 0), got %g", p->T);
  if (p->k_hits < 0 || p->n_or < 0 || p->k_hits + p->n_or < 1)
    return fail(HSG_EINVAL, "need k_hits >= 0, n_or >= 0 and k_hits + n_or >= 1");
  if (p->n_or > 0x7FFF || p->k_hits > 0xFFFF)
    return fail(HSG_EINVAL, "k_hits must be < 65536 and n_or < 32768");
  if (p->renorm_every < 0) return fail(HSG_EINVAL, "renorm_every must be >= 0");
  if (p->flags & ~(HSG_HEAT_BATH | HSG_SNAKE | HSG_FUSED | HSG_MARCH_PHASE | HSG_PLANE_LAUNCH |
                   HSG_STREAM_LOADS | HSG_PHASE_LAUNCH | HSG_PHASE_MC))
    return fail(HSG_EINVAL, "unknown flags 0x%x", (unsigned)p->flags);
  if ((p->flags & HSG_MARCH_PHASE) && !(p->flags & HSG_FUSED))
    return fail(HSG_EINVAL, "HSG_MARCH_PHASE needs HSG_FUSED");
  if ((p->flags & HSG_FUSED) &&
      (p->flags & (HSG_PLANE_LAUNCH | HSG_STREAM_LOADS | HSG_PHASE_LAUNCH | HSG_PHASE_MC)))
    return fail(HSG_EINVAL, "HSG_PLANE_LAUNCH, HSG_STREAM_LOADS, HSG_PHASE_LAUNCH and HSG_PHASE_MC "
                            "apply to the pass-by-pass schedule, not to HSG_FUSED");
  return HSG_OK;
}

// The colour passes of a sweep ("stages"): the Monte Carlo phase's colour-0 and
// colour-1 passes (k_hits > 0), then two per over-relaxation phase.
int32_t stages_per_sweep(const hsg_sweep_params* p) {
  return 2 * ((p->k_hits > 0 ? 1 : 0) + p->n_or);
}

bool renorm_due(const hsg_sweep_params* p, uint64_t sweep) {
  return p->renorm_every > 0 && (sweep + 1) % (uint64_t)p->renorm_every == 0;
}

// Pass-by-pass schedule: one launch per colour pass over the whole lattice, or with
// HSG_PLANE_LAUNCH one launch per z slab of tiles (one z plane from L = 64 up).  With
// HSG_PHASE_LAUNCH each over-relaxation phase is one launch reading one spin array and
// writing the other (the lattice's and the work buffer's second one); when a call would
// run an odd number of them, its last phase (never one that carries a Monte Carlo pass)
// runs as two colour passes in place instead, so the spins end in the lattice's own
// array without a copy (two passes cost less than a phase launch plus a copy of the
// lattice).  With HSG_PHASE_MC
// the launch of a sweep's last over-relaxation phase also runs the colour-0 Monte Carlo
// pass of the next sweep of the call (and the renormalisation between them when due);
// that sweep then starts with its colour-1 pass.
template <typename R>
int sweep_plain(hsg_lattice* lat, const hsg_sweep_params* p, int32_t n_sweeps, hipStream_t st,
                double* partials) {
  using namespace hsg;
  const Geometry g = pass_geometry(lat->L);
  const int64_t Nh = (int64_t)lat->L * lat->L * lat->L / 2;
  PassArgs<R> a{};
  const bool phase_launch =
      (p->flags & (HSG_PHASE_LAUNCH | HSG_PHASE_MC)) && phase_supported(lat->L);
  R* bufs[2] = {(R*)lat->spins,
                phase_launch ? (R*)((char*)lat->work + fused_offset(lat->L)) : nullptr};
  int cur = 0;  // buffer holding the current spins (phase launches flip it)
  const bool phase_mc = phase_launch && (p->flags & HSG_PHASE_MC) && p->k_hits > 0;
  // an odd count of phase launches: the call's last phase runs as colour passes
  const bool last_as_passes =
      phase_launch && (((int64_t)n_sweeps * p->n_or) & 1) != 0;
  PhaseArgs<R> ph{};
  ph.J = (const R*)lat->J;
  ph.beta = (R)(1.0 / p->T);
  ph.seed_lo = (uint32_t)lat->seed;
  ph.seed_hi = (uint32_t)(lat->seed >> 32);
  ph.k_hits = p->k_hits;
  ph.L = lat->L;
  a.spins = planes_of<R>(bufs[cur], Nh);
  a.J = planes_of<R>(lat->J, Nh);
  a.partials = partials;
  a.beta = (R)(1.0 / p->T);
  a.seed_lo = (uint32_t)lat->seed;
  a.seed_hi = (uint32_t)(lat->seed >> 32);
  a.k_hits = p->k_hits;
  a.g = g;
  a.nt = (p->flags & HSG_STREAM_LOADS) ? 1 : 0;
  const PassMode mc = (p->flags & HSG_HEAT_BATH) ? PassMode::HeatBath : PassMode::Metropolis;
  ph.mc_mode = (int32_t)mc;
  ph.partials = partials;
  const bool snake = (p->flags & HSG_SNAKE) != 0;
  const bool by_slab = (p->flags & HSG_PLANE_LAUNCH) != 0;
  const int32_t slab_tiles = g.tiles_x * g.tiles_y;
  int32_t pass_count = 0;
  bool mc0_done = false;  // this sweep's colour-0 Monte Carlo pass ran in the last launch
  for (int32_t n = 0; n < n_sweeps; ++n) {
    const uint64_t sweep = lat->sweep + (uint64_t)n;
    a.sweep = (uint32_t)sweep;
    bool renorm_done = false;
    for (int32_t phase = 0; phase <= p->n_or; ++phase) {
      if (phase == 0 && p->k_hits == 0) continue;
      a.phase = (uint32_t)phase;
      const bool last_phase = n + 1 == n_sweeps && phase == p->n_or;
      if (phase_launch && phase > 0 && !(last_as_passes && last_phase)) {
        const bool then_mc = phase_mc && phase == p->n_or && n + 1 < n_sweeps;
        ph.in = bufs[cur];
        ph.out = bufs[1 - cur];
        ph.sweep = (uint32_t)sweep;
        ph.phase = (uint32_t)phase;
        ph.then_mc = then_mc ? 1 : 0;
        ph.mc_sweep = (uint32_t)(sweep + 1);
        ph.renorm = then_mc && renorm_due(p, sweep) ? 1 : 0;
        int rc = device_status(
            recorded(then_mc ? HSG_LAUNCH_OR_PHASE_MC : HSG_LAUNCH_OR_PHASE, st,
                     [&] { return launch_phase<R>(ph, st); }),
            "phase launch");
        if (rc) return rc;
        cur = 1 - cur;
        a.spins = planes_of<R>(bufs[cur], Nh);
        pass_count += 2;
        mc0_done = then_mc;
        renorm_done = ph.renorm != 0;
        continue;
      }
      for (int32_t colour = 0; colour < 2; ++colour) {
        a.colour = colour;
        a.reverse = snake ? (pass_count & 1) : 0;
        ++pass_count;
        if (phase == 0 && colour == 0 && mc0_done) {
          mc0_done = false;
          continue;
        }
        const PassMode mode = phase == 0 ? mc : PassMode::OverRelax;
        if (!by_slab) {
          a.tile_base = 0;
          a.tile_count = g.n_blocks;
          int rc = device_status(
              recorded(mode == PassMode::OverRelax ? HSG_LAUNCH_OR_PASS : HSG_LAUNCH_MC_PASS, st,
                       [&] { return launch_colour_pass<R>(mode, a, st); }),
              "colour pass");
          if (rc) return rc;
          continue;
        }
        for (int32_t i = 0; i < g.tiles_z; ++i) {
          const int32_t tz = a.reverse ? g.tiles_z - 1 - i : i;
          a.tile_base = tz * slab_tiles;
          a.tile_count = slab_tiles;
          int rc = device_status(
              recorded(mode == PassMode::OverRelax ? HSG_LAUNCH_OR_PASS : HSG_LAUNCH_MC_PASS, st,
                       [&] { return launch_colour_pass<R>(mode, a, st); }),
              "colour pass (slab)");
          if (rc) return rc;
        }
      }
    }
    if (renorm_due(p, sweep) && !renorm_done) {
      int rc = device_status(recorded(HSG_LAUNCH_OTHER, st,
                                      [&] { return launch_renormalise<R>(lat->L, bufs[cur], 2, st); }),
                             "renormalise");
      if (rc) return rc;
    }
  }
  if (cur != 0) return fail(HSG_EDEVICE, "internal: spins left in the second array");
  return HSG_OK;
}

// Fused schedule: the call's stages, sweep after sweep, cut into launches of at most
// march_max_stages passes.  The first launch stops after the first Monte Carlo phase,
// so that later launches end with one (its passes then carry the smallest halos, the
// cheapest place for the expensive passes).  Each launch reads one spin array and
// writes the other; renormalisation is folded into the passes: colour-1 spins right
// after their last update of the sweep, colour-0 spins just before their first update
// of the next sweep (or by a colour-0 pass at the end of the call).
template <typename R>
int sweep_fused(hsg_lattice* lat, const hsg_sweep_params* p, int32_t n_sweeps, hipStream_t st) {
  using namespace hsg;
  if (march_blocks(lat->L) > pass_geometry(lat->L).n_blocks)
    return fail(HSG_EUNSUPPORTED, "fused passes: more workgroups than energy partials");
  const int32_t per = stages_per_sweep(p);
  const int64_t total = (int64_t)per * n_sweeps;
  const int32_t smax = (p->flags & HSG_MARCH_PHASE) ? 2 : march_max_stages<R>();
  const PassMode mc = (p->flags & HSG_HEAT_BATH) ? PassMode::HeatBath : PassMode::Metropolis;
  const int32_t first_phase = p->k_hits > 0 ? 0 : 1;
  MarchArgs<R> a{};
  a.J = (const R*)lat->J;
  a.partials = pass_partials(lat->work);
  a.beta = (R)(1.0 / p->T);
  a.seed_lo = (uint32_t)lat->seed;
  a.seed_hi = (uint32_t)(lat->seed >> 32);
  a.k_hits = p->k_hits;
  a.L = lat->L;
  R* bufs[2] = {(R*)lat->spins, (R*)((char*)lat->work + fused_offset(lat->L))};
  int cur = 0;
  int64_t g = 0;
  bool first = true;
  while (g < total) {
    int64_t n = (first && p->k_hits > 0 && per > 2) ? 2 : smax;
    if (n > total - g) n = total - g;
    first = false;
    for (int32_t i = 0; i < (int32_t)n; ++i) {
      const int64_t gi = g + i;
      const uint64_t sweep = lat->sweep + (uint64_t)(gi / per);
      const int32_t s = (int32_t)(gi % per);
      const int32_t phase = first_phase + s / 2;
      MarchStage& m = a.st[i];
      m.mode = (int32_t)(phase == 0 ? mc : PassMode::OverRelax);
      m.colour = s & 1;
      m.sweep = (uint32_t)sweep;
      m.phase = (uint32_t)phase;
      m.renorm_before = (s == 0 && gi >= per && renorm_due(p, sweep - 1)) ? 1 : 0;
      m.renorm_after = (s == per - 1 && renorm_due(p, sweep)) ? 1 : 0;
    }
    a.in = bufs[cur];
    a.out = bufs[1 - cur];
    int rc = device_status(
        recorded(HSG_LAUNCH_MARCH, st, [&] { return launch_march<R>(a, (int32_t)n, st); }),
        "fused passes");
    if (rc) return rc;
    cur = 1 - cur;
    g += n;
  }
  const size_t bytes = (size_t)3 * lat->L * lat->L * lat->L * sizeof(R);
  if (cur != 0) {
    int rc = device_status(hipMemcpyAsync(lat->spins, bufs[cur], bytes, hipMemcpyDeviceToDevice, st),
                           "copy spins");
    if (rc) return rc;
  }
  if (n_sweeps > 0 && renorm_due(p, lat->sweep + (uint64_t)n_sweeps - 1)) {
    int rc = device_status(launch_renormalise<R>(lat->L, lat->spins, 1, st), "renormalise");
    if (rc) return rc;
  }
  return HSG_OK;
}

bool use_fused(const hsg_lattice* lat, const hsg_sweep_params* p) {
  return (p->flags & HSG_FUSED) && hsg::march_supported(lat->L);
}

// partials: the per-tile energy-change partials (pass_geometry(L).n_blocks doubles, zero
// on entry and zeroed again by the fold).
template <typename R>
int sweep_impl(hsg_lattice* lat, const hsg_sweep_params* p, int32_t n_sweeps, hipStream_t st,
               double* partials) {
  using namespace hsg;
  int rc = use_fused(lat, p) ? sweep_fused<R>(lat, p, n_sweeps, st)
                             : sweep_plain<R>(lat, p, n_sweeps, st, partials);
  if (rc) return rc;
  if (n_sweeps > 0 && p->k_hits > 0) {
    rc = device_status(recorded(HSG_LAUNCH_OTHER, st,
                                [&] {
                                  return launch_fold_partials(partials,
                                                              pass_geometry(lat->L).n_blocks,
                                                              lat->E, st);
                                }),
                       "fold");
    if (rc) return rc;
  }
  return HSG_OK;
}

// Clears the pass partials and sets *E = H.
template <typename R>
int reset_energy(hsg_lattice* lat, hipStream_t st) {
  using namespace hsg;
  int rc = device_status(launch_zero(pass_partials(lat->work), pass_geometry(lat->L).n_blocks, st),
                         "clear scratch");
  if (rc) return rc;
  return device_status(launch_energy<R>(lat->L, lat->spins, lat->J,
                                        reduce_partials(lat->work, lat->L), lat->E, st),
                       "energy");
}

}  // namespace

extern "C" {

const char* hsg_last_error(void) { return g_last_error; }

int hsg_lattice_bytes(int32_t L, int32_t dtype, size_t* spin_bytes, size_t* J_bytes,
                      size_t* work_bytes) {
  int rc = check_dims(L, dtype);
  if (rc) return rc;
  const size_t elem = dtype == HSG_F32 ? 4 : 8;
  const size_t n = (size_t)3 * L * L * L;
  if (spin_bytes) *spin_bytes = n * elem;
  if (J_bytes) *J_bytes = n * elem;
  if (work_bytes) *work_bytes = hsg::work_bytes_for(L, (int32_t)elem);
  return HSG_OK;
}

int hsg_init_lattice(hsg_lattice* lat, void* stream) {
  int rc = check_lattice(lat);
  if (rc) return rc;
  hipStream_t st = as_stream(stream);
  if (lat->dtype == HSG_F32) {
    rc = device_status(hsg::launch_init<float>(lat->L, lat->seed, lat->spins, lat->J, st), "init");
    return rc ? rc : reset_energy<float>(lat, st);
  }
  rc = device_status(hsg::launch_init<double>(lat->L, lat->seed, lat->spins, lat->J, st), "init");
  return rc ? rc : reset_energy<double>(lat, st);
}

int hsg_import(hsg_lattice* lat, const void* canon_spins, const void* canon_J, void* stream) {
  int rc = check_lattice(lat);
  if (rc) return rc;
  if (!canon_spins) return fail(HSG_EINVAL, "canon_spins is NULL");
  hipStream_t st = as_stream(stream);
  if (lat->dtype == HSG_F32) {
    rc = device_status(hsg::launch_import<float>(lat->L, (const float*)canon_spins,
                                                 (const float*)canon_J, lat->spins, lat->J, st),
                       "import");
    return rc ? rc : reset_energy<float>(lat, st);
  }
  rc = device_status(hsg::launch_import<double>(lat->L, (const double*)canon_spins,
                                                (const double*)canon_J, lat->spins, lat->J, st),
                     "import");
  return rc ? rc : reset_energy<double>(lat, st);
}

int hsg_export(const hsg_lattice* lat, void* canon_spins, void* canon_J, void* stream) {
  int rc = check_lattice(lat);
  if (rc) return rc;
  if (!canon_spins && !canon_J) return HSG_OK;
  hipStream_t st = as_stream(stream);
  if (lat->dtype == HSG_F32)
    return device_status(hsg::launch_export<float>(lat->L, lat->spins, lat->J, (float*)canon_spins,
                                                   (float*)canon_J, st),
                         "export");
  return device_status(hsg::launch_export<double>(lat->L, lat->spins, lat->J,
                                                  (double*)canon_spins, (double*)canon_J, st),
                       "export");
}

static int sweep_checked(hsg_lattice* lat, const hsg_sweep_params* p, int32_t n_sweeps,
                         void* stream);

int hsg_sweep(hsg_lattice* lat, const hsg_sweep_params* p, int32_t n_sweeps, void* stream) {
  return sweep_checked(lat, p, n_sweeps, stream);
}

int hsg_sweep_timed(hsg_lattice* lat, const hsg_sweep_params* p, int32_t n_sweeps, void* stream,
                    int32_t capacity, int32_t* kinds, float* ms, int32_t* n_recorded) {
  if (capacity < 0 || (capacity > 0 && (!kinds || !ms)) || !n_recorded)
    return fail(HSG_EINVAL, "hsg_sweep_timed: bad capacity or output arrays");
  if (g_recorder) return fail(HSG_EINVAL, "hsg_sweep_timed: nested call");
  LaunchRecorder rec;
  rec.capacity = capacity;
  rec.kinds = kinds;
  rec.events.reserve((size_t)2 * (size_t)capacity);
  g_recorder = &rec;
  int rc = sweep_checked(lat, p, n_sweeps, stream);
  g_recorder = nullptr;
  *n_recorded = rec.count;
  if (rc == HSG_OK && rec.err != hipSuccess) rc = device_status(rec.err, "timing events");
  if (rc == HSG_OK && rec.count > 0)
    rc = device_status(hipEventSynchronize(rec.events.back()), "timing events");
  for (int32_t i = 0; rc == HSG_OK && i < rec.count; ++i)
    rc = device_status(hipEventElapsedTime(&ms[i], rec.events[2 * i], rec.events[2 * i + 1]),
                       "timing events");
  if (rc != HSG_OK) (void)hipStreamSynchronize(as_stream(stream));  // events idle before destroy
  for (hipEvent_t e : rec.events) (void)hipEventDestroy(e);
  return rc;
}

static int sweep_checked(hsg_lattice* lat, const hsg_sweep_params* p, int32_t n_sweeps,
                         void* stream) {
  int rc = check_lattice(lat);
  if (rc) return rc;
  rc = check_params(p);
  if (rc) return rc;
  if (n_sweeps < 0) return fail(HSG_EINVAL, "n_sweeps must be >= 0");
  if (lat->sweep + (uint64_t)n_sweeps > 0x100000000ull)
    return fail(HSG_EINVAL, "sweep index would pass 2^32");
  const size_t elem = lat->dtype == HSG_F32 ? 4 : 8;
  if (use_fused(lat, p) && lat->work_bytes < hsg::work_bytes_for(lat->L, (int32_t)elem))
    return fail(HSG_EINVAL, "HSG_FUSED needs a work buffer of %zu bytes (has %zu)",
                hsg::work_bytes_for(lat->L, (int32_t)elem), lat->work_bytes);
  if ((p->flags & (HSG_PHASE_LAUNCH | HSG_PHASE_MC)) && hsg::phase_supported(lat->L) &&
      p->n_or > 0 && lat->work_bytes < hsg::work_bytes_for(lat->L, (int32_t)elem))
    return fail(HSG_EINVAL, "HSG_PHASE_LAUNCH and HSG_PHASE_MC need a work buffer of %zu bytes "
                            "(has %zu)",
                hsg::work_bytes_for(lat->L, (int32_t)elem), lat->work_bytes);
  hipStream_t st = as_stream(stream);
  double* partials = hsg::pass_partials(lat->work);
  rc = lat->dtype == HSG_F32 ? sweep_impl<float>(lat, p, n_sweeps, st, partials)
                             : sweep_impl<double>(lat, p, n_sweeps, st, partials);
  if (rc == HSG_OK) lat->sweep += (uint64_t)n_sweeps;
  return rc;
}

/* ---------------------------------------------------- sweeps without a work buffer */

// The library's own scratch for hsg_sweep_noalloc: the per-tile energy partials of the
// pass-by-pass schedule for lattices up to HSG_NOALLOC_L_MAX, one copy per GPU (the array
// lives in every device's copy of the code object until the process ends).  Host code
// uses the device address hipGetSymbolAddress returns for the current device, never the
// array's name.
constexpr size_t kNoAllocPartials = HSG_NOALLOC_SCRATCH_BYTES / sizeof(double);
static __device__ __align__(256) double scratch[kNoAllocPartials];

constexpr int kMaxDevices = 64;
static std::mutex g_scratch_mutex;
static double* g_scratch_ptr[kMaxDevices];

// The current device's address of `scratch` (looked up once per device).
static int scratch_for_current_device(double** out) {
  int dev = -1;
  int rc = device_status(hipGetDevice(&dev), "hipGetDevice");
  if (rc) return rc;
  if (dev < 0 || dev >= kMaxDevices)
    return fail(HSG_EUNSUPPORTED, "hsg_sweep_noalloc: device %d beyond the first %d", dev,
                kMaxDevices);
  std::lock_guard<std::mutex> lock(g_scratch_mutex);
  if (!g_scratch_ptr[dev]) {
    void* ptr = nullptr;
    rc = device_status(hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)), "hipGetSymbolAddress");
    if (rc) return rc;
    if (!ptr) return fail(HSG_EDEVICE, "hipGetSymbolAddress returned NULL for the scratch array");
    g_scratch_ptr[dev] = (double*)ptr;
  }
  *out = g_scratch_ptr[dev];
  return HSG_OK;
}

int hsg_sweep_noalloc(hsg_lattice* lat, const hsg_sweep_params* p, int32_t n_sweeps,
                      void* stream) {
  if (!lat) return fail(HSG_EINVAL, "lattice descriptor is NULL");
  int rc = check_dims(lat->L, lat->dtype);
  if (rc) return rc;
  if (!lat->spins || !lat->J || !lat->E)
    return fail(HSG_EINVAL, "lattice buffers spins, J and E must be set");
  if (lat->L > HSG_NOALLOC_L_MAX)
    return fail(HSG_EINVAL, "hsg_sweep_noalloc: L = %d beyond HSG_NOALLOC_L_MAX = %d", (int)lat->L,
                HSG_NOALLOC_L_MAX);
  rc = check_params(p);
  if (rc) return rc;
  if (p->flags & (HSG_FUSED | HSG_MARCH_PHASE | HSG_PHASE_LAUNCH | HSG_PHASE_MC))
    return fail(HSG_EINVAL, "hsg_sweep_noalloc runs the pass-by-pass schedule: HSG_FUSED, "
                            "HSG_MARCH_PHASE, HSG_PHASE_LAUNCH and HSG_PHASE_MC need a second "
                            "spin array");
  if (n_sweeps < 0) return fail(HSG_EINVAL, "n_sweeps must be >= 0");
  if (lat->sweep + (uint64_t)n_sweeps > 0x100000000ull)
    return fail(HSG_EINVAL, "sweep index would pass 2^32");
  const int32_t n_blocks = hsg::pass_geometry(lat->L).n_blocks;
  if ((size_t)n_blocks > kNoAllocPartials)
    return fail(HSG_EINVAL, "hsg_sweep_noalloc: %d partials exceed the scratch array",
                (int)n_blocks);
  double* partials = nullptr;
  rc = scratch_for_current_device(&partials);
  if (rc) return rc;
  hipStream_t st = as_stream(stream);
  // the array keeps the last call's contents: the partials must start at zero (a fill
  // kernel, not a memset node, so the call can be captured in a graph)
  rc = device_status(hsg::launch_zero(partials, n_blocks, st), "clear scratch");
  if (rc) return rc;
  hsg_lattice view = *lat;  // the pass-by-pass schedule never touches work
  view.work = nullptr;
  view.work_bytes = 0;
  rc = lat->dtype == HSG_F32 ? sweep_impl<float>(&view, p, n_sweeps, st, partials)
                             : sweep_impl<double>(&view, p, n_sweeps, st, partials);
  if (rc == HSG_OK) lat->sweep += (uint64_t)n_sweeps;
  return rc;
}

int hsg_energy(const hsg_lattice* lat, int32_t recompute, double* out_dev, void* stream) {
  int rc = check_lattice(lat);
  if (rc) return rc;
  if (!out_dev) return fail(HSG_EINVAL, "out_dev is NULL");
  hipStream_t st = as_stream(stream);
  if (!recompute) return device_status(hsg::launch_copy_double(lat->E, out_dev, st), "energy copy");
  double* part = hsg::reduce_partials(lat->work, lat->L);
  if (lat->dtype == HSG_F32)
    return device_status(hsg::launch_energy<float>(lat->L, lat->spins, lat->J, part, out_dev, st),
                         "energy");
  return device_status(hsg::launch_energy<double>(lat->L, lat->spins, lat->J, part, out_dev, st),
                       "energy");
}

int hsg_overlap(const hsg_lattice* a, const hsg_lattice* b, double* out_dev, void* stream) {
  int rc = check_lattice(a);
  if (rc) return rc;
  rc = check_lattice(b);
  if (rc) return rc;
  if (a->L != b->L || a->dtype != b->dtype)
    return fail(HSG_EINVAL, "overlap needs two lattices of the same L and dtype");
  if (!out_dev) return fail(HSG_EINVAL, "out_dev is NULL");
  hipStream_t st = as_stream(stream);
  double* part = hsg::reduce_partials(a->work, a->L);
  if (a->dtype == HSG_F32)
    return device_status(hsg::launch_overlap<float>(a->L, a->spins, b->spins, part, out_dev, st),
                         "overlap");
  return device_status(hsg::launch_overlap<double>(a->L, a->spins, b->spins, part, out_dev, st),
                       "overlap");
}

int hsg_overlap_fourier(const hsg_lattice* a, const hsg_lattice* b, double* out_dev,
                        void* stream) {
  int rc = check_lattice(a);
  if (rc) return rc;
  rc = check_lattice(b);
  if (rc) return rc;
  if (a->L != b->L || a->dtype != b->dtype)
    return fail(HSG_EINVAL, "Fourier overlap needs two lattices of the same L and dtype");
  if (!out_dev) return fail(HSG_EINVAL, "out_dev is NULL");
  hipStream_t st = as_stream(stream);
  double* part = hsg::reduce_partials(a->work, a->L);
  if (a->dtype == HSG_F32)
    return device_status(
        hsg::launch_overlap_fourier<float>(a->L, a->spins, b->spins, part, out_dev, st),
        "Fourier overlap");
  return device_status(
      hsg::launch_overlap_fourier<double>(a->L, a->spins, b->spins, part, out_dev, st),
      "Fourier overlap");
}

/* ------------------------------------------------------------------- batched form */

int hsg_batch_check(const hsg_chain* c, int32_t n, int64_t spin_elems, int64_t J_elems) {
  if (!c || n < 1) return fail(HSG_EINVAL, "chain table is empty");
  std::vector<std::pair<int64_t, int64_t>> ranges;
  ranges.reserve((size_t)n);
  for (int32_t i = 0; i < n; ++i) {
    const hsg_chain& ch = c[i];
    if (ch.L < 2 || ch.L > HSG_BATCH_L_MAX || (ch.L & 1))
      return fail(HSG_EINVAL, "chain %d: L must be even, 2 <= L <= %d (got %d)", (int)i,
                  HSG_BATCH_L_MAX, (int)ch.L);
    if (ch.k_hits < 0 || ch.n_or < 0 || ch.k_hits + ch.n_or < 1 || ch.k_hits > 0xFFFF ||
        ch.n_or > 0x7FFF || ch.renorm_every < 0)
      return fail(HSG_EINVAL, "chain %d: bad k_hits / n_or / renorm_every", (int)i);
    if (ch.flags & ~(HSG_HEAT_BATH | HSG_CHAIN_INIT_J) || ch.reserved != 0)
      return fail(HSG_EINVAL, "chain %d: unknown flags 0x%x", (int)i, (unsigned)ch.flags);
    const int64_t n_el = (int64_t)3 * ch.L * ch.L * ch.L;
    // offset <= elems - n_el: no sum that could pass the int64 range
    if (ch.spin_offset < 0 || spin_elems < n_el || ch.spin_offset > spin_elems - n_el)
      return fail(HSG_EINVAL, "chain %d: spins outside the spin buffer", (int)i);
    if (ch.J_offset < 0 || J_elems < n_el || ch.J_offset > J_elems - n_el)
      return fail(HSG_EINVAL, "chain %d: couplings outside the coupling buffer", (int)i);
    ranges.emplace_back(ch.spin_offset, ch.spin_offset + n_el);
  }
  std::sort(ranges.begin(), ranges.end());
  for (size_t i = 1; i < ranges.size(); ++i)
    if (ranges[i].first < ranges[i - 1].second)
      return fail(HSG_EINVAL, "spin ranges of two chains overlap");
  return HSG_OK;
}

static int check_batch(const hsg_batch* b) {
  if (!b) return fail(HSG_EINVAL, "batch descriptor is NULL");
  if (b->n_chains < 1) return fail(HSG_EINVAL, "n_chains must be >= 1");
  if (b->dtype != HSG_F32 && b->dtype != HSG_F64) return fail(HSG_EINVAL, "bad dtype");
  if (!b->chains || !b->spins || !b->J || !b->beta || !b->E || !b->sweep || !b->order)
    return fail(HSG_EINVAL, "batch buffers chains, spins, J, beta, E, sweep, order must be set");
  if (b->threads != 0 && (b->threads < 64 || b->threads > 1024 || (b->threads & 63)))
    return fail(HSG_EINVAL, "threads must be 0 or a multiple of 64 in [64, 1024]");
  if (b->reserved != 0) return fail(HSG_EINVAL, "reserved must be 0");
  return HSG_OK;
}

int hsg_batch_init(const hsg_batch* b, void* stream) {
  int rc = check_batch(b);
  if (rc) return rc;
  hipStream_t st = as_stream(stream);
  return device_status(b->dtype == HSG_F32 ? hsg::launch_batch_init<float>(b, st)
                                           : hsg::launch_batch_init<double>(b, st),
                       "batch init");
}

int hsg_batch_sweep(const hsg_batch* b, int32_t n_sweeps, void* stream) {
  int rc = check_batch(b);
  if (rc) return rc;
  if (n_sweeps < 0) return fail(HSG_EINVAL, "n_sweeps must be >= 0");
  if (n_sweeps == 0) return HSG_OK;
  hipStream_t st = as_stream(stream);
  return device_status(b->dtype == HSG_F32 ? hsg::launch_batch_sweep<float>(b, n_sweeps, st)
                                           : hsg::launch_batch_sweep<double>(b, n_sweeps, st),
                       "batch sweep");
}

int hsg_batch_energy(const hsg_batch* b, double* out_dev, void* stream) {
  int rc = check_batch(b);
  if (rc) return rc;
  if (!out_dev) return fail(HSG_EINVAL, "out_dev is NULL");
  hipStream_t st = as_stream(stream);
  return device_status(b->dtype == HSG_F32 ? hsg::launch_batch_energy<float>(b, out_dev, st)
                                           : hsg::launch_batch_energy<double>(b, out_dev, st),
                       "batch energy");
}

int hsg_batch_overlap(const hsg_batch* b, const int32_t* pairs_dev, int32_t n_pairs,
                      double* out_dev, void* stream) {
  int rc = check_batch(b);
  if (rc) return rc;
  if (!pairs_dev || !out_dev || n_pairs < 0) return fail(HSG_EINVAL, "bad pairs or output");
  if (n_pairs == 0) return HSG_OK;
  hipStream_t st = as_stream(stream);
  return device_status(
      b->dtype == HSG_F32 ? hsg::launch_batch_overlap<float>(b, pairs_dev, n_pairs, out_dev, st)
                          : hsg::launch_batch_overlap<double>(b, pairs_dev, n_pairs, out_dev, st),
      "batch overlap");
}

int hsg_batch_overlap_fourier(const hsg_batch* b, const int32_t* pairs_dev, int32_t n_pairs,
                              double* out_dev, void* stream) {
  int rc = check_batch(b);
  if (rc) return rc;
  if (!pairs_dev || !out_dev || n_pairs < 0) return fail(HSG_EINVAL, "bad pairs or output");
  if (n_pairs == 0) return HSG_OK;
  hipStream_t st = as_stream(stream);
  return device_status(
      b->dtype == HSG_F32
          ? hsg::launch_batch_overlap_fourier<float>(b, pairs_dev, n_pairs, out_dev, st)
          : hsg::launch_batch_overlap_fourier<double>(b, pairs_dev, n_pairs, out_dev, st),
      "batch Fourier overlap");
}

int hsg_batch_tiles(const hsg_chain* c, int32_t n_chains, const int32_t* active, int32_t n_active,
                    int32_t tile_sites, int32_t* tiles_out, int32_t capacity, int32_t* n_tiles) {
  if (!c || !active || !tiles_out || !n_tiles || n_chains < 1 || n_active < 0 || capacity < 0)
    return fail(HSG_EINVAL, "bad arguments to hsg_batch_tiles");
  if (tile_sites < 64 || tile_sites > 1024 || (tile_sites & 63))
    return fail(HSG_EINVAL, "tile_sites must be a multiple of 64 in [64, 1024]");
  int64_t count = 0;
  for (int32_t i = 0; i < n_active; ++i) {
    const int32_t ci = active[i];
    if (ci < 0 || ci >= n_chains) return fail(HSG_EINVAL, "active chain %d out of range", (int)ci);
    const int64_t Nh = (int64_t)(c[ci].L / 2) * c[ci].L * c[ci].L;
    for (int64_t ic0 = 0; ic0 < Nh; ic0 += tile_sites) {
      if (count >= capacity) return fail(HSG_EINVAL, "tile table needs more than %d tiles", (int)capacity);
      tiles_out[2 * count] = ci;
      tiles_out[2 * count + 1] = (int32_t)ic0;
      ++count;
    }
  }
  *n_tiles = (int32_t)count;
  return HSG_OK;
}

int hsg_batch_pass_sweep(const hsg_batch* b, const int32_t* tiles_dev, int32_t n_tiles,
                         int32_t tile_sites, int32_t max_n_or, int32_t renorm, int32_t n_sweeps,
                         void* stream) {
  int rc = check_batch(b);
  if (rc) return rc;
  if (!b->remaining) return fail(HSG_EINVAL, "hsg_batch_pass_sweep needs b->remaining");
  if (!tiles_dev || n_tiles < 0 || n_sweeps < 0 || max_n_or < 0 || max_n_or > 0x7FFF)
    return fail(HSG_EINVAL, "bad tiles, n_sweeps or max_n_or");
  if (tile_sites < 64 || tile_sites > 1024 || (tile_sites & 63))
    return fail(HSG_EINVAL, "tile_sites must be a multiple of 64 in [64, 1024]");
  if (n_tiles == 0 || n_sweeps == 0) return HSG_OK;
  hipStream_t st = as_stream(stream);
  return device_status(
      b->dtype == HSG_F32
          ? hsg::launch_batch_pass_sweep<float>(b, tiles_dev, n_tiles, tile_sites, max_n_or, renorm,
                                                n_sweeps, st)
          : hsg::launch_batch_pass_sweep<double>(b, tiles_dev, n_tiles, tile_sites, max_n_or,
                                                 renorm, n_sweeps, st),
      "batch pass sweep");
}

static int check_pt(const hsg_pt* pt) {
  if (!pt) return fail(HSG_EINVAL, "ladder descriptor is NULL");
  if (pt->n_ladders < 1 || pt->n_temps < 1 || pt->n_temps > 65535)
    return fail(HSG_EINVAL, "need n_ladders >= 1 and 1 <= n_temps <= 65535");
  if (!pt->chain_at_slot || !pt->beta_of_slot)
    return fail(HSG_EINVAL, "chain_at_slot and beta_of_slot must be set");
  return HSG_OK;
}

int hsg_pt_exchange(const hsg_pt* pt, const hsg_batch* b, void* stream) {
  int rc = check_pt(pt);
  if (rc) return rc;
  rc = check_batch(b);
  if (rc) return rc;
  if (!pt->round) return fail(HSG_EINVAL, "round counter must be set");
  return device_status(hsg::launch_pt_exchange(pt, b, as_stream(stream)), "exchange");
}

int hsg_pt_overlap(const hsg_pt* pt, const hsg_batch* b, const int32_t* ladder_pairs_dev,
                   int32_t n_pairs, double* out_dev, void* stream) {
  int rc = check_pt(pt);
  if (rc) return rc;
  rc = check_batch(b);
  if (rc) return rc;
  if (!ladder_pairs_dev || !out_dev || n_pairs < 0) return fail(HSG_EINVAL, "bad pairs or output");
  if (n_pairs == 0) return HSG_OK;
  if (pt->n_temps > 65535) return fail(HSG_EINVAL, "too many temperatures");
  hipStream_t st = as_stream(stream);
  return device_status(
      b->dtype == HSG_F32
          ? hsg::launch_pt_overlap<float>(pt, b, ladder_pairs_dev, n_pairs, out_dev, st)
          : hsg::launch_pt_overlap<double>(pt, b, ladder_pairs_dev, n_pairs, out_dev, st),
      "ladder overlap");
}

int hsg_pt_overlap_fourier(const hsg_pt* pt, const hsg_batch* b, const int32_t* ladder_pairs_dev,
                           int32_t n_pairs, double* out_dev, void* stream) {
  int rc = check_pt(pt);
  if (rc) return rc;
  rc = check_batch(b);
  if (rc) return rc;
  if (!ladder_pairs_dev || !out_dev || n_pairs < 0) return fail(HSG_EINVAL, "bad pairs or output");
  if (n_pairs == 0) return HSG_OK;
  if (pt->n_temps > 65535) return fail(HSG_EINVAL, "too many temperatures");
  hipStream_t st = as_stream(stream);
  return device_status(
      b->dtype == HSG_F32
          ? hsg::launch_pt_overlap_fourier<float>(pt, b, ladder_pairs_dev, n_pairs, out_dev, st)
          : hsg::launch_pt_overlap_fourier<double>(pt, b, ladder_pairs_dev, n_pairs, out_dev, st),
      "ladder Fourier overlap");
}

}  // extern "C"
