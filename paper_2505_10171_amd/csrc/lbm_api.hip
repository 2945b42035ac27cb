// lbm_api.hip -- host implementation of the C ABI declared in include/lbm.h.
//
// The context carves the caller's device workspace, uploads the initial state,
// and issues the per-step kernel sequence on the caller's stream:
//   k_fused (collide + recolour + stream + bounce-back + momentum exchange)
//   k_capbox, k_capillary (capillary force)      -- if the sim has particles
//   k_dem (contacts, friction, Verlet sub-steps)
//   k_claim, k_release, k_cover (solid mask of the new positions)
//   k_refill (fresh fluid nodes)
//   k_moments (order parameter of the new state)
// No device memory is allocated and nothing is synchronised inside lbm_step.
#include <math.h>
#include <stdarg.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include <algorithm>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "../../include/lbm.h"
#include "lbm_device.h"

namespace lbm {
hipError_t launch_interface(const Batch& b, unsigned nblk, unsigned mnblk, hipStream_t st);
hipError_t launch_fused(const Batch& b, int storage, unsigned nblk, int mode, float* orho,
                        float* ou, float* ophi, float* oF, hipStream_t st);
hipError_t launch_links(const Batch& b, int storage, int np_rows, int Bmax, hipStream_t st);
hipError_t launch_moments(const Batch& b, int storage, unsigned nblk, unsigned mnblk, int mode,
                          hipStream_t st);
hipError_t launch_init_mask(const SimDev& s, hipStream_t st);
hipError_t launch_init_pops(const SimDev& s, void* pops, hipStream_t st);
hipError_t launch_mass(const SimDev& s, const float* rp, double* acc, hipStream_t st);
hipError_t launch_zero_f64(double* p, int n, hipStream_t st);
hipError_t launch_mask_update(const Batch& b, int np_rows, int Bmax, bool with_release,
                              hipStream_t st);
hipError_t launch_refill(const Batch& b, int storage, size_t fresh_cap_max, int np_max, int mode,
                         hipStream_t st);
// kernel modes (lbm_fluid.hip, lbm_particles.hip): in a step, or between steps
constexpr int MOM_STEP = 0, MOM_BOUNDARY = 1, REFILL_STEP = 0, REFILL_BOUNDARY = 1;
hipError_t launch_capillary(const Batch& b, int np_rows, int cap_B, int npts, hipStream_t st);
hipError_t launch_dem(const Batch& b, int np_max, int np_rows, int n_sub_max, hipStream_t st);
}  // namespace lbm

using namespace lbm;

// Device scratch of lbm_mass_all_noalloc: the FP64 mass accumulators of up to
// LBM_NOALLOC_MAX_SIMS simulations.  Each GPU holds its own copy; host code
// never uses this name as an address, only the pointer that
// hipGetSymbolAddress returned for the device (noalloc_scratch).
static __device__ __align__(256) double scratch[2 * LBM_NOALLOC_MAX_SIMS];

namespace {

constexpr int MAX_DEVICES = 64;
std::mutex g_scratch_mu;
double* g_scratch_ptr[MAX_DEVICES] = {};
hipError_t g_scratch_err[MAX_DEVICES] = {};
bool g_scratch_done[MAX_DEVICES] = {};

// Address of `scratch` on device dev (which must be current), resolved once per
// device; the outcome (address or error) is kept for later calls.
hipError_t noalloc_scratch(int dev, double** out) {
  *out = nullptr;
  if (dev < 0 || dev >= MAX_DEVICES) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_done[dev]) {
    void* ptr = nullptr;
    g_scratch_err[dev] = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    g_scratch_ptr[dev] = g_scratch_err[dev] == hipSuccess ? (double*)ptr : nullptr;
    g_scratch_done[dev] = true;
  }
  *out = g_scratch_ptr[dev];
  return g_scratch_err[dev];
}

constexpr size_t ALIGN = 256;
constexpr int MAX_PARTICLES = 4096;

size_t align_up(size_t v) { return (v + ALIGN - 1) / ALIGN * ALIGN; }

struct SimLayout {
  long long N;
  int np, Bmask, Bcap, hist_cap;
  size_t pop_bytes, fresh_cap;
  size_t off_pops0, off_pops1, off_rp0, off_rp1, off_nrm, off_cur, off_mask, off_claim, off_fresh, off_fresh_own,
      off_counters, off_P, off_ct, off_nb, off_view, off_hist, off_capbox, off_caporg, off_mass,
      off_step;
  size_t total;
};

double max_radius(const lbm_config& c, const lbm_particle* parts) {
  double r = 0.0;
  for (int p = 0; p < c.n_particles; ++p) r = std::max(r, parts ? parts[p].R : 0.0);
  return r;
}

bool valid_config(const lbm_config& c, char* msg, size_t len) {
  auto fail = [&](const char* m) {
    snprintf(msg, len, "%s", m);
    return false;
  };
  if (c.nx < 1 || c.ny < 1 || c.nz < 3) return fail("lattice must be nx, ny >= 1 and nz >= 3");
  // population offsets are 32-bit: 19 values per node (padded to 64 nodes)
  if (((long long)c.nx * c.ny * c.nz + 63) * 19 > 0xFFFFFFFFll) return fail("lattice too large");
  if (!(c.rho0 > 0.0)) return fail("rho0 must be positive");
  if (!(c.tau_a > 0.5) || !(c.tau_b > 0.5)) return fail("relaxation times must exceed 1/2");
  if (!(c.sigma >= 0.0) || !(c.beta >= 0.0)) return fail("sigma and beta must be >= 0");
  if (!(c.theta_wall_deg > 0.0 && c.theta_wall_deg < 180.0))
    return fail("wall contact angle must be in (0, 180) degrees");
  if (c.storage != LBM_STORE_FP32 && c.storage != LBM_STORE_FP16) return fail("unknown storage");
  if (c.has_wall < LBM_WALL_NONE || c.has_wall > LBM_WALL_BOXES) return fail("unknown wall kind");
  if (c.has_wall == LBM_WALL_BOXES) {
    if (c.n_boxes < 0 || c.n_boxes > LBM_MAX_BOXES) return fail("n_boxes out of range");
    if (c.open_x) return fail("a textured wall needs a periodic x direction");
    const int L[3] = {c.nx, c.ny, c.nz};
    for (int b = 0; b < c.n_boxes; ++b)
      for (int k = 0; k < 3; ++k)
        if (c.boxes[b][k] < 0 || c.boxes[b][k] > c.boxes[b][3 + k] || c.boxes[b][3 + k] >= L[k])
          return fail("a box of the textured wall lies outside the lattice");
  }
  if (c.has_wall == LBM_WALL_TUBE && !(c.tube_R > 0.0)) return fail("tube radius must be positive");
  if (c.open_x != 0 && c.open_x != 1) return fail("open_x must be 0 or 1");
  if (c.open_x && (!(c.rho_in > 0.0) || !(c.rho_out > 0.0)))
    return fail("boundary densities must be positive");
  if (c.n_particles < 0 || c.n_particles > MAX_PARTICLES) return fail("n_particles out of range");
  if (c.n_particles > 0) {
    if (!(c.kn > 0.0) || c.kt < 0.0 || c.kr < 0.0 || c.gn < 0.0 || c.gt < 0.0 || c.gr < 0.0 ||
        c.delta_R < 0.0)
      return fail("invalid contact parameters");
    if (!(c.cap_dang_deg > 0.0) || c.cap_dang_deg > 90.0) return fail("invalid capillary grid");
  }
  return true;
}

bool valid_particle(const lbm_config& c, const lbm_particle& p, char* msg, size_t len) {
  if (!(p.R > 0.5) || !(p.rho_p > 0.0)) {
    snprintf(msg, len, "particle radius must exceed 0.5 and density be positive");
    return false;
  }
  if (!(p.theta_deg > 0.0 && p.theta_deg < 180.0)) {
    snprintf(msg, len, "particle contact angle must be in (0, 180) degrees");
    return false;
  }
  if (2.0 * p.R + 4.0 > std::min(c.nx, std::min(c.ny, c.nz))) {
    snprintf(msg, len, "particle too large for the box");
    return false;
  }
  if (p.mu_s < 0.0 || p.mu_r < 0.0) {
    snprintf(msg, len, "friction coefficients must be >= 0");
    return false;
  }
  if (c.open_x && (p.x[0] < p.R + 4.0 || p.x[0] > (double)(c.nx - 1) - p.R - 4.0)) {
    snprintf(msg, len, "particle within R + 4 nodes of an open x end");
    return false;
  }
  return true;
}

SimLayout layout(const lbm_config& c, double Rmax, int hist_cap, size_t base) {
  SimLayout L{};
  L.N = (long long)c.nx * c.ny * c.nz;
  L.np = c.n_particles;
  L.Bmask = (int)ceil(2.0 * Rmax) + 4;
  L.Bcap = (int)ceil(2.0 * Rmax) + 3;
  L.hist_cap = L.np > 0 ? hist_cap : 0;
  // populations in blocks of 64 nodes (the last one padded)
  L.pop_bytes = (size_t)19 * ((L.N + POP_BLOCK - 1) / POP_BLOCK * POP_BLOCK) *
                (c.storage == LBM_STORE_FP16 ? 2 : 4);
  L.fresh_cap = L.np > 0 ? (size_t)L.np * L.Bmask * L.Bmask * L.Bmask : 0;
  size_t o = align_up(base);
  auto take = [&](size_t bytes) {
    size_t r = o;
    o = align_up(o + std::max<size_t>(bytes, 1));
    return r;
  };
  L.off_pops0 = take(L.pop_bytes);
  L.off_pops1 = take(L.pop_bytes);
  // per-node moments (rho, phi) of the current and the previous state
  L.off_rp0 = take(8 * L.N);
  L.off_rp1 = take(8 * L.N);
  L.off_nrm = take(16 * L.N);
  L.off_cur = take(8 * L.N);
  L.off_mask = take(2 * L.N);
  L.off_claim = take(4 * L.N);
  L.off_fresh = take(4 * L.fresh_cap);
  L.off_fresh_own = take(4 * L.fresh_cap);
  L.off_counters = take(64);
  L.off_P = take(sizeof(DevParticle) * L.np);
  L.off_ct = take(sizeof(Contact) * (size_t)L.np * MAXC);
  L.off_nb = take(sizeof(int) * (size_t)L.np * MAXNB);
  L.off_view = take(sizeof(DemView) * 2 * (size_t)L.np);
  L.off_hist = take(sizeof(double) * (size_t)L.hist_cap * L.np * LBM_HIST_DOUBLES);
  L.off_capbox = take(sizeof(float4) * (size_t)L.np * L.Bcap * L.Bcap * L.Bcap);
  L.off_caporg = take(sizeof(int) * 3 * (size_t)L.np);
  L.off_mass = take(2 * sizeof(double));
  L.off_step = take(sizeof(unsigned long long));
  L.total = o;
  return L;
}

int dem_substeps(const lbm_config& c, const lbm_particle* parts, bool* ok) {
  *ok = true;
  if (c.n_particles == 0) return 1;
  double m1 = INFINITY, m2 = INFINITY;
  for (int p = 0; p < c.n_particles; ++p) {
    const double m = parts[p].rho_p * 4.0 / 3.0 * M_PI * parts[p].R * parts[p].R * parts[p].R;
    if (m < m1) {
      m2 = m1;
      m1 = m;
    } else if (m < m2) {
      m2 = m;
    }
  }
  const double meff = c.n_particles >= 2 ? m1 * m2 / (m1 + m2) : m1;
  const double eta = c.gn / (2.0 * meff);
  const double w2 = c.kn / meff - eta * eta;
  if (!(w2 > 0.0)) {
    *ok = false;
    return 1;
  }
  const double tc = M_PI / sqrt(w2);
  const int ns = (int)ceil(45.0 / tc);
  return ns < 1 ? 1 : ns;
}

void fill_dev_particle(DevParticle& d, const lbm_particle& p, double delta_R, bool keep_dynamics) {
  for (int k = 0; k < 3; ++k) {
    d.x[k] = p.x[k];
    d.v[k] = p.v[k];
    d.w[k] = p.w[k];
  }
  for (int k = 0; k < 4; ++k) d.q[k] = p.q[k];
  d.R = p.R;
  d.rho_p = p.rho_p;
  d.theta = p.theta_deg * M_PI / 180.0;
  d.mu_s = p.mu_s;
  d.mu_r = p.mu_r;
  d.g_p = p.g_p;
  d.mass = p.rho_p * 4.0 / 3.0 * M_PI * p.R * p.R * p.R;
  d.inertia = 0.4 * d.mass * p.R * p.R;
  d.Rc = p.R + delta_R;
  d.neg_cos_t = (float)(-cos(d.theta));
  d.sin_t = (float)sin(d.theta);
  d.kin = p.kinematic ? 1 : 0;
  if (!keep_dynamics) {
    for (int k = 0; k < 3; ++k) {
      d.Fh[k] = d.Th[k] = d.Fcap[k] = d.Tcap[k] = d.Fcon[k] = d.Tcon[k] = 0.0;
      d.Fcp[k] = d.Tcp[k] = d.Fh_last[k] = d.Th_last[k] = 0.0;
    }
  }
}

}  // namespace

struct SimHost {
  lbm_config cfg;
  SimLayout L;
  SimDev d;
  double Rmax;
};

// Per-phase timing with HIP events on the context's stream: per step six
// events bracket the interface kernels, k_fused, k_links, the other particle
// kernels and k_moments.  A small ring of
// event sets is reused; a set is harvested (its elapsed times accumulated)
// before it is recorded again.
constexpr int PROF_RING = 32;
// 0 k_fused, 1 particle kernels but k_links, 2 k_moments, 3 k_interface,
// 4 k_links
constexpr int PROF_KINDS = 5;
constexpr int PROF_EVENTS = PROF_KINDS + 1;
struct Profiler {
  bool on = false;
  int every = 1;           // time every k-th step
  long long step_no = 0;
  hipEvent_t ev[PROF_RING][PROF_EVENTS];
  bool pending[PROF_RING];
  int next = 0;
  double total_ms[PROF_KINDS];
  long long count[PROF_KINDS];
};

struct lbm_ctx {
  std::vector<SimHost> sims;
  hipStream_t stream;
  int dev = 0;  // device current at creation
  char* ws;
  size_t ws_bytes;
  int err;
  char msg[512];
  Profiler prof;
  // every simulation steps together: one population buffer index and one
  // FP16 reference index for all of them
  int cur = 0, rd = 0;
  int storage = 0;
  // batch tables (in the workspace) and their host-side extents
  SimDev* d_tab = nullptr;
  uint32_t* d_blk = nullptr;
  uint32_t* d_mblk = nullptr;
  int2* d_pmap = nullptr;
  unsigned nblk = 0;
  int np_rows = 0, np_max = 0, Bmax = 0, cap_B = 0, npts = 0, n_sub_max = 1;
  bool cap_needed = false;  // some simulation with particles has a capillary force
  size_t fresh_cap_max = 0;
  unsigned mnblk = 0;  // blocks of the moments pass over the batch
  // graph replay of a pair of steps (captured with cur == graph_cur)
  bool use_graph = false;
  hipGraphExec_t graph_exec = nullptr;
  int graph_cur = 0;
};

static unsigned sim_blocks(const SimDev& d) {
  if (d.tile_x == 0) return (unsigned)((d.N + 255) / 256);
  return (unsigned)((long long)d.tiles_x * d.tiles_y * d.nz);
}

// node-block shape of a simulation: tx = 0 (256 consecutive nodes) or an x-y
// tile tx by 256 / tx (tx a power of two, 16..256)
static void set_tile(SimDev& d, int tx) {
  d.tile_x = tx;
  d.tile_lx = 0;
  d.tiles_x = d.tiles_y = 0;
  if (tx == 0) return;
  while ((1 << d.tile_lx) < tx) ++d.tile_lx;
  d.tiles_x = (d.nx + tx - 1) / tx;
  d.tiles_y = (d.ny + (256 / tx) - 1) / (256 / tx);
}

// tiling of the moments and interface passes: x-y tiles, the widest of 64,
// 32, 16 whose whole tiles cover the box's width with at most 20 % to spare
// (else 16: an 80-wide box takes three 32-wide tiles, not two 64-wide ones of
// which the second is three-quarters idle; measured on the ensemble of 48- to
// 96-wide boxes: 20 % beat 15 % and 34 %), each block marching mkz planes up z: 12 on planes
// of 64k nodes or more (the two extra planes a block loads at its ends are
// then a sixth of its work, not a third), 6 on smaller ones, whose neighbour
// planes stay in the caches anyway (measured: the moments pass of a 256x128
// plane is slower with 12)
// planes: marching depth of a block (0: the default).  The default marches
// 12 planes on planes of at least 65,536 nodes, 6 on smaller ones; and 6 also
// where 12-plane blocks would fill the 1,536 resident slots of the interface
// pass (six blocks per CU) between one and four times over, so that the last
// partial round of long blocks leaves most CUs idle (the 400 x 181 x 71 run:
// interface + moments 268 us at 12 planes, 245 us at 6; the 512 x 256 x 192
// slab and boxes of under one round are within 1 % either way).
static void set_mom_tiling(SimDev& d, int planes = 0) {
  d.mtile_x = 16;
  for (int w : {64, 32}) {
    if (100LL * ((d.nx + w - 1) / w) * w <= 120LL * d.nx) {
      d.mtile_x = w;
      break;
    }
  }
  d.mtile_lx = d.mtile_x == 64 ? 6 : (d.mtile_x == 32 ? 5 : 4);
  const int ty = 256 / d.mtile_x;
  if (planes > 0) {
    d.mkz = planes;
  } else {
    // 1,536 = the interface pass's resident blocks (six per CU): a depth whose
    // blocks overflow one round by a fraction leaves most CUs idle at the end
    d.mkz = (long long)d.nx * d.ny >= 65536 ? 12 : 6;
    const long long tiles = (long long)((d.nx + d.mtile_x - 1) / d.mtile_x) * ((d.ny + ty - 1) / ty);
    const long long b12 = tiles * ((d.nz + 11) / 12);
    if (d.mkz == 12 && b12 > 1536 && b12 < 4 * 1536) d.mkz = 6;
    const long long b6 = tiles * ((d.nz + 5) / 6), b8 = tiles * ((d.nz + 7) / 8);
    if (d.mkz == 6 && b6 > 1536 && b8 <= 1536) d.mkz = 8;
  }
  d.mtiles_x = (d.nx + d.mtile_x - 1) / d.mtile_x;
  d.mtiles_y = (d.ny + ty - 1) / ty;
  d.mtiles_z = (d.nz + d.mkz - 1) / d.mkz;
}
static unsigned mom_blocks(const SimDev& d) {
  return (unsigned)((long long)d.mtiles_x * d.mtiles_y * d.mtiles_z);
}

// open x ends, a tube or a textured wall: the interface kernel's general
// instance; open x ends: the fused kernel's
static int general_geometry(const lbm_config& c) {
  return c.open_x || c.has_wall == LBM_WALL_TUBE || c.has_wall == LBM_WALL_BOXES;
}
static Batch batch_all(const lbm_ctx* c) {
  int general = 0, open = 0;
  int mlx = c->sims.empty() ? 0 : c->sims[0].d.mtile_lx;
  for (const SimHost& sh : c->sims) {
    general |= general_geometry(sh.cfg);
    open |= sh.cfg.open_x;
    if (sh.d.mtile_lx != mlx) mlx = 0;
  }
  return Batch{c->d_tab, c->d_blk, c->d_mblk, c->d_pmap, (int)c->sims.size(), c->cur, c->rd,
               general, open, mlx};
}
static Batch batch_one(const lbm_ctx* c, int si) {
  return Batch{c->d_tab + si, nullptr, nullptr, nullptr, 1, c->cur, c->rd,
               general_geometry(c->sims[si].cfg), c->sims[si].cfg.open_x,
               c->sims[si].d.mtile_lx};
}

// workspace tail holding the batch tables
static size_t batch_tables_bytes(int n_sims, long long np_total) {
  return align_up(sizeof(SimDev) * (size_t)n_sims) + 2 * align_up(4 * (size_t)(n_sims + 1)) +
         align_up(8 * (size_t)std::max<long long>(np_total, 1));
}

static int set_err(lbm_ctx* c, int code, const char* fmt, ...) {
  if (!c) return code;
  if (c->err == 0) {
    c->err = code;
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(c->msg, sizeof(c->msg), fmt, ap);
    va_end(ap);
  }
  return code;
}

#define HIPCHK(ctx, call)                                                                  \
  do {                                                                                     \
    hipError_t e_ = (call);                                                                \
    if (e_ != hipSuccess)                                                                  \
      return set_err((ctx), LBM_EHIP, "%s failed: %s", #call, hipGetErrorString(e_));      \
  } while (0)

// Device batch tables (simulation records, block prefix of the per-node
// kernels, particle rows) and their extents; at creation `off` is the end of the
// last simulation's carve (the tables follow it), afterwards pass 0.
static int upload_tables(lbm_ctx* ctx, size_t off) {
  const int n_sims = (int)ctx->sims.size();
  if (off) {
    char* b = ctx->ws + align_up(off);
    ctx->d_tab = (SimDev*)b;
    b += align_up(sizeof(SimDev) * (size_t)n_sims);
    ctx->d_blk = (uint32_t*)b;
    b += align_up(4 * (size_t)(n_sims + 1));
    ctx->d_mblk = (uint32_t*)b;
    b += align_up(4 * (size_t)(n_sims + 1));
    ctx->d_pmap = (int2*)b;
  }
  std::vector<SimDev> tab(n_sims);
  std::vector<uint32_t> blk(n_sims + 1, 0), mblk(n_sims + 1, 0);
  std::vector<int2> pmap;
  ctx->np_max = ctx->Bmax = ctx->cap_B = ctx->npts = 0;
  ctx->cap_needed = false;
  ctx->n_sub_max = 1;
  ctx->fresh_cap_max = 0;
  for (int si = 0; si < n_sims; ++si) {
    const SimHost& sh = ctx->sims[si];
    tab[si] = sh.d;
    const unsigned long long mb = (unsigned long long)mblk[si] + mom_blocks(sh.d);
    if (mb > 0x7fffffffull) return set_err(ctx, LBM_EINVAL, "too many lattice nodes in one context");
    mblk[si + 1] = (uint32_t)mb;
    const unsigned long long nb = (unsigned long long)blk[si] + sim_blocks(sh.d);
    if (nb > 0x7fffffffull) return set_err(ctx, LBM_EINVAL, "too many lattice nodes in one context");
    blk[si + 1] = (uint32_t)nb;
    for (int p = 0; p < sh.d.np; ++p) pmap.push_back(make_int2(si, p));
    ctx->np_max = std::max(ctx->np_max, sh.d.np);
    if (sh.d.np > 0) ctx->n_sub_max = std::max(ctx->n_sub_max, sh.d.n_sub);
    if (sh.d.np > 0) {
      ctx->Bmax = std::max(ctx->Bmax, sh.L.Bmask);
      ctx->cap_B = std::max(ctx->cap_B, sh.d.cap_B);
      ctx->npts = std::max(ctx->npts, sh.d.cap_na * sh.d.cap_nphi);
      ctx->cap_needed |= sh.d.cap_pref != 0.0;
      ctx->fresh_cap_max = std::max(ctx->fresh_cap_max, (size_t)sh.d.fresh_cap);
    }
  }
  ctx->nblk = blk[n_sims];
  ctx->mnblk = mblk[n_sims];
  ctx->np_rows = (int)pmap.size();
  hipStream_t st = ctx->stream;
  HIPCHK(ctx, hipMemcpyAsync(ctx->d_tab, tab.data(), sizeof(SimDev) * n_sims, hipMemcpyHostToDevice, st));
  HIPCHK(ctx, hipMemcpyAsync(ctx->d_blk, blk.data(), 4 * (size_t)(n_sims + 1), hipMemcpyHostToDevice, st));
  HIPCHK(ctx, hipMemcpyAsync(ctx->d_mblk, mblk.data(), 4 * (size_t)(n_sims + 1), hipMemcpyHostToDevice, st));
  if (!pmap.empty())
    HIPCHK(ctx, hipMemcpyAsync(ctx->d_pmap, pmap.data(), 8 * pmap.size(), hipMemcpyHostToDevice, st));
  HIPCHK(ctx, hipStreamSynchronize(st));
  return LBM_OK;
}

// mask of the new particle positions, fresh nodes, refill, moments (one
// simulation, between steps)
static int post_dem_pipeline(lbm_ctx* ctx, int si, bool with_release) {
  const SimHost& sh = ctx->sims[si];
  const SimDev& s = sh.d;
  const Batch b = batch_one(ctx, si);
  if (s.np > 0) {
    HIPCHK(ctx, launch_mask_update(b, s.np, sh.L.Bmask, with_release, ctx->stream));
    HIPCHK(ctx, launch_refill(b, ctx->storage, s.fresh_cap, s.np, REFILL_BOUNDARY, ctx->stream));
  }
  HIPCHK(ctx, launch_moments(b, ctx->storage, sim_blocks(s), 0, MOM_BOUNDARY, ctx->stream));
  return LBM_OK;
}

extern "C" {

size_t lbm_workspace_bytes(const lbm_config* cfg, int32_t n_sims,
                           const lbm_particle* const* parts, int32_t history_steps) {
  if (!cfg || n_sims < 1 || history_steps < 0) return 0;
  char msg[256];
  size_t o = 0;
  long long np_total = 0;
  for (int s = 0; s < n_sims; ++s) {
    if (!valid_config(cfg[s], msg, sizeof msg)) return 0;
    if (cfg[s].storage != cfg[0].storage) return 0;
    if (cfg[s].n_particles > 0 && (!parts || !parts[s])) return 0;
    const double Rmax = max_radius(cfg[s], cfg[s].n_particles > 0 ? parts[s] : nullptr);
    o = layout(cfg[s], Rmax, history_steps, o).total;
    np_total += cfg[s].n_particles;
  }
  return align_up(o) + batch_tables_bytes(n_sims, np_total);
}

int lbm_create(const lbm_config* cfg, int32_t n_sims, const float* const* phi0,
               const lbm_particle* const* parts, int32_t history_steps, void* dev_workspace,
               size_t ws_bytes, void* hip_stream, lbm_ctx** out) {
  if (!out) return LBM_EINVAL;
  *out = nullptr;
  lbm_ctx* ctx = new (std::nothrow) lbm_ctx();
  if (!ctx) return LBM_ENOMEM;
  ctx->stream = (hipStream_t)hip_stream;
  ctx->ws = (char*)dev_workspace;
  ctx->ws_bytes = ws_bytes;
  ctx->err = 0;
  ctx->msg[0] = 0;
  auto fail = [&](int code, const char* m) {
    set_err(ctx, code, "%s", m);
    *out = ctx;  // the caller reads lbm_last_error, then destroys
    return code;
  };
  if (!cfg || n_sims < 1 || !dev_workspace || history_steps < 0)
    return fail(LBM_EINVAL, "invalid arguments");
  if (hipGetDevice(&ctx->dev) != hipSuccess) return fail(LBM_EHIP, "no current device");
  {
    // resolve the no-allocation scratch of this device once, while it is
    // current; a failure is reported by lbm_mass_all_noalloc
    double* unused = nullptr;
    (void)noalloc_scratch(ctx->dev, &unused);
  }
  size_t need = lbm_workspace_bytes(cfg, n_sims, parts, history_steps);
  if (need == 0) {
    char msg[256] = "invalid configuration";
    for (int s = 0; s < n_sims; ++s) valid_config(cfg[s], msg, sizeof msg);
    for (int s = 0; s < n_sims; ++s)
      if (cfg[s].storage != cfg[0].storage)
        snprintf(msg, sizeof msg, "all simulations of a context share one storage type");
    return fail(LBM_EINVAL, msg);
  }
  if (ws_bytes < need) return fail(LBM_ENOMEM, "workspace too small");
  if (((uintptr_t)dev_workspace) % ALIGN != 0)
    return fail(LBM_EINVAL, "workspace must be 256-byte aligned");
  ctx->sims.resize(n_sims);
  size_t off = 0;
  for (int si = 0; si < n_sims; ++si) {
    const lbm_config& c = cfg[si];
    const lbm_particle* pp = (parts && c.n_particles > 0) ? parts[si] : nullptr;
    if (c.n_particles > 0 && !pp) return fail(LBM_EINVAL, "particles missing");
    char msg[256];
    for (int p = 0; p < c.n_particles; ++p)
      if (!valid_particle(c, pp[p], msg, sizeof msg)) return fail(LBM_EINVAL, msg);
    bool ok;
    const int n_sub = dem_substeps(c, pp, &ok);
    if (!ok) return fail(LBM_EINVAL, "normal damping too large: k_n/m - (g_n/2m)^2 <= 0");
    SimHost& sh = ctx->sims[si];
    sh.cfg = c;
    sh.Rmax = max_radius(c, pp);
    sh.L = layout(c, sh.Rmax, history_steps, off);
    off = sh.L.total;
    SimDev& d = sh.d;
    memset(&d, 0, sizeof d);
    d.nx = c.nx;
    d.ny = c.ny;
    d.nz = c.nz;
    d.has_wall = c.has_wall;
    d.open_x = c.open_x;
    d.drho_in = (float)(c.rho_in - c.rho0);
    d.drho_out = (float)(c.rho_out - c.rho0);
    d.tube_R2 = c.tube_R * c.tube_R;
    d.tube_yc = 0.5 * (c.ny - 1);
    d.tube_zc = 0.5 * (c.nz - 1);
    d.n_boxes = c.has_wall == LBM_WALL_BOXES ? c.n_boxes : 0;
    for (int b = 0; b < d.n_boxes; ++b)
      for (int k = 0; k < 6; ++k) d.boxes[b][k] = c.boxes[b][k];
    d.N = sh.L.N;
    set_mom_tiling(d);
    d.storage = c.storage;
    d.np = c.n_particles;
    d.rho0 = (float)c.rho0;
    d.sigma = (float)c.sigma;
    d.beta = (float)c.beta;
    const double nua = (c.tau_a - 0.5) / 3.0, nub = (c.tau_b - 0.5) / 3.0;
    d.inv2nua = (float)(1.0 / (2.0 * nua));
    d.inv2nub = (float)(1.0 / (2.0 * nub));
    for (int k = 0; k < 3; ++k) d.body[k] = (float)c.body_force[k];
    d.wall_neg_cos = (float)(-cos(c.theta_wall_deg * M_PI / 180.0));
    d.wall_sin = (float)sin(c.theta_wall_deg * M_PI / 180.0);
    char* b = ctx->ws;
    d.pops[0] = b + sh.L.off_pops0;
    d.pops[1] = b + sh.L.off_pops1;
    d.rp[0] = (float*)(b + sh.L.off_rp0);
    d.rp[1] = (float*)(b + sh.L.off_rp1);
    d.nrm = (float*)(b + sh.L.off_nrm);
    d.curv = (float2*)(b + sh.L.off_cur);
    d.mask = (uint16_t*)(b + sh.L.off_mask);
    d.claim = (uint32_t*)(b + sh.L.off_claim);
    d.fresh = (uint32_t*)(b + sh.L.off_fresh);
    d.fresh_own = (uint32_t*)(b + sh.L.off_fresh_own);
    d.counters = (uint32_t*)(b + sh.L.off_counters);
    d.fresh_cap = (uint32_t)sh.L.fresh_cap;
    d.P = (DevParticle*)(b + sh.L.off_P);
    d.ct = (Contact*)(b + sh.L.off_ct);
    d.nb = (int*)(b + sh.L.off_nb);
    d.view = (DemView*)(b + sh.L.off_view);
    d.hist = (double*)(b + sh.L.off_hist);
    d.hist_cap = sh.L.hist_cap;
    d.n_sub = n_sub;
    d.kn = c.kn;
    d.kt = c.kt;
    d.kr = c.kr;
    d.gn = c.gn;
    d.gt = c.gt;
    d.gr = c.gr;
    d.delta_R = c.delta_R;
    d.cap_pref = c.sigma * 4.5 * c.cap_k * c.beta;
    d.cap_dang = c.cap_dang_deg * M_PI / 180.0;
    d.cap_na = (int)llround(180.0 / c.cap_dang_deg);
    d.cap_nphi = (int)llround(360.0 / c.cap_dang_deg);
    d.cap_B = sh.L.Bcap;
    d.capbox = (float4*)(b + sh.L.off_capbox);
    d.capbox_org = (int*)(b + sh.L.off_caporg);
    d.mass_acc = (double*)(b + sh.L.off_mass);
    d.step_counter = (unsigned long long*)(b + sh.L.off_step);

    // upload particles and contact tables
    hipStream_t st = ctx->stream;
    if (d.np > 0) {
      std::vector<DevParticle> hp(d.np);
      memset(hp.data(), 0, sizeof(DevParticle) * d.np);
      for (int p = 0; p < d.np; ++p) {
        fill_dev_particle(hp[p], pp[p], c.delta_R, false);
        for (int k = 0; k < 3; ++k) hp[p].xo[k] = hp[p].x[k];
        hp[p].Ro = hp[p].R;
      }
      std::vector<Contact> ct((size_t)d.np * MAXC);
      for (auto& e : ct) {
        memset(&e, 0, sizeof e);
        e.partner = -100;
      }
      if (hipMemcpyAsync(d.P, hp.data(), sizeof(DevParticle) * d.np, hipMemcpyHostToDevice,
                         st) != hipSuccess ||
          hipMemcpyAsync(d.ct, ct.data(), sizeof(Contact) * ct.size(), hipMemcpyHostToDevice,
                         st) != hipSuccess ||
          hipStreamSynchronize(st) != hipSuccess)
        return fail(LBM_EHIP, "particle upload failed");
    }
    if (hipMemsetAsync(d.counters, 0, 64, st) != hipSuccess ||
        hipMemsetAsync(d.step_counter, 0, sizeof(unsigned long long), st) != hipSuccess)
      return fail(LBM_EHIP, "counter initialisation failed");
    // phi0 staged in the phi plane of rp[0]
    if (phi0 && phi0[si]) {
      if (hipMemcpyAsync(d.rp[0] + d.N, phi0[si], sizeof(float) * d.N, hipMemcpyHostToDevice, st) !=
          hipSuccess)
        return fail(LBM_EHIP, "phi0 upload failed");
    } else {
      std::vector<float> ones(d.N, 1.0f);
      if (hipMemcpyAsync(d.rp[0] + d.N, ones.data(), sizeof(float) * d.N, hipMemcpyHostToDevice, st) !=
              hipSuccess ||
          hipStreamSynchronize(st) != hipSuccess)
        return fail(LBM_EHIP, "phi0 upload failed");
    }
    if (phi0 && phi0[si]) {
      // the host buffer must stay valid until the copy has completed
      if (hipStreamSynchronize(st) != hipSuccess) return fail(LBM_EHIP, "synchronise failed");
    }
  }
  // a batch whose blocks fill the GPU several times over even at a depth of
  // 24 planes marches 24 (each block re-reads its two halo planes once per 24
  // planes, not per 6 or 12; measured on the ensemble of 256 boxes 48 to 96
  // wide: 8.75 ms per step at the single-box depths, 8.54 at 12, 8.36 at 24)
  if (ctx->sims.size() > 1) {
    long long deep = 0;
    for (const SimHost& sh : ctx->sims)
      deep += (long long)sh.d.mtiles_x * sh.d.mtiles_y * ((sh.d.nz + 23) / 24);
    if (deep >= 4 * 1536)
      for (SimHost& sh : ctx->sims) set_mom_tiling(sh.d, 24);
  }
  // batch tables: simulation records, block prefix, particle rows
  ctx->storage = cfg[0].storage;
  if (int rc = upload_tables(ctx, off)) return fail(rc, ctx->msg);
  // initial state of every simulation
  ctx->cur = 0;
  ctx->rd = 0;
  for (int si = 0; si < n_sims; ++si) {
    const SimHost& sh = ctx->sims[si];
    const SimDev& d = sh.d;
    const Batch b1 = batch_one(ctx, si);
    hipStream_t st = ctx->stream;
    if (launch_init_mask(d, st) != hipSuccess) return fail(LBM_EHIP, "mask init failed");
    if (d.np > 0 && launch_mask_update(b1, d.np, sh.L.Bmask, false, st) != hipSuccess)
      return fail(LBM_EHIP, "mask build failed");
    if (launch_init_pops(d, d.pops[0], st) != hipSuccess)
      return fail(LBM_EHIP, "population init failed");
  }
  if (hipStreamSynchronize(ctx->stream) != hipSuccess) return fail(LBM_EHIP, "synchronise failed");
  *out = ctx;
  return LBM_OK;
}

static int prof_harvest(lbm_ctx* ctx, int slot) {
  Profiler& P = ctx->prof;
  if (!P.pending[slot]) return LBM_OK;
  HIPCHK(ctx, hipEventSynchronize(P.ev[slot][PROF_EVENTS - 1]));
  // events: 0 | interface | 1 | fused | 2 | links | 3 | particles | 4 | moments | 5
  const int kind_of_gap[PROF_KINDS] = {3, 0, 4, 1, 2};
  for (int k = 0; k < PROF_KINDS; ++k) {
    float ms = 0.f;
    HIPCHK(ctx, hipEventElapsedTime(&ms, P.ev[slot][k], P.ev[slot][k + 1]));
    P.total_ms[kind_of_gap[k]] += ms;
    P.count[kind_of_gap[k]] += 1;
  }
  P.pending[slot] = false;
  return LBM_OK;
}

// One step of every simulation: each phase is one launch over the batch.
static int step_once(lbm_ctx* ctx, int slot) {
  Profiler& P = ctx->prof;
  hipStream_t st = ctx->stream;
  const Batch b = batch_all(ctx);
  if (slot >= 0) HIPCHK(ctx, hipEventRecord(P.ev[slot][0], st));
  HIPCHK(ctx, launch_interface(b, ctx->nblk, ctx->mnblk, st));
  if (slot >= 0) HIPCHK(ctx, hipEventRecord(P.ev[slot][1], st));
  HIPCHK(ctx, launch_fused(b, ctx->storage, ctx->nblk, 0, nullptr, nullptr, nullptr, nullptr, st));
  if (slot >= 0) HIPCHK(ctx, hipEventRecord(P.ev[slot][2], st));
  HIPCHK(ctx, launch_links(b, ctx->storage, ctx->np_rows, ctx->Bmax, st));
  if (slot >= 0) HIPCHK(ctx, hipEventRecord(P.ev[slot][3], st));
  ctx->cur ^= 1;
  ctx->rd ^= 1;
  const Batch a = batch_all(ctx);
  if (ctx->np_rows > 0) {
    // without surface tension (sigma = 0) the capillary force is zero: the DEM
    // reads the accumulators it cleared itself
    if (ctx->cap_needed) HIPCHK(ctx, launch_capillary(a, ctx->np_rows, ctx->cap_B, ctx->npts, st));
    HIPCHK(ctx, launch_dem(a, ctx->np_max, ctx->np_rows, ctx->n_sub_max, st));
    HIPCHK(ctx, launch_mask_update(a, ctx->np_rows, ctx->Bmax, true, st));
    HIPCHK(ctx, launch_refill(a, ctx->storage, ctx->fresh_cap_max, ctx->np_max, REFILL_STEP, st));
  }
  if (slot >= 0) HIPCHK(ctx, hipEventRecord(P.ev[slot][4], st));
  HIPCHK(ctx, launch_moments(a, ctx->storage, ctx->nblk, ctx->mnblk, MOM_STEP, st));
  if (slot >= 0) {
    HIPCHK(ctx, hipEventRecord(P.ev[slot][5], st));
    P.pending[slot] = true;
  }
  return LBM_OK;
}

// Capture two steps into a graph (the buffer indices return to their values
// at capture, so the recorded kernel arguments stay valid for every replay).
static int capture_pair(lbm_ctx* ctx) {
  hipGraph_t g = nullptr;
  const int cur0 = ctx->cur, rd0 = ctx->rd;
  HIPCHK(ctx, hipStreamBeginCapture(ctx->stream, hipStreamCaptureModeThreadLocal));
  int rc = step_once(ctx, -1);
  if (rc == LBM_OK) rc = step_once(ctx, -1);
  hipError_t e = hipStreamEndCapture(ctx->stream, &g);
  ctx->cur = cur0;  // nothing ran yet: the captured steps execute on replay
  ctx->rd = rd0;
  if (rc) {
    if (g) (void)hipGraphDestroy(g);
    return rc;
  }
  if (e != hipSuccess) return set_err(ctx, LBM_EHIP, "graph capture failed: %s", hipGetErrorString(e));
  e = hipGraphInstantiate(&ctx->graph_exec, g, nullptr, nullptr, 0);
  (void)hipGraphDestroy(g);
  if (e != hipSuccess) {
    ctx->graph_exec = nullptr;
    return set_err(ctx, LBM_EHIP, "graph instantiation failed: %s", hipGetErrorString(e));
  }
  ctx->graph_cur = cur0;
  return LBM_OK;
}

int lbm_use_graph(lbm_ctx* ctx, int32_t enable) {
  if (!ctx) return LBM_EINVAL;
  if (ctx->err) return LBM_ESTATE;
  if (enable && ctx->stream == nullptr)
    return set_err(ctx, LBM_EINVAL, "graph replay needs a stream other than the null stream");
  if (!enable && ctx->graph_exec) {
    HIPCHK(ctx, hipStreamSynchronize(ctx->stream));
    (void)hipGraphExecDestroy(ctx->graph_exec);
    ctx->graph_exec = nullptr;
  }
  ctx->use_graph = enable != 0;
  return LBM_OK;
}

int lbm_step(lbm_ctx* ctx, int32_t n_steps) {
  if (!ctx) return LBM_EINVAL;
  if (ctx->err) return LBM_ESTATE;
  if (n_steps < 0) return set_err(ctx, LBM_EINVAL, "negative step count");
  Profiler& P = ctx->prof;
  if (ctx->use_graph && !P.on && n_steps >= 2) {
    if (!ctx->graph_exec) {
      int rc = capture_pair(ctx);
      if (rc) return rc;
    }
    if (ctx->cur != ctx->graph_cur) {  // one ordinary step to the captured parity
      int rc = step_once(ctx, -1);
      if (rc) return rc;
      --n_steps;
    }
    for (; n_steps >= 2; n_steps -= 2) HIPCHK(ctx, hipGraphLaunch(ctx->graph_exec, ctx->stream));
  }
  for (int t = 0; t < n_steps; ++t) {
    int slot = -1;
    if (P.on && (P.step_no++ % P.every) == 0) {
      slot = P.next;
      P.next = (P.next + 1) % PROF_RING;
      int rc = prof_harvest(ctx, slot);
      if (rc) return rc;
    }
    int rc = step_once(ctx, slot);
    if (rc) return rc;
  }
  return LBM_OK;
}

// Block-shape autotuner.  For every box class (nx, ny, nz) of the context it
// times the per-node kernels of one representative simulation -- normal,
// curvature, the fused step into the spare buffer, and the moments pass,
// which leave the current state unchanged -- with each candidate shape, and
// gives the whole class the fastest.  Choices are cached per process by
// (architecture, box, storage).
int lbm_autotune(lbm_ctx* ctx, int32_t reps, int32_t* chosen) {
  if (!ctx) return LBM_EINVAL;
  if (ctx->err) return LBM_ESTATE;
  if (reps < 1) return set_err(ctx, LBM_EINVAL, "reps must be >= 1");
  if (ctx->graph_exec) {  // its launches carry the old grid sizes
    HIPCHK(ctx, hipStreamSynchronize(ctx->stream));
    (void)hipGraphExecDestroy(ctx->graph_exec);
    ctx->graph_exec = nullptr;
  }
  static std::vector<std::pair<std::string, int>> cache;
  int dev = 0;
  HIPCHK(ctx, hipGetDevice(&dev));
  hipDeviceProp_t prop;
  HIPCHK(ctx, hipGetDeviceProperties(&prop, dev));
  const int cand[] = {0, 256, 128, 64, 32, 16};
  hipStream_t st = ctx->stream;
  hipEvent_t e0, e1;
  HIPCHK(ctx, hipEventCreate(&e0));
  HIPCHK(ctx, hipEventCreate(&e1));
  const int n_sims = (int)ctx->sims.size();
  std::vector<float> save;  // host copy of the moments the timing rewrites
  int rc = LBM_OK;
  for (int si = 0; si < n_sims && rc == LBM_OK; ++si) {
    SimDev& d = ctx->sims[si].d;
    char key[128];
    snprintf(key, sizeof key, "%s|%d|%d|%d|%d", prop.gcnArchName, d.nx, d.ny, d.nz, d.storage);
    int best = -1;
    for (auto& kv : cache)
      if (kv.first == key) best = kv.second;
    if (best < 0) {
      // each timed pass is the fluid part of a real step on the current state
      // (interface and collide-and-stream on it, the moments pass on what that
      // streamed), so every pass sees consistent data and repeats the same
      // work.  The moments pass overwrites the previous moments (the FP16
      // reference): kept aside in host memory (the library allocates no device
      // memory) and put back, with the status words
      const size_t rp_bytes = 8 * (size_t)d.N;
      save.resize(2 * (size_t)d.N);
      float* rp_prev = d.rp[ctx->rd];
      HIPCHK(ctx, hipMemcpyAsync(save.data(), rp_prev, rp_bytes, hipMemcpyDeviceToHost, st));
      uint32_t status[4];
      HIPCHK(ctx, hipMemcpyAsync(status, d.counters, sizeof status, hipMemcpyDeviceToHost, st));
      HIPCHK(ctx, hipStreamSynchronize(st));
      float best_ms = 1e30f;
      for (int c : cand) {
        if (c > 0 && c > 2 * d.nx) continue;  // over half the tile idle
        set_tile(d, c);
        HIPCHK(ctx, hipMemcpyAsync(ctx->d_tab + si, &d, sizeof(SimDev), hipMemcpyHostToDevice, st));
        const Batch b1 = batch_one(ctx, si);
        Batch a1 = b1;  // buffer indices after a step's swap
        a1.cur ^= 1;
        a1.rd ^= 1;
        const unsigned nb = sim_blocks(d);
        float ms = 0.f;
        for (int r = 0; r <= reps; ++r) {  // the first pass warms up
          if (r == 1) HIPCHK(ctx, hipEventRecord(e0, st));
          HIPCHK(ctx, launch_interface(b1, nb, mom_blocks(d), st));
          HIPCHK(ctx, launch_fused(b1, ctx->storage, nb, 0, nullptr, nullptr, nullptr, nullptr, st));
          HIPCHK(ctx, launch_moments(a1, ctx->storage, nb, mom_blocks(d), MOM_STEP, st));
        }
        HIPCHK(ctx, hipEventRecord(e1, st));
        HIPCHK(ctx, hipEventSynchronize(e1));
        HIPCHK(ctx, hipEventElapsedTime(&ms, e0, e1));
        if (ms < best_ms) {
          best_ms = ms;
          best = c;
        }
      }
      HIPCHK(ctx, hipMemcpyAsync(rp_prev, save.data(), rp_bytes, hipMemcpyHostToDevice, st));
      HIPCHK(ctx, hipMemcpyAsync(d.counters, status, sizeof status, hipMemcpyHostToDevice, st));
      HIPCHK(ctx, hipStreamSynchronize(st));
      cache.emplace_back(key, best);
    }
    set_tile(d, best);
    if (chosen) chosen[si] = best;
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (rc) return rc;
  return upload_tables(ctx, 0);
}

int lbm_set_tile(lbm_ctx* ctx, int32_t sim, int32_t tile_x) {
  if (!ctx) return LBM_EINVAL;
  if (ctx->err) return LBM_ESTATE;
  if (sim < 0 || sim >= (int)ctx->sims.size())
    return set_err(ctx, LBM_ERANGE, "simulation index out of range");
  if (!(tile_x == 0 || tile_x == 16 || tile_x == 32 || tile_x == 64 || tile_x == 128 ||
        tile_x == 256))
    return set_err(ctx, LBM_EINVAL, "tile width must be 0, 16, 32, 64, 128 or 256");
  if (ctx->graph_exec) {
    HIPCHK(ctx, hipStreamSynchronize(ctx->stream));
    (void)hipGraphExecDestroy(ctx->graph_exec);
    ctx->graph_exec = nullptr;
  }
  set_tile(ctx->sims[sim].d, tile_x);
  return upload_tables(ctx, 0);
}

int lbm_set_march(lbm_ctx* ctx, int32_t sim, int32_t planes) {
  if (!ctx) return LBM_EINVAL;
  if (ctx->err) return LBM_ESTATE;
  if (sim < 0 || sim >= (int)ctx->sims.size())
    return set_err(ctx, LBM_ERANGE, "simulation index out of range");
  if (planes < 0 || planes > 256) return set_err(ctx, LBM_EINVAL, "planes must be in [0, 256]");
  if (ctx->graph_exec) {
    HIPCHK(ctx, hipStreamSynchronize(ctx->stream));
    (void)hipGraphExecDestroy(ctx->graph_exec);
    ctx->graph_exec = nullptr;
  }
  set_mom_tiling(ctx->sims[sim].d, planes);
  return upload_tables(ctx, 0);
}

int lbm_profile(lbm_ctx* ctx, int32_t enable) {
  if (!ctx) return LBM_EINVAL;
  if (ctx->err) return LBM_ESTATE;
  Profiler& P = ctx->prof;
  if (enable < 0) return set_err(ctx, LBM_EINVAL, "profile interval must be >= 0");
  if (enable) {
    P.every = enable;
    P.step_no = 0;
  }
  if (enable && !P.on) {
    for (int r = 0; r < PROF_RING; ++r) {
      for (int k = 0; k < PROF_EVENTS; ++k) HIPCHK(ctx, hipEventCreate(&P.ev[r][k]));
      P.pending[r] = false;
    }
    P.next = 0;
    P.on = true;
  }
  if (P.on)
    for (int k = 0; k < PROF_KINDS; ++k) {
      P.total_ms[k] = 0.0;
      P.count[k] = 0;
    }
  if (!enable && P.on) {
    HIPCHK(ctx, hipStreamSynchronize(ctx->stream));
    for (int r = 0; r < PROF_RING; ++r)
      for (int k = 0; k < PROF_EVENTS; ++k) (void)hipEventDestroy(P.ev[r][k]);
    P.on = false;
  }
  return LBM_OK;
}

int lbm_profile_read(lbm_ctx* ctx, double* total_ms, int64_t* launches, int32_t n_kinds) {
  if (!ctx || !total_ms || !launches || n_kinds < 1) return LBM_EINVAL;
  if (ctx->err) return LBM_ESTATE;
  Profiler& P = ctx->prof;
  if (!P.on) return set_err(ctx, LBM_EINVAL, "profiling is not enabled");
  for (int r = 0; r < PROF_RING; ++r) {
    int rc = prof_harvest(ctx, r);
    if (rc) return rc;
  }
  for (int k = 0; k < n_kinds && k < PROF_KINDS; ++k) {
    total_ms[k] = P.total_ms[k];
    launches[k] = P.count[k];
  }
  return LBM_OK;
}

// device status words of every simulation (only = one simulation's)
static int check_status(lbm_ctx* ctx, int only = -1) {
  for (int si = 0; si < (int)ctx->sims.size(); ++si) {
    if (only >= 0 && si != only) continue;
    const SimHost& sh = ctx->sims[si];
    uint32_t cnt[4];
    HIPCHK(ctx, hipMemcpyAsync(cnt, sh.d.counters, sizeof cnt, hipMemcpyDeviceToHost, ctx->stream));
    HIPCHK(ctx, hipStreamSynchronize(ctx->stream));
    if (cnt[1] & ST_UNSTABLE)
      return set_err(ctx, LBM_EUNSTABLE, "unstable flow: NaN, rho <= 0 or |u| > 0.3");
    if (cnt[1] & ST_CONTACT_FULL)
      return set_err(ctx, LBM_ERANGE, "contact table or pair candidate list overflow");
    if (cnt[1] & ST_FRESH_FULL) return set_err(ctx, LBM_ERANGE, "fresh-node list overflow");
    if (cnt[1] & ST_OPEN_END)
      return set_err(ctx, LBM_ERANGE, "a particle came within R + 4 nodes of an open x end");
  }
  return LBM_OK;
}

int lbm_sync(lbm_ctx* ctx) {
  if (!ctx) return LBM_EINVAL;
  if (ctx->err) return LBM_ESTATE;
  HIPCHK(ctx, hipStreamSynchronize(ctx->stream));
  return check_status(ctx);
}

static SimHost* get_sim(lbm_ctx* ctx, int sim) {
  if (sim < 0 || sim >= (int)ctx->sims.size()) return nullptr;
  return &ctx->sims[sim];
}

int lbm_particles_sync(lbm_ctx* ctx, int32_t sim, int32_t dir, lbm_particle* parts, int32_t n,
                       double* history, int32_t max_steps, int32_t* n_hist) {
  if (!ctx) return LBM_EINVAL;
  if (ctx->err) return LBM_ESTATE;
  SimHost* sh = get_sim(ctx, sim);
  if (!sh) return set_err(ctx, LBM_ERANGE, "simulation index out of range");
  SimDev& d = sh->d;
  if (n != d.np || (n > 0 && !parts)) return set_err(ctx, LBM_EINVAL, "particle count mismatch");
  HIPCHK(ctx, hipStreamSynchronize(ctx->stream));
  int rc = check_status(ctx, sim);
  if (rc) return rc;
  if (n_hist) *n_hist = 0;
  if (d.np == 0) return LBM_OK;
  std::vector<DevParticle> hp(d.np);
  HIPCHK(ctx, hipMemcpyAsync(hp.data(), d.P, sizeof(DevParticle) * d.np, hipMemcpyDeviceToHost,
                             ctx->stream));
  HIPCHK(ctx, hipStreamSynchronize(ctx->stream));
  if (dir == 0) {
    for (int p = 0; p < d.np; ++p) {
      const DevParticle& s = hp[p];
      lbm_particle& o = parts[p];
      memset(&o, 0, sizeof o);
      for (int k = 0; k < 3; ++k) {
        o.x[k] = s.x[k];
        o.v[k] = s.v[k];
        o.w[k] = s.w[k];
        o.F_hyd[k] = s.Fh_last[k];
        o.T_hyd[k] = s.Th_last[k];
        o.F_cap[k] = s.Fcap[k];
        o.T_cap[k] = s.Tcap[k];
        o.F_con[k] = s.Fcon[k];
        o.T_con[k] = s.Tcon[k];
      }
      for (int k = 0; k < 4; ++k) o.q[k] = s.q[k];
      o.R = s.R;
      o.rho_p = s.rho_p;
      o.theta_deg = s.theta * 180.0 / M_PI;
      o.mu_s = s.mu_s;
      o.mu_r = s.mu_r;
      o.g_p = s.g_p;
      o.kinematic = s.kin;
    }
    if (history && max_steps > 0 && d.hist_cap > 0) {
      unsigned long long steps = 0;
      HIPCHK(ctx, hipMemcpyAsync(&steps, d.step_counter, sizeof steps, hipMemcpyDeviceToHost,
                                 ctx->stream));
      HIPCHK(ctx, hipStreamSynchronize(ctx->stream));
      const long long avail = (long long)std::min<unsigned long long>(steps, (unsigned long long)d.hist_cap);
      const long long cnt = std::min<long long>(avail, max_steps);
      std::vector<double> ring((size_t)d.hist_cap * d.np * LBM_HIST_DOUBLES);
      HIPCHK(ctx, hipMemcpyAsync(ring.data(), d.hist, sizeof(double) * ring.size(),
                                 hipMemcpyDeviceToHost, ctx->stream));
      HIPCHK(ctx, hipStreamSynchronize(ctx->stream));
      const size_t rec = (size_t)d.np * LBM_HIST_DOUBLES;
      for (long long k = 0; k < cnt; ++k) {
        const unsigned long long step = steps - cnt + k;
        memcpy(history + k * rec, ring.data() + (step % d.hist_cap) * rec, sizeof(double) * rec);
      }
      if (n_hist) *n_hist = (int32_t)cnt;
    }
    return LBM_OK;
  }
  if (dir != 1) return set_err(ctx, LBM_EINVAL, "dir must be 0 (pull) or 1 (push)");
  char msg[256];
  for (int p = 0; p < d.np; ++p) {
    if (!valid_particle(sh->cfg, parts[p], msg, sizeof msg)) return set_err(ctx, LBM_EINVAL, "%s", msg);
    if (parts[p].R > sh->Rmax)
      return set_err(ctx, LBM_ERANGE, "radius exceeds the largest radius the context was sized for");
  }
  for (int p = 0; p < d.np; ++p) {
    DevParticle& s = hp[p];
    for (int k = 0; k < 3; ++k) s.xo[k] = s.x[k];
    s.Ro = s.R;
    fill_dev_particle(s, parts[p], sh->cfg.delta_R, true);
  }
  HIPCHK(ctx, hipMemcpyAsync(d.P, hp.data(), sizeof(DevParticle) * d.np, hipMemcpyHostToDevice,
                             ctx->stream));
  HIPCHK(ctx, hipStreamSynchronize(ctx->stream));
  rc = post_dem_pipeline(ctx, sim, true);
  if (rc) return rc;
  return lbm_sync(ctx);
}

int lbm_fields(lbm_ctx* ctx, int32_t sim, uint32_t what, float* rho, float* u, float* phi,
               uint16_t* mask, void* pops, int32_t dst_is_device) {
  return lbm_fields2(ctx, sim, what, rho, u, phi, nullptr, mask, pops, dst_is_device);
}

int lbm_fields2(lbm_ctx* ctx, int32_t sim, uint32_t what, float* rho, float* u, float* phi,
                float* force, uint16_t* mask, void* pops, int32_t dst_is_device) {
  if (!ctx) return LBM_EINVAL;
  if (ctx->err) return LBM_ESTATE;
  SimHost* sh = get_sim(ctx, sim);
  if (!sh) return set_err(ctx, LBM_ERANGE, "simulation index out of range");
  SimDev& d = sh->d;
  const long long N = d.N;
  const hipMemcpyKind kind = dst_is_device ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost;
  if (what & (LBM_F_RHO | LBM_F_U | LBM_F_PHI | LBM_F_FORCE)) {
    // the spare population buffer holds the outputs: rho | phi | u | F (8N floats)
    float* scratch = (float*)d.pops[ctx->cur ^ 1];
    float* orho = scratch;
    float* ophi = scratch + N;
    float* ou = scratch + 2 * N;
    float* oF = scratch + 5 * N;
    const Batch b1 = batch_one(ctx, sim);
    HIPCHK(ctx, launch_interface(b1, sim_blocks(d), mom_blocks(d), ctx->stream));
    HIPCHK(ctx, launch_fused(b1, ctx->storage, sim_blocks(d), 1, orho, ou, ophi, oF, ctx->stream));
    if ((what & LBM_F_FORCE) && force)
      HIPCHK(ctx, hipMemcpyAsync(force, oF, 12 * N, kind, ctx->stream));
    if ((what & LBM_F_RHO) && rho)
      HIPCHK(ctx, hipMemcpyAsync(rho, orho, 4 * N, kind, ctx->stream));
    if ((what & LBM_F_PHI) && phi)
      HIPCHK(ctx, hipMemcpyAsync(phi, ophi, 4 * N, kind, ctx->stream));
    if ((what & LBM_F_U) && u) HIPCHK(ctx, hipMemcpyAsync(u, ou, 12 * N, kind, ctx->stream));
  }
  if ((what & LBM_F_MASK) && mask)
    HIPCHK(ctx, hipMemcpyAsync(mask, d.mask, 2 * N, kind, ctx->stream));
  if ((what & LBM_F_POPS) && pops)
    HIPCHK(ctx, hipMemcpyAsync(pops, d.pops[ctx->cur], sh->L.pop_bytes, kind, ctx->stream));
  return lbm_sync(ctx);
}

int lbm_links(lbm_ctx* ctx, int32_t sim, uint32_t* out, int32_t* pid, int64_t max, int64_t* count) {
  if (!ctx || !count) return LBM_EINVAL;
  if (ctx->err) return LBM_ESTATE;
  SimHost* sh = get_sim(ctx, sim);
  if (!sh) return set_err(ctx, LBM_ERANGE, "simulation index out of range");
  const SimDev& d = sh->d;
  std::vector<uint16_t> m(d.N);
  int rc = lbm_sync(ctx);
  if (rc) return rc;
  HIPCHK(ctx, hipMemcpyAsync(m.data(), d.mask, 2 * d.N, hipMemcpyDeviceToHost, ctx->stream));
  HIPCHK(ctx, hipStreamSynchronize(ctx->stream));
  int64_t cnt = 0;
  for (int p = 0; p < d.np; ++p)
    for (long long n = 0; n < d.N; ++n) {
      if (m[n] != 0) continue;
      const int x = (int)(n % d.nx), y = (int)((n / d.nx) % d.ny), z = (int)(n / ((long long)d.nx * d.ny));
      for (int i = 1; i < Q; ++i) {
        const long long t = (long long)wrapi(x + cx(i), d.nx) +
                            (long long)d.nx * ((long long)wrapi(y + cy(i), d.ny) +
                                               (long long)d.ny * wrapi(z + cz(i), d.nz));
        if (m[t] == 2 + p) {
          if (cnt < max) {
            if (out) out[cnt] = (uint32_t)((n << 5) | i);
            if (pid) pid[cnt] = p;
          }
          ++cnt;
        }
      }
    }
  *count = cnt;
  return LBM_OK;
}

int lbm_mass(lbm_ctx* ctx, int32_t sim, double out[2]) {
  if (!ctx || !out) return LBM_EINVAL;
  if (ctx->err) return LBM_ESTATE;
  SimHost* sh = get_sim(ctx, sim);
  if (!sh) return set_err(ctx, LBM_ERANGE, "simulation index out of range");
  SimDev& d = sh->d;
  HIPCHK(ctx, launch_zero_f64(d.mass_acc, 2, ctx->stream));
  HIPCHK(ctx, launch_mass(d, d.rp[ctx->rd ^ 1], d.mass_acc, ctx->stream));
  HIPCHK(ctx, hipMemcpyAsync(out, d.mass_acc, 2 * sizeof(double), hipMemcpyDeviceToHost, ctx->stream));
  return lbm_sync(ctx);
}

int lbm_mass_all_noalloc(lbm_ctx* ctx, double* out, int32_t dst_is_device) {
  if (!ctx || !out) return LBM_EINVAL;
  if (ctx->err) return LBM_ESTATE;
  const int n = (int)ctx->sims.size();
  if (n > LBM_NOALLOC_MAX_SIMS)
    return set_err(ctx, LBM_ERANGE,
                   "lbm_mass_all_noalloc: %d simulations exceed its scratch of %d", n,
                   LBM_NOALLOC_MAX_SIMS);
  double* acc = nullptr;
  const hipError_t e = noalloc_scratch(ctx->dev, &acc);
  if (e != hipSuccess || !acc)
    return set_err(ctx, LBM_EHIP, "lbm_mass_all_noalloc: no scratch address on device %d: %s",
                   ctx->dev, hipGetErrorString(e));
  hipStream_t st = ctx->stream;
  HIPCHK(ctx, launch_zero_f64(acc, 2 * n, st));
  for (int si = 0; si < n; ++si) {
    const SimDev& d = ctx->sims[si].d;
    HIPCHK(ctx, launch_mass(d, d.rp[ctx->rd ^ 1], acc + 2 * si, st));
  }
  HIPCHK(ctx, hipMemcpyAsync(out, acc, 2 * sizeof(double) * (size_t)n,
                             dst_is_device ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost, st));
  if (dst_is_device) return LBM_OK;
  return lbm_sync(ctx);
}

int lbm_dem_substeps(lbm_ctx* ctx, int32_t sim, int32_t* out) {
  if (!ctx || !out) return LBM_EINVAL;
  SimHost* sh = get_sim(ctx, sim);
  if (!sh) return LBM_ERANGE;
  *out = sh->d.n_sub;
  return LBM_OK;
}

void lbm_destroy(lbm_ctx* ctx) {
  if (!ctx) return;
  (void)hipStreamSynchronize(ctx->stream);
  if (ctx->graph_exec) (void)hipGraphExecDestroy(ctx->graph_exec);
  if (ctx->prof.on)
    for (int r = 0; r < PROF_RING; ++r)
      for (int k = 0; k < PROF_EVENTS; ++k) (void)hipEventDestroy(ctx->prof.ev[r][k]);
  delete ctx;
}

const char* lbm_last_error(const lbm_ctx* ctx) {
  if (!ctx || ctx->err == 0) return nullptr;
  return ctx->msg;
}

}  // extern "C"
