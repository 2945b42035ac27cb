// lbm_device.h -- device-side data structures and lattice constants shared by the
// HIP kernels of liblbm (gfx950).  Not part of the public ABI.
#pragma once
#include <hip/hip_runtime.h>
#include <hip/hip_fp16.h>
#include <stdint.h>

namespace lbm {

// ---------------------------------------------------------------- lattice
// D3Q19: rest, +-x, +-y, +-z, (+-1,+-1,0), (+-1,0,+-1), (0,+-1,+-1).
constexpr int Q = 19;
__host__ __device__ constexpr int cx(int i) {
  constexpr int t[Q] = {0, 1, -1, 0, 0, 0, 0, 1, 1, -1, -1, 1, 1, -1, -1, 0, 0, 0, 0};
  return t[i];
}
__host__ __device__ constexpr int cy(int i) {
  constexpr int t[Q] = {0, 0, 0, 1, -1, 0, 0, 1, -1, 1, -1, 0, 0, 0, 0, 1, 1, -1, -1};
  return t[i];
}
__host__ __device__ constexpr int cz(int i) {
  constexpr int t[Q] = {0, 0, 0, 0, 0, 1, -1, 0, 0, 0, 0, 1, -1, 1, -1, 1, -1, 1, -1};
  return t[i];
}
__host__ __device__ constexpr int opp(int i) {
  constexpr int t[Q] = {0, 2, 1, 4, 3, 6, 5, 10, 9, 8, 7, 14, 13, 12, 11, 18, 17, 16, 15};
  return t[i];
}
__host__ __device__ constexpr float wq(int i) {
  return i == 0 ? (1.0f / 3.0f) : (i <= 6 ? (1.0f / 18.0f) : (1.0f / 36.0f));
}
__host__ __device__ constexpr double wqd(int i) {
  return i == 0 ? (1.0 / 3.0) : (i <= 6 ? (1.0 / 18.0) : (1.0 / 36.0));
}

// interface normal n = G / max(|G|, EPS_G): the unit normal inside the diffuse
// interface, fading continuously to zero where phi is nearly uniform
constexpr float EPS_G = 1e-4f;
constexpr float EPS_GT = 1e-4f;  // tangential |G| below which wetting leaves G alone
constexpr float EPS_T = 1e-3f;   // capillary direction length below which a point is skipped
constexpr int MAXC = 16;        // contact slots per particle
constexpr int MAXNB = 24;       // DEM pair candidates per particle
constexpr uint16_t FRESH_BIT = 0x8000;
constexpr float PHI_SOLID = 4.0f;       // phi stored at solid nodes (never a fluid value)
constexpr float PHI_SOLID_TEST = 2.0f;  // phi above this marks a solid node

// -------------------------------------------------------------- particles
struct alignas(16) DevParticle {
  double x[3], v[3], w[3], q[4];
  double R, rho_p, theta, mu_s, mu_r, g_p;
  double mass, inertia, Rc;
  float neg_cos_t, sin_t;   // -cos(theta), sin(theta) for the wetting rotation
  int kin, pad;
  double Fh[3], Th[3];      // momentum exchange accumulators (FP64 atomics)
  double Fcap[3], Tcap[3];  // capillary force, last step
  double Fcon[3], Tcon[3];  // contact force, sub-step mean of the last step
  double Fcp[3], Tcp[3];    // contact force/torque of the last DEM sub-step
  double Fh_last[3], Th_last[3];  // momentum exchange of the last step (output copy)
  // DEM scratch
  double xo[3], Ro;         // centre and radius before the last update (mask release)
  double Ff[3], Tf[3];      // fluid force/torque held over the sub-steps (incl. gravity)
  double Facc[3], Tacc[3];  // contact sums over the sub-steps
  double ao[3], bo[3];      // accelerations at the start of the sub-step
  double vp[3], wp[3];      // predicted velocities
  double Fcn[3], Tcn[3];    // contact force/torque of the current sub-step
  double Ffp[3], Tfp[3];    // fluid force/torque of the previous lattice step
  double Fca[3], Tca[3];    // capillary accumulators (FP64 atomics)
  int havep, pad2;          // 1 once Ffp/Tfp hold a previous step
};

constexpr int LBM_HIST_DOUBLES_DEV = 27;

struct Contact {
  int partner;  // -1 wall surface, -2 wall underside, >= 0 particle, -100 free
  int pad;
  double xt[3], xr[3];
};

// ------------------------------------------------------------- simulation
// ------------------------------------------------------ population codecs
// Every population i of a node is held as a pair (d, g): d = f_i - w_i rho0 the
// deviation of the total population from rest, g = f^a_i - f^b_i the colour
// population.  Arguments: wr0 = w_i rho0; for FP16 the node's reference
// (R, P) enters as wR = w_i R and P.
//
// FP32: d and g stored as they are.
// FP16: h = (f - w_i R) / wr0 and k = (g - P f) / wr0, with (R, P) the node's
// density and order parameter of the previous step.  h and k then hold only
// the parts of f and g that the previous state does not predict (velocity,
// non-equilibrium, interface motion), not the Laplace pressure offset or the
// bulk colour, and keep FP16's relative precision for them.  In the bulk of
// either fluid (P = +-1, g = +-f) k is exactly 0, so g = +-f and phi = +-1 hold
// exactly after decoding.
// Global-memory view of a pointer.  Pointers read from the simulation table
// are generic to the compiler; the hot kernels convert them once so that every
// access compiles to a global (not flat) memory instruction.
#define GLB __attribute__((address_space(1)))
template <class T>
__device__ __forceinline__ GLB T* gp(T* p) {
  return (GLB T*)p;
}

template <int STORE>
struct Codec;

// iwr0 = 1 / (w_i rho0) (encoding multiplies by it)
template <>
struct Codec<0> {
  using T = float;
  template <class PD, class PG>
  static __device__ __forceinline__ void ld(PD pd, PG pg, float, float, float, float& d, float& g) {
    d = *pd;
    g = *pg;
  }
  template <class PD>
  static __device__ __forceinline__ float ld_d(PD pd, float, float) {
    return *pd;
  }
  template <class PD, class PG>
  static __device__ __forceinline__ void st(PD pd, PG pg, float, float, float, float, float d,
                                            float g) {
    *pd = d;
    *pg = g;
  }
};

// wr0 = w_i rho0, iwr0 = 1 / wr0, wR = w_i R; values stored as raw FP16 bits
template <>
struct Codec<1> {
  using T = uint16_t;
  static __device__ __forceinline__ float h2f(uint16_t v) { return __half2float(__ushort_as_half(v)); }
  static __device__ __forceinline__ uint16_t f2h(float v) {
    return __half_as_ushort(__float2half_rn(v));
  }
  template <class PD>
  static __device__ __forceinline__ float f_of(PD pd, float wr0, float wR) {
    return __fadd_rn(wR, __fmul_rn(wr0, h2f(*pd)));
  }
  template <class PD, class PG>
  static __device__ __forceinline__ void ld(PD pd, PG pg, float wr0, float wR, float P, float& d,
                                            float& g) {
    const float f = f_of(pd, wr0, wR);
    d = __fsub_rn(f, wr0);
    g = __fadd_rn(__fmul_rn(P, f), __fmul_rn(wr0, h2f(*pg)));
  }
  template <class PD>
  static __device__ __forceinline__ float ld_d(PD pd, float wr0, float wR) {
    return __fsub_rn(f_of(pd, wr0, wR), wr0);
  }
  template <class PD, class PG>
  static __device__ __forceinline__ void st(PD pd, PG pg, float wr0, float iwr0, float wR, float P,
                                            float d, float g) {
    const float f = __fadd_rn(d, wr0);
    *pd = f2h((f - wR) * iwr0);
    *pg = f2h(__fsub_rn(g, __fmul_rn(P, f)) * iwr0);
  }
};

// FP16 reference (R, P) of a node as floats; both the encoder and the decoder
// read it from the same stored pair
__device__ __forceinline__ float2 ref_of(const __half2* r, long long n) {
  return __half22float2(r[n]);
}
// the same from a global view of the pairs as 32-bit words
__device__ __forceinline__ float2 ref_of(const GLB uint32_t* r, long long n) {
  const uint32_t v = r[n];
  return make_float2(__half2float(__ushort_as_half((unsigned short)(v & 0xFFFFu))),
                     __half2float(__ushort_as_half((unsigned short)(v >> 16))));
}
__device__ __forceinline__ uint32_t ref_pack(float rho, float phi) {
  return (uint32_t)__half_as_ushort(__float2half_rn(rho)) |
         ((uint32_t)__half_as_ushort(__float2half_rn(phi)) << 16);
}
template <class T>
__device__ __forceinline__ const GLB uint32_t* gref(T* p) {
  return (const GLB uint32_t*)p;
}

struct SimDev {
  int nx, ny, nz, has_wall;
  long long N;
  int storage, np;
  float rho0, sigma, beta, inv2nua, inv2nub;
  float body[3];
  float wall_neg_cos, wall_sin;
  // fields
  void* pops[2];       // ping-pong population buffers: 38 planes of N
  __half2* ref[2];     // FP16 storage: per-node reference (rho, phi), ping-pong
  float* phi;          // order parameter of the current state (PHI_SOLID at solids)
  float* nrm;          // 4 planes of N: n_x, n_y, n_z (NaN at solids), |G| (-1 at solids)
  float2* curv;        // per node (CSF coefficient, solid-neighbour bits as float)
  uint16_t* mask;      // 0 fluid, 1 wall, 2+p particle p; FRESH_BIT while refilling
  uint32_t* claim;     // per node: lowest particle claiming it in the new mask, ~0u none
  uint32_t* fresh;     // fresh-node list: node index
  uint32_t* fresh_own; // fresh-node list: particle that uncovered it
  uint32_t* counters;  // [0] fresh count, [1] status flags, [2] fresh overflow
  uint32_t fresh_cap;
  // particles
  DevParticle* P;
  Contact* ct;         // np * MAXC
  int* nb;             // np * MAXNB candidate partners
  double* hist;        // hist_cap * np * 27
  int hist_cap;
  int n_sub;
  double kn, kt, kr, gn, gt, gr, delta_R;
  double cap_pref;     // sigma * 9/2 * k * beta (times sin(theta_p) per particle)
  double cap_dang;     // radians
  int cap_na, cap_nphi;
  int cap_B;           // side of the per-particle capillary box
  float4* capbox;      // np * B^3: (phi, Gx, Gy, Gz); phi = 2 marks a solid corner
  int* capbox_org;     // np * 3 box origins
  double* mass_acc;    // 2 doubles
  unsigned long long* step_counter;
  // node blocks of the per-node kernels (256 threads): tile_x = 0 runs 256
  // consecutive nodes per block; otherwise an x-y tile of tile_x by
  // 256 / tile_x nodes (tile_x = 1 << tile_lx), tiles_x by tiles_y per plane
  int tile_x, tile_lx, tiles_x, tiles_y;
};

// lattice node of thread threadIdx.x in block lb of simulation s; false if the
// thread lies outside the lattice
__device__ __forceinline__ bool tile_node(const SimDev& s, int lb, int& n, int& gx, int& gy,
                                          int& gz) {
  const int nx = s.nx, ny = s.ny;
  if (s.tile_x == 0) {
    n = lb * 256 + (int)threadIdx.x;
    if (n >= (int)s.N) return false;
    const int nxny = nx * ny;
    gz = n / nxny;
    const int rem = n - gz * nxny;
    gy = rem / nx;
    gx = rem - gy * nx;
    return true;
  }
  const int tx = (int)threadIdx.x & (s.tile_x - 1), ty = (int)threadIdx.x >> s.tile_lx;
  const int bx = lb % s.tiles_x, r = lb / s.tiles_x;
  const int by = r % s.tiles_y;
  gz = r / s.tiles_y;
  gx = bx * s.tile_x + tx;
  gy = by * (256 >> s.tile_lx) + ty;
  if (gx >= nx || gy >= ny) return false;
  n = gx + nx * (gy + ny * gz);
  return true;
}

enum StatusBits : uint32_t { ST_UNSTABLE = 1u, ST_CONTACT_FULL = 2u, ST_FRESH_FULL = 4u };

// One launch covers a batch of simulations (an ensemble, or a single one).
// Per-node kernels run 256-node blocks; blk[s] is the first global block of
// simulation s (blk[nsim] the total).  Particle kernels run one grid row per
// particle; pmap[row] = (simulation, particle).  With nsim == 1 the tables are
// not read: the block index is the simulation's own and row = particle.
// cur: population buffer holding the current state; rd: FP16 reference buffer
// it is encoded with (both uniform over the batch).
struct Batch {
  const SimDev* tab;
  const uint32_t* blk;
  const int2* pmap;
  int nsim;
  int cur, rd;
};

// (simulation, block within it) of global block g
__device__ __forceinline__ int2 batch_block(const Batch& b, int g) {
  if (b.nsim == 1) return make_int2(0, g);
  int lo = 0, hi = b.nsim;  // blk[lo] <= g < blk[hi]
  while (hi - lo > 1) {
    const int mid = (lo + hi) >> 1;
    if ((int)b.blk[mid] <= g)
      lo = mid;
    else
      hi = mid;
  }
  return make_int2(lo, g - (int)b.blk[lo]);
}

// (simulation, particle) of grid row r
__device__ __forceinline__ int2 batch_particle(const Batch& b, int r) {
  return b.nsim == 1 ? make_int2(0, r) : b.pmap[r];
}

__host__ __device__ inline int wrapi(int a, int n) {
  a %= n;
  return a < 0 ? a + n : a;
}
// minimum image: wrap once into (-L/2, L/2]
__host__ __device__ inline double wrapd(double d, double L) {
  if (d > 0.5 * L)
    d -= L;
  else if (d <= -0.5 * L)
    d += L;
  return d;
}

}  // namespace lbm
