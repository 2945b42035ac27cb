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
// phi stored at solid nodes (never a fluid value): PHI_SOLID + the node's mask
// code, 5 on the static wall, 6 + p inside particle p (exact in FP32), so that
// the stencils tell solids, and which solid, from phi alone; PHI_SOLID itself
// stands for the nodes beyond an open end
constexpr float PHI_SOLID = 4.0f;
constexpr float PHI_SOLID_TEST = 2.0f;  // phi above this marks a solid node
__host__ __device__ inline float solid_phi(uint32_t mask_code) { return PHI_SOLID + (float)mask_code; }

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
  int havep;                // 1 once Ffp/Tfp hold a previous step
  // 1: the capillary box of this step holds a fluid node with |G| near EPS_G
  // or above (set by the box kernel, cleared by the DEM with the accumulators)
  int cap_on;
};

constexpr int LBM_HIST_DOUBLES_DEV = 27;

// What a particle's contacts read of it: centre, contact radius, predicted
// velocities and friction coefficients (96 bytes).
struct DemView {
  double x[3], Rc, vp[3], mu_s, wp[3], mu_r;
};

struct Contact {
  int partner;  // -1 wall surface, -2 wall underside, >= 0 particle, -100 free
  int pad;
  double xt[3], xr[3];
};

// ------------------------------------------------------------- simulation
// ------------------------------------------------------ population codecs
// Only the total populations f_i are stored.  The colour populations are not:
// after the recolouring every streamed colour population is the source node's
// order parameter times f_i plus its segregation term, so the moments pass
// rebuilds them from f_i and the per-node (rho, phi, n) of the state that
// collided.  Kernels work with d = f_i - w_i rho0.  Arguments: wr0 = w_i rho0,
// iwr0 = 1 / wr0, wR = w_i R with R the reference density of the node that
// stores the population (FP16 only).
//
// FP32: d stored as it is.
// FP16: h = (f - w_i R) / wr0, R the node's density of the previous state: h
// holds only the part of f that the previous density does not predict
// (velocity, non-equilibrium), not the Laplace pressure offset, and keeps
// FP16's relative precision for it.
// Global-memory view of a pointer.  Pointers read from the simulation table
// are generic to the compiler; the hot kernels convert them once so that every
// access compiles to a global (not flat) memory instruction.
#define GLB __attribute__((address_space(1)))
// four floats as one 16-byte load or store (a clang vector, usable through GLB)
typedef float v4f __attribute__((ext_vector_type(4)));
template <class T>
__device__ __forceinline__ GLB T* gp(T* p) {
  return (GLB T*)p;
}

template <int STORE>
struct Codec;

template <>
struct Codec<0> {
  using T = float;
  template <class PD>
  static __device__ __forceinline__ float ld(PD pd, float, float) {
    return *pd;
  }
  template <class PD>
  static __device__ __forceinline__ void st(PD pd, float, float, float, float d) {
    *pd = d;
  }
};

// values stored as raw FP16 bits
template <>
struct Codec<1> {
  using T = uint16_t;
  static __device__ __forceinline__ float h2f(uint16_t v) { return __half2float(__ushort_as_half(v)); }
  static __device__ __forceinline__ uint16_t f2h(float v) {
    return __half_as_ushort(__float2half_rn(v));
  }
  template <class PD>
  static __device__ __forceinline__ float ld(PD pd, float wr0, float wR) {
    return __fsub_rn(__fadd_rn(wR, __fmul_rn(wr0, h2f(*pd))), wr0);
  }
  template <class PD>
  static __device__ __forceinline__ void st(PD pd, float wr0, float iwr0, float wR, float d) {
    const float f = __fadd_rn(d, wr0);
    *pd = f2h((f - wR) * iwr0);
  }
};

struct SimDev {
  int nx, ny, nz, has_wall;  // has_wall: 0 none, 1 the plane z = 0, 2 a tube along x
  // open x ends (pressure boundaries at x = -1/2 and nx - 1/2) and their
  // densities as departures from rho0 (formed in FP64: a small pressure drop
  // keeps its digits); tube radius squared and axis (has_wall 2)
  int open_x;
  float drho_in, drho_out;
  double tube_R2, tube_yc, tube_zc;
  // boxes of solid nodes on the plane (has_wall 3, a textured wall): per box
  // lo x, y, z, hi x, y, z (node indices, inclusive); the solid surface is the
  // box grown by half a node
  int n_boxes;
  int boxes[8][6];
  long long N;
  int storage, np;
  float rho0, sigma, beta, inv2nua, inv2nub;
  float body[3];
  float wall_neg_cos, wall_sin;
  // fields
  void* pops[2];       // ping-pong population buffers: 19 planes of N (f only)
  // per-node moments of a state, 2 planes of N: rho, then phi (rho0 and
  // PHI_SOLID at solids); rp[rd ^ 1] belongs to the state in pops[cur], rp[rd]
  // to the state before it (the FP16 reference of pops[cur])
  float* rp[2];
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
  DemView* view;       // 2 * np: the DEM's views of the particles, two sub-steps
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
  // blocks of the moments pass: x-y tiles of mtile_x (16, 32 or 64) by
  // 256 / mtile_x nodes
  // (mtile_x = 1 << mtile_lx), each over mkz planes; mtiles_x by mtiles_y
  // by mtiles_z of them
  int mtile_x, mtile_lx, mtiles_x, mtiles_y, mtiles_z, mkz;
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

enum StatusBits : uint32_t {
  ST_UNSTABLE = 1u,
  ST_CONTACT_FULL = 2u,
  ST_FRESH_FULL = 4u,
  ST_OPEN_END = 8u  // a particle came within R + 4 nodes of an open x end
};

// Static solid of the simulation at node (x, y, z): the plane z = 0; the
// outside of a tube of radius R_t about the axis through ((ny - 1)/2,
// (nz - 1)/2), solid iff dy^2 + dz^2 >= R_t^2 (dy, dz are multiples of 1/2, so
// the sum is exact in FP64); or the plane with its boxes.
__host__ __device__ inline bool static_wall(const SimDev& s, int x, int y, int z) {
  if (s.has_wall == 1) return z == 0;
  if (s.has_wall == 3) {
    if (z == 0) return true;
    for (int b = 0; b < s.n_boxes; ++b) {
      const int* B = s.boxes[b];
      if (x >= B[0] && x <= B[3] && y >= B[1] && y <= B[4] && z >= B[2] && z <= B[5]) return true;
    }
    return false;
  }
  if (s.has_wall == 2) {
    const double dy = (double)y - s.tube_yc, dz = (double)z - s.tube_zc;
    return dy * dy + dz * dz >= s.tube_R2;
  }
  return false;
}

// A particle keeps R + 4 nodes from an open x end: its mask box, links,
// capillary points and refill stay clear of the boundary planes.
__host__ __device__ inline bool near_open_end(const SimDev& s, double x, double R) {
  return s.open_x && (x < R + 4.0 || x > (double)(s.nx - 1) - R - 4.0);
}

// One launch covers a batch of simulations (an ensemble, or a single one).
// Per-node kernels run 256-node blocks; blk[s] is the first global block of
// simulation s (blk[nsim] the total).  Particle kernels run one grid row per
// particle; pmap[row] = (simulation, particle).  With nsim == 1 the tables are
// not read: the block index is the simulation's own and row = particle.
// cur: population buffer holding the current state; rd: moments buffer of the
// state before it (both uniform over the batch).
struct Batch {
  const SimDev* tab;
  const uint32_t* blk;
  const uint32_t* mblk;  // as blk, for the blocks of the moments pass
  const int2* pmap;
  int nsim;
  int cur, rd;
  int general;  // some simulation has open x ends, a tube or a textured wall
  int open;     // some simulation has open x ends
  int mlx;      // log2 of the moments tiles' x width if every simulation has the same, else 0
};

// (simulation, block within it) of global block g, given the block prefix blk
__device__ __forceinline__ int2 batch_block_in(const Batch& b, const uint32_t* blk, int g) {
  if (b.nsim == 1) return make_int2(0, g);
  int lo = 0, hi = b.nsim;  // blk[lo] <= g < blk[hi]
  while (hi - lo > 1) {
    const int mid = (lo + hi) >> 1;
    if ((int)blk[mid] <= g)
      lo = mid;
    else
      hi = mid;
  }
  return make_int2(lo, g - (int)blk[lo]);
}
// the per-node kernels' blocks
__device__ __forceinline__ int2 batch_block(const Batch& b, int g) {
  return batch_block_in(b, b.blk, g);
}

// (simulation, particle) of grid row r
__device__ __forceinline__ int2 batch_particle(const Batch& b, int r) {
  return b.nsim == 1 ? make_int2(0, r) : b.pmap[r];
}

// wrapped neighbour offsets of node (x, y, z): index of x + c is
// X[1+cx] + Y[1+cy] + Z[1+cz]
struct Nbr {
  int X[3], Y[3], Z[3];
  __device__ __forceinline__ Nbr(int gx, int gy, int gz, int nx, int ny, int nz) {
    // two multiplies; the wrapped rows and planes are a uniform offset away
    const int nxny = nx * ny, ylast = nxny - nx, zlast = nxny * (nz - 1);
    X[0] = gx == 0 ? nx - 1 : gx - 1;
    X[1] = gx;
    X[2] = gx == nx - 1 ? 0 : gx + 1;
    Y[1] = gy * nx;
    Y[0] = gy == 0 ? Y[1] + ylast : Y[1] - nx;
    Y[2] = gy == ny - 1 ? Y[1] - ylast : Y[1] + nx;
    Z[1] = gz * nxny;
    Z[0] = gz == 0 ? Z[1] + zlast : Z[1] - nxny;
    Z[2] = gz == nz - 1 ? Z[1] - zlast : Z[1] + nxny;
  }
  __device__ __forceinline__ int operator()(int i) const {
    return X[1 + cx(i)] + Y[1 + cy(i)] + Z[1 + cz(i)];
  }
};

// offset of population i of node n: blocks of 64 consecutive nodes, each
// holding its 19 populations as 19 runs of 64 values (a wave's 19 loads stay
// within 4.75 KB (FP32) instead of 19 planes apart); 19 N < 2^32
constexpr int POP_BLOCK = 64;
__device__ __forceinline__ unsigned pidx(int i, int N, int n) {
  (void)N;
  // n / 64 < 2^22 (19 N < 2^32): the full-rate 24-bit multiply suffices
  return __umul24((unsigned)n / POP_BLOCK, (unsigned)(Q * POP_BLOCK)) + (unsigned)i * POP_BLOCK +
         ((unsigned)n % POP_BLOCK);
}

// population 0 of node n; population i sits at i * POP_BLOCK past it (64-bit
// arithmetic, so that the 19 loads share one address and immediate offsets)
template <class T>
__device__ __forceinline__ T* pop_base(T* pops, int n) {
  return pops + ((size_t)((unsigned)n / POP_BLOCK) * (size_t)(Q * POP_BLOCK) +
                 (size_t)((unsigned)n % POP_BLOCK));
}

// element idx of a plane through a 32-bit byte offset from the plane's base
// (a plane holds fewer than 2^30 elements): with the base uniform the load takes
// the scalar-base form and one 32-bit register instead of a 64-bit address
template <class T>
__device__ __forceinline__ T at(const T* base, unsigned idx) {
  return *(const T*)((const char*)base + (unsigned)(idx * (unsigned)sizeof(T)));
}

// Moments of the post-stream state at fluid node n (order-parameter eq.), with
// the colour populations rebuilt from the state that collided.  The
// recolouring (recolouring eqs.) gave the population leaving x' in direction i
// the colour difference f^a_i - f^b_i = phi' f*_i + r' w_i (c_i . n'), with
// r' = beta rho' (1 - phi'^2) / 2 = 2 beta rho_a' rho_b' / rho'.  So f_i at x
// carries that of its source: x' = x - c_i if that node was fluid when the
// state streamed (its colour source is not NaN), else x itself, whose
// f*_opp(i) was bounced back (the moving-wall term of the bounce-back eqs. is
// coloured by phi(x) as well), giving phi(x) f_i - r(x) w_i (c_i . n(x)).
// Colour sources (phi, r n) of the state that collided; Rd: the FP16
// reference density of the stored populations at n.  Returns rabs = sum f_i,
// with f_i = d_i + w_i rho0 rounded as the collision formed it, and sg = sum of
// the colour differences: in the bulk of either fluid (phi' = +-1, r' = 0)
// sg = +-rabs exactly.
// c_i . a over the components where c_i is not zero, in the order x, y, z: equal
// to the full sum for finite a (the compiler keeps a zero term as 0 * a, since
// IEEE arithmetic does not fold it); -0 + v is v for every v
__device__ __forceinline__ float cdot(int i, float ax, float ay, float az) {
  float r = -0.0f;
  if (cx(i) != 0) r += (float)cx(i) * ax;
  if (cy(i) != 0) r += (float)cy(i) * ay;
  if (cz(i) != 0) r += (float)cz(i) * az;
  return r;
}

// The node's populations f_i - w_i rho0 (decoded with the reference density Rd).
template <int STORE, class PT>
__device__ __forceinline__ void load_pops(PT pops, int N, int n, float rho0, float Rd, float* d) {
  using IO = Codec<STORE>;
  (void)N;
  const auto pb = pop_base(pops, n);
#pragma unroll
  for (int i = 0; i < Q; ++i) d[i] = IO::ld(pb + i * POP_BLOCK, wq(i) * rho0, wq(i) * Rd);
}

// The sums from the populations d; CSRC(i): colour source of x - c_i
// (i = 1..18), own: that of x.
template <class CSRC>
__device__ __forceinline__ void colour_sums(const float* d, CSRC cs_src, const v4f own, float rho0,
                                            float& rabs, float& sg) {
  // f_i = d_i + w_i rho0 with one rounding (an explicit fused multiply-add:
  // left to the compiler, its contraction depends on where w_i rho0 is formed)
  rabs = __fmaf_rn(wq(0), rho0, d[0]);
  const float sg0 = own.x * rabs;
  // every source fluid: no selects.  A solid source carries NaN in r n, which
  // turns the sum to NaN; only then the sum is redone with the bounce rule.
  sg = sg0;
#pragma unroll
  for (int i = 1; i < Q; ++i) {
    const v4f c = cs_src(i);
    const float fi = __fmaf_rn(wq(i), rho0, d[i]);
    rabs += fi;
    sg += c.x * fi + wq(i) * cdot(i, c.y, c.z, c.w);
  }
  if (sg != sg) {
    sg = sg0;
#pragma unroll
    for (int i = 1; i < Q; ++i) {
      const v4f c = cs_src(i);
      // an all-NaN source: the population entered through an open end (the
      // anti-bounce-back, applied to each fluid with the node's colour shares,
      // gives phi(x) f_i + r(x) w_i (c_i . n(x)))
      const bool open = c.x != c.x;
      const bool solid = c.y != c.y;
      const float fi = __fmaf_rn(wq(i), rho0, d[i]);
      const float ts = cdot(i, c.y, c.z, c.w);
      const float to = cdot(i, own.y, own.z, own.w);
      const float ph = solid ? own.x : c.x;
      const float t = open ? to : (solid ? -to : ts);
      sg += ph * fi + wq(i) * t;
    }
  }
}

// Colour source (phi, r n_x, r n_y, r n_z) of node m of the state that
// collided, r = beta rho (1 - phi^2) / 2, from its moments RO (rho plane, phi
// plane) and normal planes NX; NaN in r n at a solid node (its normal is NaN).
__device__ __forceinline__ v4f colour_record(float rho, float phi, float nx, float ny, float nz,
                                             float hb) {
  const float r = hb * rho * (1.0f - phi) * (1.0f + phi);
  return v4f{phi, r * nx, r * ny, r * nz};
}
__device__ __forceinline__ v4f colour_source(const GLB float* RO, const GLB float* NX, int N,
                                             int m, float hb) {
  const unsigned u = (unsigned)m;
  return colour_record(at(RO, u), at(RO + N, u), at(NX, u), at(NX + N, u), at(NX + 2 * N, u), hb);
}

// both, for one node, with the colour sources read from the global planes
template <int STORE, class PT>
__device__ __forceinline__ void rebuild_moments(PT pops, const GLB float* RO, const GLB float* NX,
                                                int N, int n, const Nbr& nb, float rho0, float hb,
                                                float Rd, float& rabs, float& sg) {
  float d[Q];
  load_pops<STORE>(pops, N, n, rho0, Rd, d);
  colour_sums(
      d, [&](int i) { return colour_source(RO, NX, N, nb(opp(i)), hb); },
      colour_source(RO, NX, N, n, hb), rho0, rabs, sg);
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
