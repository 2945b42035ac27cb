// lbm_fluid.hip -- lattice kernels of liblbm for gfx950.
//
// Storage: the 19 total populations f of each node, in blocks of 64 nodes (19
// runs of 64 values; see pidx).  The colour is carried by the per-node order
// parameter; the colour populations are rebuilt by the moments pass (see
// rebuild_moments).
// FP32 storage keeps the deviation d_i = f_i - w_i rho0 (so that the small
// velocity survives FP32 rounding); FP16 storage keeps
// h_i = (f_i - w_i R) / (w_i rho0) with R the node's density of the previous
// state.  All arithmetic is FP32; momentum exchange sums are FP64.
//
// A step of the fluid runs k_interface (interface normal, curvature and CSF
// coefficient from phi, in one z-march), k_fused (collision, force, streaming and
// bounce-back of f, one thread per node, reading and writing every population
// exactly once), k_links (moving-wall terms and momentum exchange at particle
// links) and k_moments (density and order parameter of the post-stream state).
#include "lbm_device.h"

namespace lbm {

// ------------------------------------------------------------ wetting rotation
// Geometric wetting (n_pm equation): at a fluid node with a solid neighbour the
// colour gradient is rotated to make the angle theta (through fluid a) with the
// solid's outward normal n_s, keeping |G|: G <- |G| (-cos(theta) n_s + sin(theta) t^),
// t = n* - (n*.n_s) n_s.  The solid is the lowest-index neighbouring particle,
// else the wall.  Applied inside the diffuse interface (|G| > EPS_G); left
// unchanged if the tangential part |G - (G.n_s) n_s| <= EPS_GT (axis undefined).
// Between those thresholds and twice their value the rotated vector is blended
// in with weight w = min(1, |t|/EPS_GT - 1) min(1, |G|/EPS_G - 1), so that G is
// continuous in phi (no last-bit difference can switch the rotation on or off).
// GENERAL: the tube's wall normal is compiled in.
template <bool GENERAL = true>
__device__ __forceinline__ void wetting_rotate(const SimDev& s, int gx, int gy, int gz, int minp,
                                               bool wall_nb, float& Gx, float& Gy, float& Gz) {
  float g = sqrtf(Gx * Gx + Gy * Gy + Gz * Gz);
  if (!(g > EPS_G)) return;
  float nsx, nsy, nsz, nc, ns;
  if (minp >= 0) {
    // in FP64, rounded once to FP32 (the wetting direction next to a particle
    // moves the velocity there at the 1e-5 level)
    const DevParticle& P = s.P[minp];
    const double dx = wrapd((double)gx - P.x[0], (double)s.nx);
    const double dy = wrapd((double)gy - P.x[1], (double)s.ny);
    const double dz = wrapd((double)gz - P.x[2], (double)s.nz);
    const double idn = 1.0 / sqrt(dx * dx + dy * dy + dz * dz);
    nsx = (float)(dx * idn);
    nsy = (float)(dy * idn);
    nsz = (float)(dz * idn);
    nc = P.neg_cos_t;
    ns = P.sin_t;
  } else if (wall_nb && (!GENERAL || s.has_wall == 1)) {
    nsx = 0.f;
    nsy = 0.f;
    nsz = (gz == 1) ? 1.f : -1.f;
    nc = s.wall_neg_cos;
    ns = s.wall_sin;
  } else if (wall_nb && s.has_wall == 3) {
    // textured wall: the normal of the nearest point of the solid surface (the
    // plane's top face z = 1/2, or its underside z = nz - 1/2 through the
    // periodic z direction; the boxes grown by half a node), from it to the
    // node; on ties the plane, then the lowest box index
    // (distances compared squared: node and surface coordinates are
    // multiples of 1/2, so the squares are exact; one square root, for the
    // winner)
    const double dt = (double)gz - 0.5, du = ((double)s.nz - 0.5) - (double)gz;
    const double dp = dt <= du ? dt : du;
    double best2 = dp * dp;
    double bx = 0.0, by = 0.0, bz = dt <= du ? 1.0 : -1.0;
    bool boxed = false;
    for (int b = 0; b < s.n_boxes; ++b) {
      const int* B = s.boxes[b];
      const double p[3] = {(double)gx, (double)gy, (double)gz};
      double d[3];
      for (int k = 0; k < 3; ++k) {
        const double lo = B[k] - 0.5, hi = B[3 + k] + 0.5;
        d[k] = p[k] - (p[k] < lo ? lo : (p[k] > hi ? hi : p[k]));
      }
      const double d2 = d[0] * d[0] + d[1] * d[1] + d[2] * d[2];
      if (d2 > 0.0 && d2 < best2) {
        best2 = d2;
        bx = d[0];
        by = d[1];
        bz = d[2];
        boxed = true;
      }
    }
    if (boxed) {
      const double idn = 1.0 / sqrt(best2);
      bx *= idn;
      by *= idn;
      bz *= idn;
    }
    nsx = (float)bx;
    nsy = (float)by;
    nsz = (float)bz;
    nc = s.wall_neg_cos;
    ns = s.wall_sin;
  } else if (wall_nb) {
    // tube: the wall's outward normal points from the node to the axis
    const double dy = (double)gy - s.tube_yc, dz = (double)gz - s.tube_zc;
    const double r = sqrt(dy * dy + dz * dz);
    if (!(r > 0.0)) return;
    nsx = 0.f;
    nsy = (float)(-dy / r);
    nsz = (float)(-dz / r);
    nc = s.wall_neg_cos;
    ns = s.wall_sin;
  } else {
    return;
  }
  float a = Gx * nsx + Gy * nsy + Gz * nsz;
  float tx = Gx - a * nsx, ty = Gy - a * nsy, tz = Gz - a * nsz;
  float tn = sqrtf(tx * tx + ty * ty + tz * tz);
  if (!(tn > EPS_GT)) return;
  float it = 1.0f / tn;
  const float rx = g * (nc * nsx + ns * tx * it);
  const float ry = g * (nc * nsy + ns * ty * it);
  const float rz = g * (nc * nsz + ns * tz * it);
  const float w = fminf(1.0f, tn / EPS_GT - 1.0f) * fminf(1.0f, g / EPS_G - 1.0f);
  if (w >= 1.0f) {
    Gx = rx;
    Gy = ry;
    Gz = rz;
  } else {
    Gx += w * (rx - Gx);
    Gy += w * (ry - Gy);
    Gz += w * (rz - Gz);
  }
}

// One direction of each opposite pair: +x, +y, +z, (1,1,0), (1,-1,0), (1,0,1),
// (1,0,-1), (0,1,1), (0,1,-1).
__host__ __device__ constexpr int pair_dir(int k) {
  constexpr int t[9] = {1, 3, 5, 7, 8, 11, 12, 15, 16};
  return t[k];
}

// index of halo record j of thread t
__device__ __forceinline__ int k_of(int t, int j) { return t + 256 * j; }

// XCD-aware block order: consecutive dispatches go round-robin over the 8 XCDs;
// give each XCD a contiguous range of blocks so that data shared by neighbouring
// blocks (halo reads, pushed populations) meets in the same L2.
__device__ __forceinline__ int xcd_tile(int lin, int nblk) {
  if ((nblk & 7) == 0) {
    const int per = nblk >> 3;
    return (lin & 7) * per + (lin >> 3);
  }
  return lin;
}

// ------------------------------------------------------------- moments kernel
// Density and order parameter phi = sum g / rho (order-parameter eq.) of every
// fluid node of the post-stream state into rp[rd ^ 1], the colour populations
// rebuilt from the state that collided (the colour source (phi, r n) of each
// node, formed from its moments and normal).  Runs after the
// refill, which has written the moments of the fresh nodes; clears their FRESH
// mark.  Solid nodes get (rho0, solid_phi(mask)), so that stencils can tell solids
// from phi alone.
//
// A block takes an x-y tile of the simulation's moments tiling and marches up
// s.mkz planes.  The colour sources of three planes of the tile grown by one
// node sit in an LDS ring; each plane adds the sources of the plane above.
constexpr int MOM_HALO = 66 * 6;  // largest tile plane grown by one: (64 + 2)(4 + 2)
// LX: log2 of the tiles' x width when the launch fixes it (the tile's LDS
// offsets are then immediates), 0 to read it from the simulation
template <int STORE, int LX>
__global__ __launch_bounds__(256) void k_moments(Batch bt) {
  using IO = Codec<STORE>;
  using T = typename IO::T;
  __shared__ v4f ring[3][MOM_HALO];
  const int2 sb = batch_block_in(bt, bt.mblk, blockIdx.x);
  const SimDev& s = bt.tab[sb.x];
  const int N = (int)s.N;
  const int nx = s.nx, ny = s.ny, nz = s.nz, P = nx * ny;
  if (sb.y == 0 && threadIdx.x == 0) s.counters[0] = 0u;  // fresh list consumed
  const GLB float* __restrict__ NX = gp((const float*)s.nrm);
  const float hb = 0.5f * s.beta;
  const GLB T* __restrict__ pops = gp((const T*)s.pops[bt.cur]);
  const GLB float* __restrict__ RO = gp((const float*)s.rp[bt.rd]);
  GLB float* __restrict__ RN = gp(s.rp[bt.rd ^ 1]);
  GLB uint16_t* __restrict__ MASK = gp(s.mask);
  const int tlx = LX > 0 ? LX : s.mtile_lx;
  const int tx = 1 << tlx, ty = 256 >> tlx, HX = tx + 2, HY = ty + 2;
  const int bx = sb.y % s.mtiles_x, r = sb.y / s.mtiles_x;
  const int by = r % s.mtiles_y, z0 = (r / s.mtiles_y) * s.mkz;
  const int kz = min(s.mkz, nz - z0);
  const int t = (int)threadIdx.x;
  const int lx = t & (tx - 1), ly = t >> tlx;
  const int gx = bx * tx + lx, gy = by * ty + ly;
  const bool in = gx < nx && gy < ny;
  // this thread's halo records of a plane: t and t + 256 (a plane has at
  // most 396); past a partial tile's end they are only kept in bounds
  // (-1: beyond an open x end; its record is all NaN, the mark of a
  // population that entered through the pressure boundary)
  int hoff[2];
  bool hon[2];
#pragma unroll
  for (int j = 0; j < 2; ++j) {
    const int k = t + 256 * j;
    hon[j] = k < HX * HY;
    const int hy = k / HX, hx = k - hy * HX;
    int x = bx * tx - 1 + hx, y = by * ty - 1 + hy;
    const bool out = s.open_x && (x < 0 || x >= nx);
    x = x < 0 ? x + nx : (x >= nx ? x - nx : x);
    y = y < 0 ? y + ny : (y >= ny ? y - ny : y);
    hoff[j] = !hon[j] ? 0 : out ? -1 : min(x, nx - 1) + nx * min(y, ny - 1);
  }
  const float qnan = __int_as_float(0x7fc00000);
  const v4f open_rec = v4f{qnan, qnan, qnan, qnan};
  auto zwrap = [&](int z) { return z < 0 ? z + nz : (z >= nz ? z - nz : z); };
  // planes z0 - 1 and z0 into the ring
#pragma unroll
  for (int dz = 0; dz < 2; ++dz) {
    const int zp = zwrap(z0 - 1 + dz);
#pragma unroll
    for (int j = 0; j < 2; ++j)
      if (hon[j])
        ring[(z0 + 2 + dz) % 3][k_of(t, j)] =
            hoff[j] < 0 ? open_rec : colour_source(RO, NX, N, hoff[j] + P * zp, hb);
  }
  // Each plane takes one round of global loads: the node's populations and
  // the raw moments and normal of the next plane's halo records, all issued
  // before the first wait (indices clamped in bounds instead of branches, which
  // would wait inside them); the records are formed once the loads are in.
  float sr[2][5];
  auto fetch_raw = [&](int z) {
    const int zp = zwrap(z + 1);
#pragma unroll
    for (int j = 0; j < 2; ++j) {
      const int m = max(hoff[j], 0) + P * zp;
      sr[j][0] = RO[m];
      sr[j][1] = RO[N + m];
      sr[j][2] = NX[m];
      sr[j][3] = NX[N + m];
      sr[j][4] = NX[2 * N + m];
    }
  };
  const int gxc = min(gx, nx - 1), gyc = min(gy, ny - 1);
  const float rho0 = s.rho0;  // kept in a register: the stores below may alias s
  // a plane's results are stored once the next plane's loads are in, so that
  // they are in flight during the sums instead of ahead of the next loads
  int pn = -1;
  uint16_t pm = 0;
  float prabs = 0.f, psg = 0.f;
  auto store_pending = [&]() {
    if (pn < 0) return;
    if (pm & FRESH_BIT) {  // refilled node: moments written by the refill
      MASK[pn] = (uint16_t)(pm & ~FRESH_BIT);
    } else if (pm != 0) {
      RN[pn] = rho0;
      RN[N + pn] = solid_phi(pm);
    } else {
      RN[pn] = prabs;
      RN[N + pn] = psg / prabs;
    }
  };
  for (int zz = 0; zz < kz; ++zz) {
    const int z = z0 + zz;
    const int n = gxc + nx * (gyc + ny * z);
    float d[Q];
    const uint16_t m = MASK[n];
    load_pops<STORE>(pops, N, n, rho0, STORE ? RO[n] : 0.f, d);
    fetch_raw(z);
#pragma unroll
    for (int j = 0; j < 2; ++j)
      if (hon[j])
        ring[(z + 1) % 3][k_of(t, j)] =
            hoff[j] < 0 ? open_rec
                        : colour_record(sr[j][0], sr[j][1], sr[j][2], sr[j][3], sr[j][4], hb);
    store_pending();
    __syncthreads();
    if (in) {
      const int c0 = (lx + 1) + HX * (ly + 1);
      colour_sums(
          d, [&](int i) { return ring[(z + 3 - cz(i)) % 3][c0 - cx(i) - HX * cy(i)]; },
          ring[z % 3][c0], rho0, prabs, psg);
      pn = n;
      pm = m;
    }
    __syncthreads();
  }
  store_pending();
}

// Between steps, after the mask changed with the populations in place (and
// the refill of fresh nodes): solid nodes get (rho0, solid_phi(mask)), fresh nodes
// lose their mark, fluid nodes keep their moments.
__global__ __launch_bounds__(256) void k_moments_boundary(Batch bt) {
  const int2 sb = batch_block(bt, blockIdx.x);
  const SimDev& s = bt.tab[sb.x];
  int n, gx, gy, gz;
  if (sb.y == 0 && threadIdx.x == 0) s.counters[0] = 0u;
  if (!tile_node(s, sb.y, n, gx, gy, gz)) return;
  const uint16_t m = s.mask[n];
  if (m & FRESH_BIT) {
    s.mask[n] = (uint16_t)(m & ~FRESH_BIT);
  } else if (m != 0) {
    float* RN = s.rp[bt.rd ^ 1];
    RN[n] = s.rho0;
    RN[s.N + n] = solid_phi(m);
  }
}

// ------------------------------------------------------------ init kernels
__global__ void k_init_mask(SimDev s) {
  long long n = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (n >= s.N) return;
  int z = (int)(n / ((long long)s.nx * s.ny));
  const int x = (int)(n % s.nx), y = (int)((n / s.nx) % s.ny);
  s.mask[n] = static_wall(s, x, y, z) ? 1 : 0;
  s.claim[n] = 0xFFFFFFFFu;
}

// fluid at rest: f = w rho0 (d = 0), moments (rho0, phi0) in both moment
// buffers (phi0 staged in the phi plane of rp[0]; (rho0, solid_phi(mask)) at solids)
template <int STORE>
__global__ void k_init_pops(SimDev s, void* pops) {
  using IO = Codec<STORE>;
  using T = typename IO::T;
  long long n = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (n >= s.N) return;
  T* b = (T*)pops;
#pragma unroll
  for (int i = 0; i < Q; ++i) {
    const float wr0 = wq(i) * s.rho0;
    IO::st(b + pidx(i, (int)s.N, (int)n), wr0, 1.0f / wr0, wr0, 0.f);
  }
  const uint16_t m0 = s.mask[n];
  const float p0 = (m0 == 0) ? s.rp[0][s.N + n] : solid_phi(m0);
  for (int k = 0; k < 2; ++k) {
    s.rp[k][n] = s.rho0;
    s.rp[k][s.N + n] = p0;
  }
}

// --------------------------------------------------------- global mass (FP64)
// masses of fluids a and b, sum of rho (1 +- phi) / 2 over fluid nodes, from
// the moments rp (rho plane, phi plane) of the current state, added into
// acc[0], acc[1] (cleared by the caller)
__global__ __launch_bounds__(256) void k_mass(SimDev s, const float* __restrict__ rp,
                                              double* __restrict__ acc) {
  __shared__ double sh[2][256];
  double a = 0.0, b = 0.0;
  for (long long n = (long long)blockIdx.x * blockDim.x + threadIdx.x; n < s.N;
       n += (long long)gridDim.x * blockDim.x) {
    if (s.mask[n] != 0) continue;
    const double rho = (double)rp[n], sg = rho * (double)rp[s.N + n];
    a += 0.5 * (rho + sg);
    b += 0.5 * (rho - sg);
  }
  sh[0][threadIdx.x] = a;
  sh[1][threadIdx.x] = b;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if ((int)threadIdx.x < o) {
      sh[0][threadIdx.x] += sh[0][threadIdx.x + o];
      sh[1][threadIdx.x] += sh[1][threadIdx.x + o];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    atomicAdd(&acc[0], sh[0][0]);
    atomicAdd(&acc[1], sh[1][0]);
  }
}

// n doubles set to zero (a kernel, not a memset: safe inside a captured graph)
__global__ void k_zero_f64(double* __restrict__ p, int n) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = 0.0;
}

enum { MODE_STEP = 0, MODE_FIELDS = 1 };

// ------------------------------------------------------ interface kernels
// Colour gradient G = 3 sum_i w_i c_i phi(x + c_i) (isotropic stencil, the value
// at x for solid neighbours), the geometric wetting rotation next to solids,
// the normal n = G / max(|G|, EPS_G); then the curvature kappa = div n (same
// stencil and closure), the CSF coefficient c = -sigma kappa max(|G|, EPS_G) / 2
// (the surface-tension force is c n) and the set of directions whose neighbour
// is solid (bit i, bit 31 = node solid).  Written: the normal planes (n_x, n_y,
// n_z, |G|; NaN and -1 at a solid node) and the curvature word.
//
// One kernel: a block takes an x-y tile of the moments tiling and marches up
// its s.mkz planes.  phi of the tile grown by two nodes sits in an LDS ring of
// four planes, the normals of the tile grown by one node in a ring of three;
// per plane z the block loads phi of plane z + 2, forms the normals of plane
// z + 1 on the grown tile (a node's normal is formed once per block that needs
// it: 1.55 times per node for 64 x 4 tiles) and the curvature of plane z.  The
// normals never travel to HBM and back between the two stencils.
constexpr int IF_PHI = 68 * 8;          // largest tile plane grown by two: (64 + 4)(4 + 4)
constexpr int IF_NRM = MOM_HALO;  // grown by one: (64 + 2)(4 + 2)
// OPEN: the batch has simulations with open x ends or a tube wall (a
// separate instance, so that the periodic box on a plane carries none of their
// bookkeeping).
// LX: as for the moments pass
template <bool OPEN, int LX>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(6, 8))) void k_interface(Batch bt) {
  __shared__ float fring[4][IF_PHI];
  // normals of three planes, one array per component (the curvature reads
  // only the components its stencil direction needs); |G| only where the
  // curvature needs it, at the tile's own nodes
  __shared__ float nrx[3][IF_NRM], nry[3][IF_NRM], nrz[3][IF_NRM], nrg[3][256];
  const int2 sb = batch_block_in(bt, bt.mblk, blockIdx.x);
  const SimDev& s = bt.tab[sb.x];
  const int N = (int)s.N;
  const GLB float* __restrict__ PHI = gp((const float*)s.rp[bt.rd ^ 1]) + s.N;
  GLB float* __restrict__ NX = gp(s.nrm);
  GLB float* __restrict__ CUR = gp((float*)s.curv);
  const int nx = s.nx, ny = s.ny, nz = s.nz, P = nx * ny;
  const int tlx = LX > 0 ? LX : s.mtile_lx;
  const int tx = 1 << tlx, ty = 256 >> tlx;
  const int FX = tx + 4, FY = ty + 4, HX = tx + 2, HY = ty + 2;
  const int bx = sb.y % s.mtiles_x, r = sb.y / s.mtiles_x;
  const int by = r % s.mtiles_y, z0 = (r / s.mtiles_y) * s.mkz;
  const int kz = min(s.mkz, nz - z0);
  const int t = (int)threadIdx.x;
  const int lx = t & (tx - 1), ly = t >> tlx;
  const int gx = bx * tx + lx, gy = by * ty + ly;
  const bool in = gx < nx && gy < ny;
  const int x0 = bx * tx, y0 = by * ty;
  // this thread's phi region entries (t, t + 256, t + 512): plane offsets
  // (-1: beyond an open x end, where phi reads as a solid's: the gradient and
  // curvature take the node's own value there and the direction is flagged)
  int foff[3];
  bool fon[3];
#pragma unroll
  for (int j = 0; j < 3; ++j) {
    const int k = t + 256 * j;
    fon[j] = k < FX * FY;
    const int fy = k / FX, fx = k - fy * FX;
    const int ax = x0 - 2 + fx;
    foff[j] = !fon[j] ? 0
              : (OPEN && s.open_x && (ax < 0 || ax >= nx)) ? -1
                                                   : wrapi(ax, nx) + nx * wrapi(y0 - 2 + fy, ny);
  }
  // this thread's normal region entries: first its own column and row of the
  // region's first tx x ty entries, then the region's two top rows and its
  // two right columns (2 tx + 2 ty + 4 <= 256 entries for the tiles used), so
  // that a wave's entries lie in whole rows: its phi reads are consecutive
  // LDS words (taken in region order, a wave's 64 entries crossed a row end,
  // and two of them met in one LDS bank)
  int hx_[2], hy_[2];
  bool hon[2];
  hx_[0] = lx;
  hy_[0] = ly;
  hon[0] = true;
  {
    const int u = t - 2 * tx;
    hon[1] = u < 2 * HY;
    hx_[1] = u < 0 ? lx : tx + (u & 1);
    hy_[1] = u < 0 ? ty + (t >> tlx) : (u >> 1);
  }
  auto zw = [&](int z) { return wrapi(z, nz); };
  auto fslot = [&](int z) { return (z + 8) & 3; };  // z >= -2
  auto nslot = [&](int z) { return (z + 3) % 3; };   // z >= -1
  auto load_phi = [&](int z, float* v) {
    const int zp = zw(z);
#pragma unroll
    for (int j = 0; j < 3; ++j)
      v[j] = !fon[j] ? 0.f : (OPEN && foff[j] < 0) ? PHI_SOLID : PHI[foff[j] + P * zp];
  };
  auto store_phi = [&](int z, const float* v) {
#pragma unroll
    for (int j = 0; j < 3; ++j)
      if (fon[j]) fring[fslot(z)][t + 256 * j] = v[j];
  };
  const float qnan = __int_as_float(0x7fc00000);
  // normal of region entry (hx, hy) of plane z from the phi ring
  // SOL: a solid (or open-end) node may lie in the three phi planes read;
  // without, the per-neighbour tests are left out (a block-uniform choice)
  auto normal = [&](int hx, int hy, int z, auto SOL) -> v4f {
    const int c = (hx + 1) + FX * (hy + 1);
    const float* fm = fring[fslot(z - 1)];
    const float* f0 = fring[fslot(z)];
    const float* fp = fring[fslot(z + 1)];
    const float p0 = f0[c];
    if (decltype(SOL)::value && !(p0 < PHI_SOLID_TEST)) return v4f{qnan, qnan, qnan, -1.0f};
    float Gx = 0.f, Gy = 0.f, Gz = 0.f;
    bool solid = false;
#pragma unroll
    for (int q = 0; q < 9; ++q) {
      const int i = pair_dir(q);
      const float* sp_ = cz(i) > 0 ? fp : (cz(i) < 0 ? fm : f0);
      const float* sm_ = cz(i) > 0 ? fm : (cz(i) < 0 ? fp : f0);
      float vp = sp_[c + cx(i) + FX * cy(i)];
      float vm = sm_[c - cx(i) - FX * cy(i)];
      if constexpr (decltype(SOL)::value) {
        const bool spd = vp > PHI_SOLID_TEST, smd = vm > PHI_SOLID_TEST;
        solid |= spd | smd;
        vp = spd ? p0 : vp;
        vm = smd ? p0 : vm;
      }
      // G += 3 w_i c_i (phi(x + c_i) - phi(x - c_i)), each term one fused
      // multiply-add; terms with a zero lattice coefficient add nothing and are
      // left out (the compiler keeps 0 * d, which IEEE arithmetic does not fold)
      const float k = 3.0f * wq(i), df = vp - vm;
      if (cx(i) != 0) Gx = __fmaf_rn((float)cx(i) * k, df, Gx);
      if (cy(i) != 0) Gy = __fmaf_rn((float)cy(i) * k, df, Gy);
      if (cz(i) != 0) Gz = __fmaf_rn((float)cz(i) * k, df, Gz);
    }
    // the wetting rotation applies only inside the interface (|G| > EPS_G, its
    // own first test); only there the solid is identified, from the phi
    // codes of the neighbours in the ring: the lowest-index particle, else
    // the wall (an open end is neither)
    if (decltype(SOL)::value && solid && sqrtf(Gx * Gx + Gy * Gy + Gz * Gz) > EPS_G) {
      float pmin = 3.0e38f;
      bool wall = false;
#pragma unroll
      for (int q = 0; q < 9; ++q) {
        const int i = pair_dir(q);
        const float* sp_ = cz(i) > 0 ? fp : (cz(i) < 0 ? fm : f0);
        const float* sm_ = cz(i) > 0 ? fm : (cz(i) < 0 ? fp : f0);
        const float vp = sp_[c + cx(i) + FX * cy(i)];
        const float vm = sm_[c - cx(i) - FX * cy(i)];
        wall |= vp == solid_phi(1) || vm == solid_phi(1);
        if (vp >= solid_phi(2)) pmin = fminf(pmin, vp);
        if (vm >= solid_phi(2)) pmin = fminf(pmin, vm);
      }
      if (wall || pmin < 3.0e38f) {
        const int ax = wrapi(x0 - 1 + hx, nx), ay = wrapi(y0 - 1 + hy, ny), az = zw(z);
        const int minp = pmin < 3.0e38f ? (int)(pmin - solid_phi(2)) : -1;
        wetting_rotate<OPEN>(s, ax, ay, az, minp, wall, Gx, Gy, Gz);
      }
    }
    const float g = sqrtf(Gx * Gx + Gy * Gy + Gz * Gz);
    // 1 / max(g, EPS_G): the hardware reciprocal (within 1 ulp) and one Newton
    // step, which leaves it within a hair of half an ulp (the divisor lies in
    // [1e-4, 4], far from denormals and overflow); three instructions where the
    // full division takes twelve
    const float m = fmaxf(g, EPS_G);
    const float r0 = __builtin_amdgcn_rcpf(m);
    const float ig = __fmaf_rn(__fmaf_rn(-m, r0, 1.0f), r0, r0);
    return v4f{Gx * ig, Gy * ig, Gz * ig, g};
  };
  auto normals = [&](int z, auto SOL) {
    const int sl = nslot(z);
#pragma unroll
    for (int j = 0; j < 2; ++j)
      if (hon[j]) {
        const v4f v = normal(hx_[j], hy_[j], z, SOL);
        const int k = hx_[j] + HX * hy_[j];
        nrx[sl][k] = v.x;
        nry[sl][k] = v.y;
        nrz[sl][k] = v.z;
        // a tile node: its |G| kept for the curvature
        const int tlx = hx_[j] - 1, tly = hy_[j] - 1;
        if (tlx >= 0 && tlx < tx && tly >= 0 && tly < ty) nrg[sl][tlx + tx * tly] = v.w;
      }
  };
  const std::integral_constant<bool, true> with_solids;
  const std::integral_constant<bool, false> no_solids;
  auto has_solid = [&](const float* v) {
    bool r = false;
#pragma unroll
    for (int j = 0; j < 3; ++j) r |= fon[j] && v[j] > PHI_SOLID_TEST;
    return (int)r;
  };
  // prologue: phi of planes z0 - 2 .. z0 + 1, normals of planes z0 - 1, z0
  int psol = 0;
  {
    float v[3];
    for (int dz = -2; dz <= 1; ++dz) {
      load_phi(z0 + dz, v);
      store_phi(z0 + dz, v);
      psol |= has_solid(v);
    }
  }
  float nxt[3];
  load_phi(z0 + 2, nxt);
  // bit k: a solid in phi plane (z + 2 - k) of the current plane z, once the
  // loop has shifted in plane z + 2 (the prologue's planes all take the
  // block's flag over the four)
  uint32_t hist = __syncthreads_or(psol) ? 0xFu : 0u;
  if (hist) {
    normals(z0 - 1, with_solids);
    normals(z0, with_solids);
  } else {
    normals(z0 - 1, no_solids);
    normals(z0, no_solids);
  }
  __syncthreads();  // the loop's first phi store reuses the slot of plane z0 - 2
  // kept in a register: read from s after the stores below, it would be a
  // load behind them (they may alias s) and its wait would wait for them too
  const float csf = -0.5f * s.sigma;
  for (int zz = 0; zz < kz; ++zz) {
    const int z = z0 + zz;
    store_phi(z + 2, nxt);
    hist = (hist << 1) | (__syncthreads_or(has_solid(nxt)) ? 1u : 0u);
    if (zz + 1 < kz) load_phi(z + 3, nxt);
    if (hist & 7u)  // planes z .. z + 2
      normals(z + 1, with_solids);
    else
      normals(z + 1, no_solids);
    __syncthreads();
    // the curvature reads the normals of planes z - 1 .. z + 1
    const bool csol = (hist & 0xEu) != 0u;
    if (in && !csol) {
      const int c0 = (lx + 1) + HX * (ly + 1);
      const int n = gx + nx * (gy + ny * z);
      const int s0 = nslot(z);
      const v4f own = v4f{nrx[s0][c0], nry[s0][c0], nrz[s0][c0], nrg[s0][t]};
      float kappa = 0.f;
#pragma unroll
      for (int q = 0; q < 9; ++q) {
        const int i = pair_dir(q);
        const int sp_ = nslot(z + cz(i)), sm_ = nslot(z - cz(i));
        const int cp = c0 + cx(i) + HX * cy(i), cm = c0 - cx(i) - HX * cy(i);
        float dn = 0.f;
        if (cx(i) != 0) dn += (float)cx(i) * (nrx[sp_][cp] - nrx[sm_][cm]);
        if (cy(i) != 0) dn += (float)cy(i) * (nry[sp_][cp] - nry[sm_][cm]);
        if (cz(i) != 0) dn += (float)cz(i) * (nrz[sp_][cp] - nrz[sm_][cm]);
        kappa += 3.0f * wq(i) * dn;
      }
      NX[n] = own.x;
      NX[N + n] = own.y;
      NX[2 * N + n] = own.z;
      NX[3 * N + n] = own.w;
      CUR[2 * n] = csf * kappa * fmaxf(own.w, EPS_G);
      CUR[2 * n + 1] = __uint_as_float(0u);
    } else if (in) {
      const int c0 = (lx + 1) + HX * (ly + 1);
      const int n = gx + nx * (gy + ny * z);
      const int s0 = nslot(z);
      const v4f own = v4f{nrx[s0][c0], nry[s0][c0], nrz[s0][c0], nrg[s0][t]};
      float c = 0.f;
      uint32_t bits = 0x80000000u;
      if (own.w >= 0.f) {
        // pair by pair: the components c_i selects, of both neighbours (a
        // NaN marks a solid neighbour: its value is replaced by the node's own)
        float kappa = 0.f;
        bits = 0u;
#pragma unroll
        for (int q = 0; q < 9; ++q) {
          const int i = pair_dir(q), o = opp(i);
          const int sp_ = nslot(z + cz(i)), sm_ = nslot(z - cz(i));
          const int cp = c0 + cx(i) + HX * cy(i), cm = c0 - cx(i) - HX * cy(i);
          float px = cx(i) != 0 ? nrx[sp_][cp] : 0.f;
          float mx = cx(i) != 0 ? nrx[sm_][cm] : 0.f;
          float py = cy(i) != 0 ? nry[sp_][cp] : 0.f;
          float my = cy(i) != 0 ? nry[sm_][cm] : 0.f;
          float pz = cz(i) != 0 ? nrz[sp_][cp] : 0.f;
          float mz = cz(i) != 0 ? nrz[sm_][cm] : 0.f;
          const bool sp = (px != px) | (py != py) | (pz != pz);
          const bool sm = (mx != mx) | (my != my) | (mz != mz);
          if (sp) {
            px = own.x;
            py = own.y;
            pz = own.z;
          }
          if (sm) {
            mx = own.x;
            my = own.y;
            mz = own.z;
          }
          kappa += 3.0f * wq(i) * cdot(i, px - mx, py - my, pz - mz);
          bits |= (sp ? (1u << i) : 0u) | (sm ? (1u << o) : 0u);
        }
        c = csf * kappa * fmaxf(own.w, EPS_G);
      }
      NX[n] = own.x;
      NX[N + n] = own.y;
      NX[2 * N + n] = own.z;
      NX[3 * N + n] = own.w;
      CUR[2 * n] = c;
      CUR[2 * n + 1] = __uint_as_float(bits);
    }
  }
}

// ------------------------------------------------------------- fused kernel
// Per fluid node (one thread, x-fastest): populations in, the paper's collision
// on the total f (MRT + Guo forcing; the printed relaxation vector gives omega
// to every even and omega' = 8(2-omega)/(8-omega) to every odd non-conserved
// moment -- the two-relaxation-time operator computed here), the force c n +
// body force on fluid a, push streaming, and half-way bounce-back at every
// solid link.  The recolouring of f* into the two colours is not stored: the
// next moments pass rebuilds it from phi, rho and n of this state.  At
// particle links the moving-wall term and the momentum exchange are added by
// k_links.
// OPEN: the batch has simulations with open x ends (their anti-bounce-back is
// compiled into this instance only).
template <int STORE, int MODE, bool OPEN>
// six waves per SIMD: the FP16 instance fits 80 VGPRs without spills (it took
// 85 and five waves; eight waves spill and nearly double its time); the FP32
// instances need fewer anyway
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(6, 8))) void k_fused(Batch bt, float* __restrict__ out_rho,
                                              float* __restrict__ out_u,
                                              float* __restrict__ out_phi,
                                              float* __restrict__ out_F) {
  using IO = Codec<STORE>;
  using T = typename IO::T;
  const int2 sb = batch_block(bt, xcd_tile(blockIdx.x, gridDim.x));
  const SimDev& s = bt.tab[sb.x];
  const GLB T* __restrict__ sp_ = gp((const T*)s.pops[bt.cur]);
  GLB T* __restrict__ dp_ = gp((T*)s.pops[bt.cur ^ 1]);
  const GLB float* __restrict__ NX = gp((const float*)s.nrm);
  const GLB float* __restrict__ cur = gp((const float*)s.curv);
  // moments of this state (rho, phi planes) and of the one before it; FP16
  // decodes with the latter's density and encodes with the former's
  const GLB float* __restrict__ RM = gp((const float*)s.rp[bt.rd ^ 1]);
  const GLB float* __restrict__ RP = gp((const float*)s.rp[bt.rd]);
  const int nx = s.nx, ny = s.ny, nz = s.nz;
  const int N = (int)s.N;
  int n, gx, gy, gz;
  if (!tile_node(s, sb.y, n, gx, gy, gz)) return;
  const float rho0 = s.rho0;
  const float inv_rho0 = 1.0f / rho0;
  const float2 cb = make_float2(at(cur, 2u * (unsigned)n), at(cur, 2u * (unsigned)n + 1u));
  const uint32_t bits = __float_as_uint(cb.y);

  if (bits & 0x80000000u) {
    if (MODE == MODE_FIELDS) {
      const uint16_t m0 = s.mask[n];
      float ux = 0.f, uy = 0.f, uz = 0.f;
      if (m0 >= 2) {
        const DevParticle& P = s.P[m0 - 2];
        double rx = wrapd((double)gx - P.x[0], (double)nx);
        double ry = wrapd((double)gy - P.x[1], (double)ny);
        double rz = wrapd((double)gz - P.x[2], (double)nz);
        ux = (float)(P.v[0] + P.w[1] * rz - P.w[2] * ry);
        uy = (float)(P.v[1] + P.w[2] * rx - P.w[0] * rz);
        uz = (float)(P.v[2] + P.w[0] * ry - P.w[1] * rx);
      }
      out_rho[n] = 0.f;
      out_phi[n] = 0.f;
      out_u[n] = ux;
      out_u[N + n] = uy;
      out_u[2 * N + n] = uz;
      out_F[n] = 0.f;
      out_F[N + n] = 0.f;
      out_F[2 * N + n] = 0.f;
    }
    return;
  }
  const Nbr nb(gx, gy, gz, nx, ny, nz);
  float d[Q];
  const float Rn = STORE ? at(RP, (unsigned)n) : 0.f;
  const auto pb = pop_base(sp_, n);
#pragma unroll
  for (int i = 0; i < Q; ++i) d[i] = IO::ld(pb + i * POP_BLOCK, wq(i) * rho0, wq(i) * Rn);
  // FP16: the densities of this state at the node and at its 18 neighbours,
  // the references the pushed populations are encoded with.  Loaded here with
  // the populations (neighbour indices wrap, so every load is in bounds): a
  // load at the push, behind the stores before it, would wait for those too.
  float Rd[Q];
#pragma unroll
  for (int i = 0; i < Q; ++i) Rd[i] = STORE ? at(RM, (unsigned)(i == 0 ? n : nb(i))) : 0.f;
  const float3 nc =
      make_float3(at(NX, (unsigned)n), at(NX + N, (unsigned)n), at(NX + 2 * N, (unsigned)n));
  const float phi = at(RM + N, (unsigned)n);
  float drho = 0.f, jx = 0.f, jy = 0.f, jz = 0.f;
#pragma unroll
  for (int i = 0; i < Q; ++i) {
    drho += d[i];
    if (cx(i) != 0) jx += (float)cx(i) * d[i];
    if (cy(i) != 0) jy += (float)cy(i) * d[i];
    if (cz(i) != 0) jz += (float)cz(i) * d[i];
  }
  const float rho = rho0 + drho;
  // force: CSF surface tension c n + body force on fluid a (weight (1+phi)/2)
  const float fa = 0.5f * (1.0f + phi);
  const float Fx = cb.x * nc.x + s.body[0] * fa;
  const float Fy = cb.x * nc.y + s.body[1] * fa;
  const float Fz = cb.x * nc.z + s.body[2] * fa;
  const float irho = 1.0f / rho;
  const float ux = (jx + 0.5f * Fx) * irho;
  const float uy = (jy + 0.5f * Fy) * irho;
  const float uz = (jz + 0.5f * Fz) * irho;
  const float uu = ux * ux + uy * uy + uz * uz;

  if (MODE == MODE_FIELDS) {
    out_rho[n] = rho;
    out_phi[n] = phi;
    out_u[n] = ux;
    out_u[N + n] = uy;
    out_u[2 * N + n] = uz;
    out_F[n] = Fx;
    out_F[N + n] = Fy;
    out_F[2 * N + n] = Fz;
    return;
  }
  if (!(rho > 0.f) || !(uu <= 0.09f)) atomicOr(&s.counters[1], (uint32_t)ST_UNSTABLE);
  // local relaxation: harmonic mean of the kinematic viscosities
  const float inv_nu = (1.0f + phi) * s.inv2nua + (1.0f - phi) * s.inv2nub;
  const float om = 1.0f / (0.5f + 3.0f / inv_nu);
  const float om2 = 8.0f * (2.0f - om) / (8.0f - om);
  const float cfs = 1.0f - 0.5f * om, cfa = 1.0f - 0.5f * om2;
  const float uF = ux * Fx + uy * Fy + uz * Fz;

  // FP16: each population is encoded with the density of the node that
  // stores it
  auto st_pop = [&](int i, int node, float R, float dv) {
    IO::st(dp_ + pidx(i, N, node), wq(i) * rho0, inv_rho0 * (1.0f / wq(i)), wq(i) * R, dv);
  };
  // push to the neighbour in direction i, or bounce back into direction opp(i);
  // through an open x end the anti-bounce-back of the pressure boundary
  // (pressure inlet/outlet eq.): f_opp = -f*_i + 2 w_i rho_w (1 + 9/2 (c_i.u)^2
  // - 3/2 u^2), u the node's velocity, p_w = rho_w / 3
  auto emit = [&](int i, float dv) {
    if (bits & (1u << i)) {
      if (OPEN && s.open_x && ((cx(i) < 0 && gx == 0) || (cx(i) > 0 && gx == nx - 1))) {
        const float drw = cx(i) < 0 ? s.drho_in : s.drho_out;
        const float cu = cdot(i, ux, uy, uz);
        const float w = wq(i);
        // as deviations from w rho0: -d*_i + 2 w (drho_w + rho_w (9/2 cu^2 - 3/2 u^2))
        st_pop(opp(i), n, Rd[0], -dv + 2.0f * w * (drw + (rho0 + drw) * (4.5f * cu * cu - 1.5f * uu)));
      } else {
        st_pop(opp(i), n, Rd[0], dv);
      }
    } else {
      st_pop(i, nb(i), Rd[i], dv);
    }
  };

  {
    const float w0 = wq(0);
    const float deq = w0 * (drho - 1.5f * rho * uu);
    const float fb = w0 * (-3.0f * uF);
    st_pop(0, n, Rd[0], d[0] - om * (d[0] - deq) + cfs * fb);
  }
#pragma unroll
  for (int q = 0; q < 9; ++q) {
    const int i = pair_dir(q);
    const int o = opp(i);
    const float w = wq(i);
    const float cu = cdot(i, ux, uy, uz);
    const float cF = cdot(i, Fx, Fy, Fz);
    const float eqs = w * (drho + rho * (4.5f * cu * cu - 1.5f * uu));
    const float eqa = w * rho * 3.0f * cu;
    const float fs = w * (9.0f * cu * cF - 3.0f * uF);
    const float fa2 = w * 3.0f * cF;
    const float sy = 0.5f * (d[i] + d[o]) - eqs;
    const float an = 0.5f * (d[i] - d[o]) - eqa;
    const float common = -om * sy + cfs * fs;
    const float anti = -om2 * an + cfa * fa2;
    emit(i, d[i] + common + anti);
    emit(o, d[o] + common - anti);
  }
}

// Moving-wall correction and momentum exchange on particle links, after
// k_fused has bounced f*_i back into direction opp(i) at the fluid node x:
// f_opp(x) += 6 w_i rho(x) (c_opp . u_w) (its colour share phi(x) is added by
// the moments pass, as for every bounced population), with
// u_w = V + Omega x (x + c_i/2 - X) (half-way bounce-back eqs.), and the
// momentum given to the particle dP = (c_i - u_w) f*_i - (c_opp - u_w) f_opp
// (hydrodynamic force eqs.), summed in FP64 per particle.  One grid row per
// particle over the nodes of its bounding box grown by one.
template <int STORE>
__global__ __launch_bounds__(256) void k_links(Batch bt) {
  // one thread per node of the particle's box; runs after k_fused, before the
  // buffers swap: src holds the state it read, dst the state it wrote
  using IO = Codec<STORE>;
  using T = typename IO::T;
  const int2 sp = batch_particle(bt, blockIdx.y);
  const SimDev& s = bt.tab[sp.x];
  const int p = sp.y;
  GLB T* __restrict__ dp_ = gp((T*)s.pops[bt.cur ^ 1]);
  // moments of the state that collided: rho(x), and the FP16 reference of the
  // populations k_fused wrote
  const GLB float* __restrict__ RM = gp((const float*)s.rp[bt.rd ^ 1]);
  const GLB uint16_t* __restrict__ MASK = gp((const uint16_t*)s.mask);
  const DevParticle& P = s.P[p];
  const int nx = s.nx, ny = s.ny, nz = s.nz, N = (int)s.N;
  const float rho0 = s.rho0;
  int lo[3], w[3];
  const int L[3] = {nx, ny, nz};
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    lo[k] = (int)floor(P.x[k] - P.R) - 2;
    w[k] = (int)floor(P.x[k] + P.R) + 2 - lo[k] + 1;
    if (w[k] > L[k]) {
      lo[k] = 0;
      w[k] = L[k];
    }
  }
  const int vol = w[0] * w[1] * w[2];
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  double acc[6] = {0, 0, 0, 0, 0, 0};
  bool any = false;
  if (k < vol) {
    const int gx = wrapi(lo[0] + k % w[0], nx);
    const int gy = wrapi(lo[1] + (k / w[0]) % w[1], ny);
    const int gz = wrapi(lo[2] + k / (w[0] * w[1]), nz);
    // a fluid node with a link to p lies within R + sqrt(2) of its centre and
    // not inside (R - 0.5 leaves room for rounding): others load nothing
    const double dx = wrapd((double)gx - P.x[0], (double)nx);
    const double dy = wrapd((double)gy - P.x[1], (double)ny);
    const double dz = wrapd((double)gz - P.x[2], (double)nz);
    const double d2 = dx * dx + dy * dy + dz * dz;
    const double rlo = P.R - 0.5, rhi = P.R + 1.5;
    const int n = gx + nx * (gy + ny * gz);
    if (d2 < rhi * rhi && (rlo <= 0.0 || d2 >= rlo * rlo)) {
      // the node's and its neighbours' masks, its density and the 18
      // populations that bounce-back may have written, all in one round trip
      // (reading the populations only after the masks, in the link directions,
      // moves less data but adds a round trip: C2 16 -> 20 us)
      const Nbr nb(gx, gy, gz, nx, ny, nz);
      const uint16_t me = (uint16_t)(2 + p);
      const uint16_t m0 = at(MASK, (unsigned)n);
      uint32_t lm = 0;  // bit i: the neighbour in direction i is a solid node of p
#pragma unroll
      for (int i = 1; i < Q; ++i) lm |= (at(MASK, (unsigned)nb(i)) == me) ? (1u << i) : 0u;
      const float rho = at(RM, (unsigned)n);
      const float Re = STORE ? rho : 0.f;
      const auto pb = pop_base(dp_, n);
      float ds[Q];
#pragma unroll
      for (int i = 1; i < Q; ++i) {
        const int o = opp(i);
        ds[i] = IO::ld(pb + o * POP_BLOCK, wq(o) * rho0, wq(o) * Re);
      }
      if (m0 != 0) lm = 0;
      if (lm) {
        any = true;
#pragma unroll
        for (int i = 1; i < Q; ++i) {
          if (!(lm & (1u << i))) continue;
          const int o = opp(i);
          const float wr0 = wq(o) * rho0;
          const double rx = wrapd((double)gx + 0.5 * cx(i) - P.x[0], (double)nx);
          const double ry = wrapd((double)gy + 0.5 * cy(i) - P.x[1], (double)ny);
          const double rz = wrapd((double)gz + 0.5 * cz(i) - P.x[2], (double)nz);
          const double uwx = P.v[0] + (P.w[1] * rz - P.w[2] * ry);
          const double uwy = P.v[1] + (P.w[2] * rx - P.w[0] * rz);
          const double uwz = P.v[2] + (P.w[0] * ry - P.w[1] * rx);
          const float cu = (float)(-(cx(i) * uwx + cy(i) * uwy + cz(i) * uwz));  // c_opp . u_w
          const float corr = 6.0f * wq(i) * rho * cu;
          const float dso = ds[i] + corr;
          IO::st(pb + o * POP_BLOCK, wr0, 1.0f / wr0, wq(o) * Re, dso);
          const double wr = wqd(i) * (double)rho0;
          const double fin = (double)ds[i] + wr;
          const double fout = (double)dso + wr;
          const double dPx = (cx(i) - uwx) * fin - (-cx(i) - uwx) * fout;
          const double dPy = (cy(i) - uwy) * fin - (-cy(i) - uwy) * fout;
          const double dPz = (cz(i) - uwz) * fin - (-cz(i) - uwz) * fout;
          acc[0] += dPx;
          acc[1] += dPy;
          acc[2] += dPz;
          acc[3] += ry * dPz - rz * dPy;
          acc[4] += rz * dPx - rx * dPz;
          acc[5] += rx * dPy - ry * dPx;
        }
      }
    }
  }
  if (!__syncthreads_or(any)) return;  // no link in this block
  // wave reduction, then across the block's waves
#pragma unroll
  for (int c = 0; c < 6; ++c)
    for (int off = 32; off > 0; off >>= 1) acc[c] += __shfl_xor(acc[c], off, 64);
  __shared__ double red[4][6];
  const int wave = threadIdx.x >> 6;
  if ((threadIdx.x & 63) == 0)
    for (int c = 0; c < 6; ++c) red[wave][c] = acc[c];
  __syncthreads();
  if (threadIdx.x < 6) {
    const double v = red[0][threadIdx.x] + red[1][threadIdx.x] + red[2][threadIdx.x] +
                     red[3][threadIdx.x];
    if (v != 0.0) {
      DevParticle* Pw = s.P + p;
      if (threadIdx.x < 3)
        atomicAdd(&Pw->Fh[threadIdx.x], v);
      else
        atomicAdd(&Pw->Th[threadIdx.x - 3], v);
    }
  }
}

// ------------------------------------------------------------ host launchers
static inline unsigned nblocks(long long n, int b) { return (unsigned)((n + b - 1) / b); }

// Batched launchers: one launch over every simulation of the batch.
// nblk: total 256-node blocks; np_rows: total particle rows; Bmax: the largest
// mask-box side of the batch.
// nblk: per-node blocks; mnblk: blocks of the moments tiling (k_interface)
hipError_t launch_interface(const Batch& b, unsigned nblk, unsigned mnblk, hipStream_t st) {
  (void)nblk;
  const bool w64 = b.mlx == 6;  // 64-wide tiles: the instance with them fixed
  if (b.general) {
    if (w64)
      hipLaunchKernelGGL((k_interface<true, 6>), dim3(mnblk), dim3(256), 0, st, b);
    else
      hipLaunchKernelGGL((k_interface<true, 0>), dim3(mnblk), dim3(256), 0, st, b);
  } else {
    if (w64)
      hipLaunchKernelGGL((k_interface<false, 6>), dim3(mnblk), dim3(256), 0, st, b);
    else
      hipLaunchKernelGGL((k_interface<false, 0>), dim3(mnblk), dim3(256), 0, st, b);
  }
  return hipGetLastError();
}

hipError_t launch_fused(const Batch& b, int storage, unsigned nblk, int mode, float* orho,
                        float* ou, float* ophi, float* oF, hipStream_t st) {
  const dim3 grid(nblk);
  // the fields pass writes no populations: it needs no open-end instance
  if (mode != MODE_STEP) {
    if (storage == 0)
      hipLaunchKernelGGL((k_fused<0, MODE_FIELDS, false>), grid, dim3(256), 0, st, b, orho, ou,
                         ophi, oF);
    else
      hipLaunchKernelGGL((k_fused<1, MODE_FIELDS, false>), grid, dim3(256), 0, st, b, orho, ou,
                         ophi, oF);
  } else if (storage == 0) {
    if (b.open)
      hipLaunchKernelGGL((k_fused<0, MODE_STEP, true>), grid, dim3(256), 0, st, b, orho, ou, ophi, oF);
    else
      hipLaunchKernelGGL((k_fused<0, MODE_STEP, false>), grid, dim3(256), 0, st, b, orho, ou, ophi, oF);
  } else {
    if (b.open)
      hipLaunchKernelGGL((k_fused<1, MODE_STEP, true>), grid, dim3(256), 0, st, b, orho, ou, ophi, oF);
    else
      hipLaunchKernelGGL((k_fused<1, MODE_STEP, false>), grid, dim3(256), 0, st, b, orho, ou, ophi, oF);
  }
  return hipGetLastError();
}

hipError_t launch_links(const Batch& b, int storage, int np_rows, int Bmax, hipStream_t st) {
  if (np_rows == 0) return hipSuccess;
  // the box of k_links spans at most 2 R + 6 nodes per axis, R <= (Bmask - 5) / 2
  const long long B = Bmax + 1;
  const dim3 grid((unsigned)((B * B * B + 255) / 256), np_rows);
  if (storage == 0)
    hipLaunchKernelGGL(k_links<0>, grid, dim3(256), 0, st, b);
  else
    hipLaunchKernelGGL(k_links<1>, grid, dim3(256), 0, st, b);
  return hipGetLastError();
}

// mode MOM_STEP (in a step, after the refill; mnblk blocks of the moments
// tiling) or MOM_BOUNDARY (between steps; nblk per-node blocks)
enum { MOM_STEP = 0, MOM_BOUNDARY = 1 };
hipError_t launch_moments(const Batch& b, int storage, unsigned nblk, unsigned mnblk, int mode,
                          hipStream_t st) {
  if (mode == MOM_BOUNDARY)
    hipLaunchKernelGGL(k_moments_boundary, dim3(nblk), dim3(256), 0, st, b);
  else if (b.mlx == 6) {
    if (storage == 0)
      hipLaunchKernelGGL((k_moments<0, 6>), dim3(mnblk), dim3(256), 0, st, b);
    else
      hipLaunchKernelGGL((k_moments<1, 6>), dim3(mnblk), dim3(256), 0, st, b);
  } else if (storage == 0) {
    hipLaunchKernelGGL((k_moments<0, 0>), dim3(mnblk), dim3(256), 0, st, b);
  } else {
    hipLaunchKernelGGL((k_moments<1, 0>), dim3(mnblk), dim3(256), 0, st, b);
  }
  return hipGetLastError();
}

hipError_t launch_init_mask(const SimDev& s, hipStream_t st) {
  hipLaunchKernelGGL(k_init_mask, dim3(nblocks(s.N, 256)), dim3(256), 0, st, s);
  return hipGetLastError();
}

hipError_t launch_init_pops(const SimDev& s, void* pops, hipStream_t st) {
  if (s.storage == 0)
    hipLaunchKernelGGL(k_init_pops<0>, dim3(nblocks(s.N, 256)), dim3(256), 0, st, s, pops);
  else
    hipLaunchKernelGGL(k_init_pops<1>, dim3(nblocks(s.N, 256)), dim3(256), 0, st, s, pops);
  return hipGetLastError();
}

// rp: moments (rho plane, phi plane) of the current state; acc: 2 doubles,
// cleared before
hipError_t launch_mass(const SimDev& s, const float* rp, double* acc, hipStream_t st) {
  unsigned nb = nblocks(s.N, 256);
  if (nb > 4096) nb = 4096;
  hipLaunchKernelGGL(k_mass, dim3(nb), dim3(256), 0, st, s, rp, acc);
  return hipGetLastError();
}

hipError_t launch_zero_f64(double* p, int n, hipStream_t st) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_zero_f64, dim3(nblocks(n, 256)), dim3(256), 0, st, p, n);
  return hipGetLastError();
}

}  // namespace lbm
