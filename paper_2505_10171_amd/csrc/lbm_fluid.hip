// lbm_fluid.hip -- lattice kernels of liblbm for gfx950.
//
// Storage: structure-of-arrays populations, 38 planes of N values (19 planes of
// the total f, then 19 of the colour difference g = f_a - f_b), x-fastest.  FP32
// storage keeps the deviation d_i = f_i - w_i rho0 (so that the small velocity
// survives FP32 rounding); FP16 storage keeps the scaled offsets
// h_i = f_i / (w_i rho0) - 1 and k_i = g_i / (w_i rho0).  All arithmetic is FP32;
// momentum exchange sums are FP64.
//
// k_fused performs, per fluid node, the paper's collision step on the total f
// (MRT with Guo forcing; the printed relaxation vector gives omega to every even
// and omega' = 8(2-omega)/(8-omega) to every odd non-conserved moment, which is
// the two-relaxation-time operator computed here), the CSF surface-tension force
// -sigma kappa grad(phi)/2 with the geometric wetting rotation of grad(phi) next
// to solids, the recolouring of f* into the two colours, push streaming, the
// half-way bounce-back with moving walls and the momentum exchange on particle
// links.  A workgroup owns a TX x TY column tile and marches along z through LZ
// planes, keeping five planes of phi and mask (halo 2) and three planes of the
// interface normal (halo 1) in LDS, so phi and the normals are computed once per
// node and the populations are read and written exactly once.
#include "lbm_device.h"

namespace lbm {

// ------------------------------------------------------- population storage
template <int STORE>
struct PopIO;

template <>
struct PopIO<0> {
  using T = float;
  static __device__ __forceinline__ float ld(const T* p, float, float) { return *p; }
  static __device__ __forceinline__ void st(T* p, float v, float) { *p = v; }
};
template <>
struct PopIO<1> {
  using T = __half;
  // value = stored * scale ; stored = value * inv_scale
  static __device__ __forceinline__ float ld(const T* p, float scale, float) {
    return __half2float(*p) * scale;
  }
  static __device__ __forceinline__ void st(T* p, float v, float inv_scale) {
    *p = __float2half_rn(v * inv_scale);
  }
};

__device__ __forceinline__ long long node_index(const SimDev& s, int x, int y, int z) {
  return (long long)x + (long long)s.nx * ((long long)y + (long long)s.ny * z);
}

// ------------------------------------------------------------ wetting rotation
// Geometric wetting (n_pm equation): at a fluid node with a solid neighbour the
// colour gradient is rotated to make the angle theta (through fluid a) with the
// solid's outward normal n_s, keeping |G|: G <- |G| (-cos(theta) n_s + sin(theta) t^),
// t = n* - (n*.n_s) n_s.  The solid is the lowest-index neighbouring particle,
// else the wall.  Applied inside the diffuse interface (|G| > EPS_G); left
// unchanged if the tangential part |G - (G.n_s) n_s| <= EPS_GT (axis undefined).
__device__ __forceinline__ void wetting_rotate(const SimDev& s, int gx, int gy, int gz, int minp,
                                               bool wall_nb, float& Gx, float& Gy, float& Gz) {
  float g = sqrtf(Gx * Gx + Gy * Gy + Gz * Gz);
  if (!(g > EPS_G)) return;
  float nsx, nsy, nsz, nc, ns;
  if (minp >= 0) {
    const DevParticle& P = s.P[minp];
    double dx = wrapd((double)gx - P.x[0], (double)s.nx);
    double dy = wrapd((double)gy - P.x[1], (double)s.ny);
    double dz = wrapd((double)gz - P.x[2], (double)s.nz);
    double dn = sqrt(dx * dx + dy * dy + dz * dz);
    nsx = (float)(dx / dn);
    nsy = (float)(dy / dn);
    nsz = (float)(dz / dn);
    nc = P.neg_cos_t;
    ns = P.sin_t;
  } else if (wall_nb) {
    nsx = 0.f;
    nsy = 0.f;
    nsz = (gz == 1) ? 1.f : -1.f;
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
  Gx = g * (nc * nsx + ns * tx * it);
  Gy = g * (nc * nsy + ns * ty * it);
  Gz = g * (nc * nsz + ns * tz * it);
}

// One direction of each opposite pair: +x, +y, +z, (1,1,0), (1,-1,0), (1,0,1),
// (1,0,-1), (0,1,1), (0,1,-1).
__host__ __device__ constexpr int pair_dir(int k) {
  constexpr int t[9] = {1, 3, 5, 7, 8, 11, 12, 15, 16};
  return t[k];
}

// ------------------------------------------------------------- moments kernel
// Order parameter phi = sum g / rho of every fluid node (order-parameter eq.),
// after the refill of fresh nodes; clears their FRESH mark.
template <int STORE>
__global__ __launch_bounds__(256) void k_moments(SimDev s, const void* __restrict__ pops) {
  using IO = PopIO<STORE>;
  using T = typename IO::T;
  const long long N = s.N;
  long long n = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (n == 0) s.counters[0] = 0u;  // fresh list consumed
  if (n >= N) return;
  uint16_t m = s.mask[n];
  if (m & FRESH_BIT) {
    m = (uint16_t)(m & ~FRESH_BIT);
    s.mask[n] = m;
  }
  float out = 0.f;
  if (m == 0) {
    const T* b = (const T*)pops;
    // phi = sum g / sum f with f_i = d_i + w_i rho0 rounded exactly as the
    // recolouring forms it, so that a pure fluid (g_i = +-f_i) has phi = +-1
    // exactly and its colour stays segregated without FP32 leakage
    float rabs = 0.f, sg = 0.f;
#pragma unroll
    for (int i = 0; i < Q; ++i) {
      float sc = wq(i) * s.rho0;
      rabs += IO::ld(b + (long long)i * N + n, sc, 0.f) + sc;
      sg += IO::ld(b + (long long)(Q + i) * N + n, sc, 0.f);
    }
    out = sg / rabs;
  }
  s.phi[n] = out;
}

// ------------------------------------------------------------ init kernels
__global__ void k_init_mask(SimDev s) {
  long long n = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (n >= s.N) return;
  int z = (int)(n / ((long long)s.nx * s.ny));
  s.mask[n] = (s.has_wall && z == 0) ? 1 : 0;
  s.claim[n] = 0xFFFFFFFFu;
}

// fluid at rest: f = w rho0, g = w rho0 phi0 (phi0 staged in s.phi)
template <int STORE>
__global__ void k_init_pops(SimDev s, void* pops) {
  using IO = PopIO<STORE>;
  using T = typename IO::T;
  long long n = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (n >= s.N) return;
  T* b = (T*)pops;
  float p0 = (s.mask[n] == 0) ? s.phi[n] : 0.f;
#pragma unroll
  for (int i = 0; i < Q; ++i) {
    float sc = wq(i) * s.rho0;
    IO::st(b + (long long)i * s.N + n, 0.f, 1.0f / sc);
    IO::st(b + (long long)(Q + i) * s.N + n, sc * p0, 1.0f / sc);
  }
}

// --------------------------------------------------------- global mass (FP64)
template <int STORE>
__global__ __launch_bounds__(256) void k_mass(SimDev s, const void* __restrict__ pops) {
  using IO = PopIO<STORE>;
  using T = typename IO::T;
  __shared__ double sh[2][256];
  double a = 0.0, b = 0.0;
  const T* p = (const T*)pops;
  for (long long n = (long long)blockIdx.x * blockDim.x + threadIdx.x; n < s.N;
       n += (long long)gridDim.x * blockDim.x) {
    if (s.mask[n] != 0) continue;
    double drho = 0.0, sg = 0.0;
#pragma unroll
    for (int i = 0; i < Q; ++i) {
      float sc = wq(i) * s.rho0;
      drho += (double)IO::ld(p + (long long)i * s.N + n, sc, 0.f);
      sg += (double)IO::ld(p + (long long)(Q + i) * s.N + n, sc, 0.f);
    }
    double rho = (double)s.rho0 + drho;
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
    atomicAdd(&s.mass_acc[0], sh[0][0]);
    atomicAdd(&s.mass_acc[1], sh[1][0]);
  }
}

// ------------------------------------------------------------- fused kernel
enum { MODE_STEP = 0, MODE_FIELDS = 1 };

// wave64 sum of a double
__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

template <int STORE, int TX, int TY, int MODE>
__global__ __launch_bounds__(TX* TY) void k_fused(SimDev s, const void* __restrict__ src,
                                                 void* __restrict__ dst, int LZ, int ntx, int nty,
                                                 int ntz, float* __restrict__ out_rho,
                                                 float* __restrict__ out_u,
                                                 float* __restrict__ out_phi,
                                                 float* __restrict__ out_F) {
  using IO = PopIO<STORE>;
  using T = typename IO::T;
  constexpr int NT = TX * TY;
  constexpr int HX = TX + 4, HY = TY + 4;
  constexpr int NX1 = TX + 2, NY1 = TY + 2;
  __shared__ float s_phi[5][HY][HX];
  __shared__ uint16_t s_mask[5][HY][HX];
  __shared__ float4 s_n[3][NY1][NX1];

  const int nx = s.nx, ny = s.ny, nz = s.nz;
  const long long N = s.N;

  // XCD-aware tile order: consecutive dispatches go round-robin over the 8
  // XCDs; give each XCD a contiguous range of tiles so that halo planes shared
  // by neighbouring tiles meet in the same L2.
  const int nblk = ntx * nty * ntz;
  int lin = blockIdx.x;
  int tile = lin;
  if ((nblk & 7) == 0) {
    const int per = nblk >> 3;
    tile = (lin & 7) * per + (lin >> 3);
  }
  const int bx = tile % ntx;
  const int rr = tile / ntx;
  const int by = rr % nty;
  const int bz = rr / nty;
  const int x0 = bx * TX, y0 = by * TY, z0 = bz * LZ;
  const int z1 = min(z0 + LZ, nz);
  const int tid = threadIdx.x;
  const int tx = tid % TX, ty = tid / TX;
  const int gx = x0 + tx, gy = y0 + ty;
  const bool active = (gx < nx) && (gy < ny);

  auto slot5 = [](int zrel) { return (zrel + 10) % 5; };
  auto slot3 = [](int zrel) { return (zrel + 9) % 3; };

  auto load_plane = [&](int zrel) {
    const int gz = wrapi(z0 + zrel, nz);
    const int sl = slot5(zrel);
    for (int k = tid; k < HX * HY; k += NT) {
      const int lx = k % HX, ly = k / HX;
      const int xg = wrapi(x0 - 2 + lx, nx), yg = wrapi(y0 - 2 + ly, ny);
      const long long n = node_index(s, xg, yg, gz);
      const uint16_t m = s.mask[n];
      s_mask[sl][ly][lx] = m;
      s_phi[sl][ly][lx] = (m == 0) ? s.phi[n] : 0.f;
    }
  };

  // colour gradient (isotropic stencil with the zero-gradient closure at solid
  // neighbours), wetting rotation, unit normal; for the halo-1 region of a plane
  auto normals_plane = [&](int zrel) {
    const int gz = wrapi(z0 + zrel, nz);
    const int sc = slot5(zrel), sm = slot5(zrel - 1), sp = slot5(zrel + 1);
    const int so = slot3(zrel);
    for (int k = tid; k < NX1 * NY1; k += NT) {
      const int hx = k % NX1, hy = k / NX1;
      const int lx = hx + 1, ly = hy + 1;
      float4 out = make_float4(0.f, 0.f, 0.f, 0.f);
      if (s_mask[sc][ly][lx] == 0) {
        const float p0 = s_phi[sc][ly][lx];
        float Gx = 0.f, Gy = 0.f, Gz = 0.f;
        int minp = 0x7fffffff;
        bool solid = false, wall = false;
#pragma unroll
        for (int q = 0; q < 9; ++q) {
          const int i = pair_dir(q);
          const int slp = cz(i) > 0 ? sp : (cz(i) < 0 ? sm : sc);
          const int slm = cz(i) > 0 ? sm : (cz(i) < 0 ? sp : sc);
          const uint16_t mp = s_mask[slp][ly + cy(i)][lx + cx(i)];
          const uint16_t mm = s_mask[slm][ly - cy(i)][lx - cx(i)];
          const float vp = (mp == 0) ? s_phi[slp][ly + cy(i)][lx + cx(i)] : p0;
          const float vm = (mm == 0) ? s_phi[slm][ly - cy(i)][lx - cx(i)] : p0;
          const float d = 3.0f * wq(i) * (vp - vm);
          Gx += (float)cx(i) * d;
          Gy += (float)cy(i) * d;
          Gz += (float)cz(i) * d;
          if (mp) {
            solid = true;
            if (mp >= 2) minp = min(minp, (int)mp - 2); else wall = true;
          }
          if (mm) {
            solid = true;
            if (mm >= 2) minp = min(minp, (int)mm - 2); else wall = true;
          }
        }
        if (solid) {
          const int hgx = wrapi(x0 - 1 + hx, nx), hgy = wrapi(y0 - 1 + hy, ny);
          wetting_rotate(s, hgx, hgy, gz, minp == 0x7fffffff ? -1 : minp, wall, Gx, Gy, Gz);
        }
        const float g = sqrtf(Gx * Gx + Gy * Gy + Gz * Gz);
        const float ig = 1.0f / fmaxf(g, EPS_G);
        out = make_float4(Gx * ig, Gy * ig, Gz * ig, g);
      }
      s_n[so][hy][hx] = out;
    }
  };

  // prologue
  for (int zr = -2; zr <= 1; ++zr) load_plane(zr);
  __syncthreads();
  normals_plane(-1);
  normals_plane(0);

  const T* __restrict__ sp_ = (const T*)src;
  T* __restrict__ dp_ = (T*)dst;
  const float rho0 = s.rho0;

  for (int z = z0; z < z1; ++z) {
    const int zrel = z - z0;
    load_plane(zrel + 2);
    __syncthreads();
    normals_plane(zrel + 1);
    __syncthreads();

    // ------------------------------------------------------- node update
    double accF0 = 0.0, accF1 = 0.0, accF2 = 0.0, accT0 = 0.0, accT1 = 0.0, accT2 = 0.0;
    int key = -1;
    const int lx = tx + 2, ly = ty + 2;
    const int sc = slot5(zrel), sm = slot5(zrel - 1), spl = slot5(zrel + 1);
    const uint16_t m0 = active ? s_mask[sc][ly][lx] : (uint16_t)1;
    const long long n = active ? node_index(s, gx, gy, z) : 0;

    if (active && m0 != 0) {
      if (MODE == MODE_FIELDS) {
        float ux = 0.f, uy = 0.f, uz = 0.f;
        if (m0 >= 2) {
          const DevParticle& P = s.P[m0 - 2];
          double rx = wrapd((double)gx - P.x[0], (double)nx);
          double ry = wrapd((double)gy - P.x[1], (double)ny);
          double rz = wrapd((double)z - P.x[2], (double)nz);
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
    } else if (active) {
      // own populations
      float d[Q], g[Q];
#pragma unroll
      for (int i = 0; i < Q; ++i) {
        const float sc_ = wq(i) * rho0;
        d[i] = IO::ld(sp_ + (long long)i * N + n, sc_, 0.f);
        g[i] = IO::ld(sp_ + (long long)(Q + i) * N + n, sc_, 0.f);
      }
      float drho = 0.f, jx = 0.f, jy = 0.f, jz = 0.f;
#pragma unroll
      for (int i = 0; i < Q; ++i) {
        drho += d[i];
        jx += (float)cx(i) * d[i];
        jy += (float)cy(i) * d[i];
        jz += (float)cz(i) * d[i];
      }
      const float rho = rho0 + drho;
      const float phi = s_phi[sc][ly][lx];

      // curvature kappa = div n (same stencil and closure as the gradient)
      const int nsl = slot3(zrel), nsm = slot3(zrel - 1), nsp = slot3(zrel + 1);
      const float4 nc = s_n[nsl][ty + 1][tx + 1];
      float kappa = 0.f;
#pragma unroll
      for (int q = 0; q < 9; ++q) {
        const int i = pair_dir(q);
        const int slp = cz(i) > 0 ? spl : (cz(i) < 0 ? sm : sc);
        const int slm = cz(i) > 0 ? sm : (cz(i) < 0 ? spl : sc);
        const int nlp = cz(i) > 0 ? nsp : (cz(i) < 0 ? nsm : nsl);
        const int nlm = cz(i) > 0 ? nsm : (cz(i) < 0 ? nsp : nsl);
        const float4 np_ = (s_mask[slp][ly + cy(i)][lx + cx(i)] == 0)
                               ? s_n[nlp][ty + 1 + cy(i)][tx + 1 + cx(i)] : nc;
        const float4 nm_ = (s_mask[slm][ly - cy(i)][lx - cx(i)] == 0)
                               ? s_n[nlm][ty + 1 - cy(i)][tx + 1 - cx(i)] : nc;
        kappa += 3.0f * wq(i) *
                 ((float)cx(i) * (np_.x - nm_.x) + (float)cy(i) * (np_.y - nm_.y) +
                  (float)cz(i) * (np_.z - nm_.z));
      }
      // force: CSF surface tension -sigma kappa G / 2 + body force on fluid a
      // (weight (1+phi)/2); G = n max(|G|, EPS_G)
      const float cst = -0.5f * s.sigma * kappa * fmaxf(nc.w, EPS_G);
      const float fa = 0.5f * (1.0f + phi);
      const float Fx = cst * nc.x + s.body[0] * fa;
      const float Fy = cst * nc.y + s.body[1] * fa;
      const float Fz = cst * nc.z + s.body[2] * fa;
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
      } else {
        if (!(rho > 0.f) || !(uu <= 0.09f)) atomicOr(&s.counters[1], (uint32_t)ST_UNSTABLE);
        // local relaxation: harmonic mean of the kinematic viscosities
        const float inv_nu = (1.0f + phi) * s.inv2nua + (1.0f - phi) * s.inv2nub;
        const float om = 1.0f / (0.5f + 3.0f / inv_nu);
        const float om2 = 8.0f * (2.0f - om) / (8.0f - om);
        const float cfs = 1.0f - 0.5f * om, cfa = 1.0f - 0.5f * om2;
        const float uF = ux * Fx + uy * Fy + uz * Fz;
        const float rec = 0.5f * s.beta * rho * (1.0f - phi) * (1.0f + phi);

        // rest population
        {
          const float w0 = wq(0);
          const float deq = w0 * (drho - 1.5f * rho * uu);
          const float fb = w0 * (-3.0f * uF);
          const float ds = d[0] - om * (d[0] - deq) + cfs * fb;
          const float gs = phi * (ds + w0 * rho0);
          const float sc_ = w0 * rho0;
          IO::st(dp_ + n, ds, 1.0f / sc_);
          IO::st(dp_ + (long long)Q * N + n, gs, 1.0f / sc_);
        }

        auto emit = [&](int i, float ds, float gs, float rci) {
          const int xx = wrapi(gx + cx(i), nx), yy = wrapi(gy + cy(i), ny),
                    zz = wrapi(z + cz(i), nz);
          const int sl = cz(i) > 0 ? spl : (cz(i) < 0 ? sm : sc);
          const uint16_t mt = s_mask[sl][ly + cy(i)][lx + cx(i)];
          const float sc_ = wq(i) * rho0;
          if (mt == 0) {
            const long long m = node_index(s, xx, yy, zz);
            IO::st(dp_ + (long long)i * N + m, ds, 1.0f / sc_);
            IO::st(dp_ + (long long)(Q + i) * N + m, gs, 1.0f / sc_);
          } else {
            const int o = opp(i);
            if (mt == 1) {
              IO::st(dp_ + (long long)o * N + n, ds, 1.0f / sc_);
              IO::st(dp_ + (long long)(Q + o) * N + n, gs, 1.0f / sc_);
            } else {
              const int p = mt - 2;
              const DevParticle& P = s.P[p];
              // wall velocity at the link midpoint
              const double rx = wrapd((double)gx + 0.5 * cx(i) - P.x[0], (double)nx);
              const double ry = wrapd((double)gy + 0.5 * cy(i) - P.x[1], (double)ny);
              const double rz = wrapd((double)z + 0.5 * cz(i) - P.x[2], (double)nz);
              const double uwx = P.v[0] + (P.w[1] * rz - P.w[2] * ry);
              const double uwy = P.v[1] + (P.w[2] * rx - P.w[0] * rz);
              const double uwz = P.v[2] + (P.w[0] * ry - P.w[1] * rx);
              // c_opp . u_w
              const float cu = (float)(-(cx(i) * uwx + cy(i) * uwy + cz(i) * uwz));
              // f_opp = f*_i + 6 w rho (c_opp.u_w); g_opp = phi f_opp + recolour
              // term (the same as g*_i + 6 w rho phi (c_opp.u_w))
              const float dso = ds + 6.0f * wq(i) * rho * cu;
              const float gso = phi * (dso + wq(i) * rho0) + rci;
              IO::st(dp_ + (long long)o * N + n, dso, 1.0f / sc_);
              IO::st(dp_ + (long long)(Q + o) * N + n, gso, 1.0f / sc_);
              // momentum exchange (Galilean invariant): momentum given to p
              const double wr = wqd(i) * (double)rho0;
              const double fin = (double)ds + wr;
              const double fout = (double)dso + wr;
              const double dPx = (cx(i) - uwx) * fin - (-cx(i) - uwx) * fout;
              const double dPy = (cy(i) - uwy) * fin - (-cy(i) - uwy) * fout;
              const double dPz = (cz(i) - uwz) * fin - (-cz(i) - uwz) * fout;
              const double tX = ry * dPz - rz * dPy;
              const double tY = rz * dPx - rx * dPz;
              const double tZ = rx * dPy - ry * dPx;
              if (key < 0) key = p;
              if (p == key) {
                accF0 += dPx; accF1 += dPy; accF2 += dPz;
                accT0 += tX; accT1 += tY; accT2 += tZ;
              } else {
                DevParticle* Pw = s.P + p;
                atomicAdd(&Pw->Fh[0], dPx); atomicAdd(&Pw->Fh[1], dPy);
                atomicAdd(&Pw->Fh[2], dPz); atomicAdd(&Pw->Th[0], tX);
                atomicAdd(&Pw->Th[1], tY); atomicAdd(&Pw->Th[2], tZ);
              }
            }
          }
        };

#pragma unroll
        for (int q = 0; q < 9; ++q) {
          const int i = pair_dir(q);
          const int o = opp(i);
          const float w = wq(i);
          const float cu = (float)cx(i) * ux + (float)cy(i) * uy + (float)cz(i) * uz;
          const float cF = (float)cx(i) * Fx + (float)cy(i) * Fy + (float)cz(i) * Fz;
          const float eqs = w * (drho + rho * (4.5f * cu * cu - 1.5f * uu));
          const float eqa = w * rho * 3.0f * cu;
          const float fs = w * (9.0f * cu * cF - 3.0f * uF);
          const float fa2 = w * 3.0f * cF;
          const float sy = 0.5f * (d[i] + d[o]) - eqs;
          const float an = 0.5f * (d[i] - d[o]) - eqa;
          const float common = -om * sy + cfs * fs;
          const float anti = -om2 * an + cfa * fa2;
          const float ds_i = d[i] + common + anti;
          const float ds_o = d[o] + common - anti;
          const float cn = (float)cx(i) * nc.x + (float)cy(i) * nc.y + (float)cz(i) * nc.z;
          const float rc = rec * w * cn;
          const float wr0 = w * rho0;
          const float gs_i = phi * (ds_i + wr0) + rc;
          const float gs_o = phi * (ds_o + wr0) - rc;
          emit(i, ds_i, gs_i, rc);
          emit(o, ds_o, gs_o, -rc);
        }
        (void)g;
      }
    }

    if (MODE == MODE_STEP && s.np > 0) {
      // segmented wave64 reduction of the per-particle momentum exchange
      while (true) {
        const unsigned long long act = __ballot(key >= 0);
        if (act == 0ull) break;
        const int leader = __ffsll((long long)act) - 1;
        const int lk = __shfl(key, leader, 64);
        const bool mine = (key == lk);
        const double v0 = wave_sum(mine ? accF0 : 0.0);
        const double v1 = wave_sum(mine ? accF1 : 0.0);
        const double v2 = wave_sum(mine ? accF2 : 0.0);
        const double v3 = wave_sum(mine ? accT0 : 0.0);
        const double v4 = wave_sum(mine ? accT1 : 0.0);
        const double v5 = wave_sum(mine ? accT2 : 0.0);
        if ((int)(threadIdx.x & 63) == leader) {
          DevParticle* Pw = s.P + lk;
          atomicAdd(&Pw->Fh[0], v0); atomicAdd(&Pw->Fh[1], v1); atomicAdd(&Pw->Fh[2], v2);
          atomicAdd(&Pw->Th[0], v3); atomicAdd(&Pw->Th[1], v4); atomicAdd(&Pw->Th[2], v5);
        }
        if (mine) key = -1;
      }
    }
  }
}

// ------------------------------------------------------------ host launchers
static inline unsigned nblocks(long long n, int b) { return (unsigned)((n + b - 1) / b); }

template <int STORE>
static hipError_t launch_fused_t(const SimDev& s, const void* src, void* dst, int mode, int LZ,
                                 float* orho, float* ou, float* ophi, float* oF, hipStream_t st) {
  if (s.nx >= 64) {
    constexpr int TX = 64, TY = 4;
    int ntx = (s.nx + TX - 1) / TX, nty = (s.ny + TY - 1) / TY, ntz = (s.nz + LZ - 1) / LZ;
    dim3 grid(ntx * nty * ntz);
    if (mode == MODE_STEP)
      hipLaunchKernelGGL((k_fused<STORE, TX, TY, MODE_STEP>), grid, dim3(TX * TY), 0, st, s, src,
                         dst, LZ, ntx, nty, ntz, orho, ou, ophi, oF);
    else
      hipLaunchKernelGGL((k_fused<STORE, TX, TY, MODE_FIELDS>), grid, dim3(TX * TY), 0, st, s,
                         src, dst, LZ, ntx, nty, ntz, orho, ou, ophi, oF);
  } else {
    constexpr int TX = 32, TY = 8;
    int ntx = (s.nx + TX - 1) / TX, nty = (s.ny + TY - 1) / TY, ntz = (s.nz + LZ - 1) / LZ;
    dim3 grid(ntx * nty * ntz);
    if (mode == MODE_STEP)
      hipLaunchKernelGGL((k_fused<STORE, TX, TY, MODE_STEP>), grid, dim3(TX * TY), 0, st, s, src,
                         dst, LZ, ntx, nty, ntz, orho, ou, ophi, oF);
    else
      hipLaunchKernelGGL((k_fused<STORE, TX, TY, MODE_FIELDS>), grid, dim3(TX * TY), 0, st, s,
                         src, dst, LZ, ntx, nty, ntz, orho, ou, ophi, oF);
  }
  return hipGetLastError();
}

hipError_t launch_fused(const SimDev& s, const void* src, void* dst, int mode, int LZ, float* orho,
                        float* ou, float* ophi, float* oF, hipStream_t st) {
  return s.storage == 0 ? launch_fused_t<0>(s, src, dst, mode, LZ, orho, ou, ophi, oF, st)
                        : launch_fused_t<1>(s, src, dst, mode, LZ, orho, ou, ophi, oF, st);
}

hipError_t launch_moments(const SimDev& s, const void* pops, hipStream_t st) {
  if (s.storage == 0)
    hipLaunchKernelGGL(k_moments<0>, dim3(nblocks(s.N, 256)), dim3(256), 0, st, s, pops);
  else
    hipLaunchKernelGGL(k_moments<1>, dim3(nblocks(s.N, 256)), dim3(256), 0, st, s, pops);
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

hipError_t launch_mass(const SimDev& s, const void* pops, hipStream_t st) {
  unsigned nb = nblocks(s.N, 256);
  if (nb > 4096) nb = 4096;
  if (s.storage == 0)
    hipLaunchKernelGGL(k_mass<0>, dim3(nb), dim3(256), 0, st, s, pops);
  else
    hipLaunchKernelGGL(k_mass<1>, dim3(nb), dim3(256), 0, st, s, pops);
  return hipGetLastError();
}

}  // namespace lbm
