// lbm_particles.hip -- particle kernels of liblbm for gfx950: solid mask update,
// refilling of fresh fluid nodes, capillary force on the Lagrangian surface grid
// and the DEM (contacts with sliding and rolling friction, velocity Verlet).
#include <algorithm>

#include "lbm_device.h"

namespace lbm {

// ------------------------------------------------------------------ masks
// Particle bounding box: every node inside the sphere lies in it.
struct Box {
  int lo[3], w[3];
};
__device__ __forceinline__ Box particle_box(const SimDev& s, const double* X, double R) {
  Box b;
  const int L[3] = {s.nx, s.ny, s.nz};
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    b.lo[k] = (int)floor(X[k] - R) - 1;
    b.w[k] = (int)floor(X[k] + R) + 1 - b.lo[k] + 1;
    if (b.w[k] > L[k]) {
      b.lo[k] = 0;
      b.w[k] = L[k];
    }
  }
  return b;
}

// Inside test: ((dx*dx)+(dy*dy))+(dz*dz) < R*R in FP64, rounded operation by
// operation (no contraction), d wrapped once into (-L/2, L/2].
__device__ __attribute__((noinline)) bool inside_sphere(int x, int y, int z, const double* X,
                                                        double R, int nx, int ny, int nz) {
#pragma clang fp contract(off)
  double dx = wrapd((double)x - X[0], (double)nx);
  double dy = wrapd((double)y - X[1], (double)ny);
  double dz = wrapd((double)z - X[2], (double)nz);
  double a = dx * dx;
  double b = dy * dy;
  double c = dz * dz;
  double d2 = (a + b) + c;
  return d2 < R * R;
}

// claim: lowest particle index inside which a node lies (new positions)
__global__ void k_claim(Batch bt) {
  const int2 sp = batch_particle(bt, blockIdx.y);
  const SimDev& s = bt.tab[sp.x];
  const int p = sp.y;
  const DevParticle& P = s.P[p];
  const Box b = particle_box(s, P.x, P.R);
  const int vol = b.w[0] * b.w[1] * b.w[2];
  for (int k = blockIdx.x * blockDim.x + threadIdx.x; k < vol; k += gridDim.x * blockDim.x) {
    const int ix = k % b.w[0], iy = (k / b.w[0]) % b.w[1], iz = k / (b.w[0] * b.w[1]);
    const int x = wrapi(b.lo[0] + ix, s.nx), y = wrapi(b.lo[1] + iy, s.ny),
              z = wrapi(b.lo[2] + iz, s.nz);
    if (static_wall(s, x, y, z)) continue;
    if (inside_sphere(x, y, z, P.x, P.R, s.nx, s.ny, s.nz)) {
      const long long n = (long long)x + (long long)s.nx * ((long long)y + (long long)s.ny * z);
      atomicMin(&s.claim[n], (uint32_t)p);
    }
  }
}

// release: nodes that belonged to p (old box) become fluid (fresh) or pass to
// the particle that claims them now.  Each such node is visited once (by p).
__global__ void k_release(Batch bt) {
  const int2 sp = batch_particle(bt, blockIdx.y);
  const SimDev& s = bt.tab[sp.x];
  const int p = sp.y;
  const DevParticle& P = s.P[p];
  double Xo[3] = {P.xo[0], P.xo[1], P.xo[2]};
  const Box b = particle_box(s, Xo, P.Ro);
  const int vol = b.w[0] * b.w[1] * b.w[2];
  // the record's fields held in registers (the stores below may alias it)
  const int nx = s.nx, ny = s.ny, nz = s.nz;
  GLB uint16_t* __restrict__ MASK = gp(s.mask);
  const GLB uint32_t* __restrict__ CLAIM = gp((const uint32_t*)s.claim);
  for (int k = blockIdx.x * blockDim.x + threadIdx.x; k < vol; k += gridDim.x * blockDim.x) {
    const int ix = k % b.w[0], iy = (k / b.w[0]) % b.w[1], iz = k / (b.w[0] * b.w[1]);
    const int x = wrapi(b.lo[0] + ix, nx), y = wrapi(b.lo[1] + iy, ny), z = wrapi(b.lo[2] + iz, nz);
    const unsigned n = (unsigned)(x + nx * (y + ny * z));
    // mask and claim in one round trip
    const uint16_t m = at((const GLB uint16_t*)MASK, n);
    const uint32_t c = at(CLAIM, n);
    const bool mine = m == (uint16_t)(2 + p);
    const bool fresh = mine && c == 0xFFFFFFFFu;
    // the wave's fresh nodes take consecutive slots of the fresh list: one
    // atomic per wave (the list's order does not matter to the refill)
    const unsigned long long want = __ballot(fresh);
    uint32_t base0 = 0;
    const int lane = (int)(threadIdx.x & 63);
    const int first = want ? __ffsll((long long)want) - 1 : 0;
    if (want && lane == first) base0 = atomicAdd(&s.counters[0], (uint32_t)__popcll(want));
    base0 = (uint32_t)__shfl((int)base0, first, 64);
    if (!mine) continue;
    if (fresh) {
      MASK[n] = FRESH_BIT;
      const uint32_t slot = base0 + (uint32_t)__popcll(want & ((1ull << lane) - 1ull));
      if (slot < s.fresh_cap) {
        s.fresh[slot] = n;
        s.fresh_own[slot] = (uint32_t)p;
      } else {
        atomicOr(&s.counters[1], (uint32_t)ST_FRESH_FULL);
      }
    } else if (c != (uint32_t)p) {
      MASK[n] = (uint16_t)(2 + c);
    }
  }
}

// cover: nodes claimed by p become p's solid nodes; claims are cleared
__global__ void k_cover(Batch bt) {
  const int2 sp = batch_particle(bt, blockIdx.y);
  const SimDev& s = bt.tab[sp.x];
  const int p = sp.y;
  const DevParticle& P = s.P[p];
  const Box b = particle_box(s, P.x, P.R);
  const int vol = b.w[0] * b.w[1] * b.w[2];
  // the record's fields held in registers (the stores below may alias it)
  const int nx = s.nx, ny = s.ny, nz = s.nz;
  GLB uint16_t* __restrict__ MASK = gp(s.mask);
  GLB uint32_t* __restrict__ CLAIM = gp(s.claim);
  for (int k = blockIdx.x * blockDim.x + threadIdx.x; k < vol; k += gridDim.x * blockDim.x) {
    const int ix = k % b.w[0], iy = (k / b.w[0]) % b.w[1], iz = k / (b.w[0] * b.w[1]);
    const int x = wrapi(b.lo[0] + ix, nx), y = wrapi(b.lo[1] + iy, ny), z = wrapi(b.lo[2] + iz, nz);
    const unsigned n = (unsigned)(x + nx * (y + ny * z));
    if (at((const GLB uint32_t*)CLAIM, n) == (uint32_t)p) {
      MASK[n] = (uint16_t)(2 + p);
      CLAIM[n] = 0xFFFFFFFFu;
    }
  }
}

// Refilling (refilling eqs.): f_a, f_b of a fresh node = equilibria of the mean
// neighbour densities (fluid, not fresh, D3Q19 neighbours; rho0/2 each if none)
// at the surface velocity of the particle that uncovered it.  Stored are the
// total f and the node's moments (rho, phi) in rp[rd ^ 1].  The neighbour
// densities are those of the post-stream state: in a step (REFILL_STEP) rebuilt
// from the state that collided, as the moments pass does; between steps
// (REFILL_BOUNDARY) the current moments rp[rd ^ 1].
enum { REFILL_STEP = 0, REFILL_BOUNDARY = 1 };
template <int STORE, int MODE>
__global__ __launch_bounds__(256) void k_refill(Batch bt) {
  // one thread per (fresh node, neighbour direction): 14 fresh nodes per
  // block; grid row = simulation
  using IO = Codec<STORE>;
  using T = typename IO::T;
  const SimDev& s = bt.tab[blockIdx.y];
  if (s.np == 0) return;
  T* b = (T*)s.pops[bt.cur];
  const GLB float* RO = gp((const float*)s.rp[bt.rd]);
  float* RN = s.rp[bt.rd ^ 1];
  constexpr int PER = 14;
  __shared__ float sh_a[PER][18], sh_b[PER][18];
  __shared__ int sh_c[PER][18];
  const uint32_t cnt = min(s.counters[0], s.fresh_cap);
  const int N = (int)s.N;
  const int slot = threadIdx.x / 18, dir = threadIdx.x % 18 + 1;
  for (uint32_t base = blockIdx.x * PER; base < cnt; base += gridDim.x * PER) {
    const uint32_t k = base + slot;
    if (slot < PER) {
      float ra = 0.f, rb = 0.f;
      int c = 0;
      if (k < cnt) {
        const int n = (int)s.fresh[k];
        const int x = n % s.nx, y = (n / s.nx) % s.ny, z = n / (s.nx * s.ny);
        const int mx = wrapi(x + cx(dir), s.nx), my = wrapi(y + cy(dir), s.ny),
                  mz = wrapi(z + cz(dir), s.nz);
        const int m = mx + s.nx * (my + s.ny * mz);
        if (s.mask[m] == 0) {
          float rho, sg;
          if (MODE == REFILL_STEP) {
            const Nbr nbm(mx, my, mz, s.nx, s.ny, s.nz);
            rebuild_moments<STORE>(gp((const T*)b), RO, gp((const float*)s.nrm), N, m, nbm,
                                   s.rho0, 0.5f * s.beta, STORE ? RO[m] : 0.f, rho, sg);
          } else {
            rho = RN[m];
            sg = rho * RN[N + m];
          }
          ra = 0.5f * (rho + sg);
          rb = 0.5f * (rho - sg);
          c = 1;
        }
      }
      sh_a[slot][dir - 1] = ra;
      sh_b[slot][dir - 1] = rb;
      sh_c[slot][dir - 1] = c;
    }
    __syncthreads();
    if ((int)threadIdx.x < PER && base + threadIdx.x < cnt) {
      const uint32_t kk = base + threadIdx.x;
      float sa = 0.f, sb = 0.f;
      int c = 0;
      for (int i = 0; i < 18; ++i) {
        sa += sh_a[threadIdx.x][i];
        sb += sh_b[threadIdx.x][i];
        c += sh_c[threadIdx.x][i];
      }
      const int n = (int)s.fresh[kk];
      const int p = (int)s.fresh_own[kk];
      const int x = n % s.nx, y = (n / s.nx) % s.ny, z = n / (s.nx * s.ny);
      const float ra = c ? sa / c : 0.5f * s.rho0;
      const float rb = c ? sb / c : 0.5f * s.rho0;
      const DevParticle& P = s.P[p];
      const double rx = wrapd((double)x - P.x[0], (double)s.nx);
      const double ry = wrapd((double)y - P.x[1], (double)s.ny);
      const double rz = wrapd((double)z - P.x[2], (double)s.nz);
      const float ux = (float)(P.v[0] + P.w[1] * rz - P.w[2] * ry);
      const float uy = (float)(P.v[1] + P.w[2] * rx - P.w[0] * rz);
      const float uz = (float)(P.v[2] + P.w[0] * ry - P.w[1] * rx);
      const float uu = ux * ux + uy * uy + uz * uz;
      const float rho = ra + rb;
      // FP16: encoded with the reference the decoders of this state use
      const float Rn = STORE ? RO[n] : 0.f;
      for (int q = 0; q < Q; ++q) {
        const float cu = cx(q) * ux + cy(q) * uy + cz(q) * uz;
        const float poly = 3.0f * cu + 4.5f * cu * cu - 1.5f * uu;
        const float dq = wq(q) * ((rho - s.rho0) + rho * poly);
        IO::st(b + pidx(q, N, n), wq(q) * s.rho0, 1.0f / (wq(q) * s.rho0), wq(q) * Rn, dq);
      }
      // f^a - f^b = (ra - rb) / rho f: the order parameter of the node
      RN[n] = rho;
      RN[N + n] = (ra - rb) / rho;
    }
    __syncthreads();
  }
}

// -------------------------------------------------------------- capillary
// per-particle box of (phi, G) at the nodes the Lagrangian points interpolate
// (G after the wetting rotation, from the step's normal field)
__global__ void k_capbox(Batch bt) {
  const int2 sp = batch_particle(bt, blockIdx.y);
  const SimDev& s = bt.tab[sp.x];
  const int p = sp.y;
  DevParticle& P = s.P[p];
  const int B = s.cap_B;
  int org[3];
#pragma unroll
  for (int k = 0; k < 3; ++k) org[k] = (int)floor(P.x[k] - P.R);
  if (blockIdx.x == 0 && threadIdx.x < 3) s.capbox_org[3 * p + threadIdx.x] = org[threadIdx.x];
  if (s.cap_pref == 0.0) return;  // no surface tension: no capillary force
  float4* box = s.capbox + (long long)p * B * B * B;
  // phi of the state that collided this step (the buffers have swapped); the
  // record's fields held in registers (the box stores may alias the record)
  const int nx = s.nx, ny = s.ny, nz = s.nz, N = (int)s.N;
  const GLB float* __restrict__ PHI = gp((const float*)s.rp[bt.rd]) + N;
  const GLB float* __restrict__ NRM = gp((const float*)s.nrm);
  // a particle whose box holds no fluid node with |G| near EPS_G or above gets
  // no force: every point's G is a convex combination of corner values, so it
  // would fail the |G| > EPS_G test of the force kernel (the 0.99 margin covers
  // rounding); the box's nodes say so here, once, for that kernel
  bool iface = false;
  for (int k = blockIdx.x * blockDim.x + threadIdx.x; k < B * B * B; k += gridDim.x * blockDim.x) {
    const int ix = k % B, iy = (k / B) % B, iz = k / (B * B);
    const int x = wrapi(org[0] + ix, nx), y = wrapi(org[1] + iy, ny), z = wrapi(org[2] + iz, nz);
    const unsigned n = (unsigned)(x + nx * (y + ny * z));
    // every plane read at once and the solid case taken by selects (a load
    // used only inside a branch is made there, a second round trip)
    const float gw = at(NRM + 3 * N, n), ph = at(PHI, n);
    const float n0 = at(NRM, n), n1 = at(NRM + N, n), n2 = at(NRM + 2 * N, n);
    // G = n max(|G|, EPS_G): the colour gradient after the wetting rotation;
    // phi = 2 marks a solid node
    const bool fl = gw >= 0.f;
    const float gm = fmaxf(gw, EPS_G);
    const float4 v = make_float4(fl ? ph : 2.f, fl ? n0 * gm : 0.f, fl ? n1 * gm : 0.f,
                                 fl ? n2 * gm : 0.f);
    box[k] = v;
    iface |= v.x <= 1.5f && v.y * v.y + v.z * v.z + v.w * v.w > (0.99f * EPS_G) * (0.99f * EPS_G);
  }
  if (__syncthreads_or(iface) && threadIdx.x == 0) P.cap_on = 1;
}

// Capillary force (capillary-force eq.): sum over the polar/azimuthal grid of
// sigma 9/2 k beta max(0, 1 - phi^2) dA sin(theta_p) m^, m^ = normalise(n_s - (n.n_s) n),
// torque arm R n_s; phi and G trilinear over fluid corners.  A grid row of
// workgroups per particle, FP64 block reductions combined with FP64 atomics
// (the accumulators are consumed and cleared by the DEM).
__global__ __launch_bounds__(256) void k_capillary(Batch bt) {
  const int2 sp = batch_particle(bt, blockIdx.y);
  const SimDev& s = bt.tab[sp.x];
  const int p = sp.y;
  DevParticle& P = s.P[p];
  if (s.cap_pref == 0.0) return;  // no surface tension: no capillary force
  const int B = s.cap_B;
  const GLB v4f* box = gp((const v4f*)s.capbox) + (long long)p * B * B * B;
  const int org0 = (int)floor(P.x[0] - P.R), org1 = (int)floor(P.x[1] - P.R),
            org2 = (int)floor(P.x[2] - P.R);
  const double R = P.R, da = s.cap_dang;
  const double pref = s.cap_pref * (double)P.sin_t;
  const int na = s.cap_na, nph = s.cap_nphi;
  // the polar and azimuthal grids are fixed: their sines and cosines once per
  // workgroup (same arguments, same values as per point)
  // no fluid node of the box near the interface (the box kernel's flag): no force
  if (!P.cap_on) return;
  constexpr int TAB = 512;
  __shared__ double t_sa[TAB], t_ca[TAB], t_sp[TAB], t_cp[TAB];
  const bool tab = na <= TAB && nph <= TAB;
  if (tab) {
    for (int j = threadIdx.x; j < na; j += blockDim.x) sincos((j + 0.5) * da, &t_sa[j], &t_ca[j]);
    for (int k = threadIdx.x; k < nph; k += blockDim.x) sincos(k * da, &t_sp[k], &t_cp[k]);
  }
  __syncthreads();
  double acc[6] = {0, 0, 0, 0, 0, 0};
  for (int idx = blockIdx.x * blockDim.x + threadIdx.x; idx < na * nph;
       idx += gridDim.x * blockDim.x) {
    const int j = idx / nph, k = idx % nph;
    double sa, ca, sp, cp;
    if (tab) {
      sa = t_sa[j];
      ca = t_ca[j];
      sp = t_sp[k];
      cp = t_cp[k];
    } else {
      sincos((j + 0.5) * da, &sa, &ca);
      sincos(k * da, &sp, &cp);
    }
    const double sh[3] = {sa * cp, sa * sp, ca};
    const double xp[3] = {P.x[0] + R * sh[0], P.x[1] + R * sh[1], P.x[2] + R * sh[2]};
    const double f0 = floor(xp[0]), f1 = floor(xp[1]), f2 = floor(xp[2]);
    const double fr0 = xp[0] - f0, fr1 = xp[1] - f1, fr2 = xp[2] - f2;
    const int i0 = (int)f0 - org0, i1 = (int)f1 - org1, i2 = (int)f2 - org2;
    // per-point arithmetic in FP64: the torque is a small residual of large,
    // cancelling per-point moments
    double W = 0.0, phi = 0.0, Gx = 0.0, Gy = 0.0, Gz = 0.0;
    // the eight corners loaded at once; a solid corner (phi = 2) takes weight
    // 0, which adds exact zeros (the box holds finite values): the same sums as
    // leaving it out, without a load round trip per corner
    v4f cv[8];
#pragma unroll
    for (int c = 0; c < 8; ++c) {
      const int ox = c & 1, oy = (c >> 1) & 1, oz = c >> 2;
      cv[c] = box[(i0 + ox) + B * ((i1 + oy) + B * (i2 + oz))];
    }
#pragma unroll
    for (int c = 0; c < 8; ++c) {
      const int ox = c & 1, oy = (c >> 1) & 1, oz = c >> 2;
      const v4f v = cv[c];
      const double w = (ox ? fr0 : 1.0 - fr0) * (oy ? fr1 : 1.0 - fr1) * (oz ? fr2 : 1.0 - fr2);
      const double wf = v.x > 1.5f ? 0.0 : w;
      W += wf;
      phi += wf * (double)v.x;
      Gx += wf * (double)v.y;
      Gy += wf * (double)v.z;
      Gz += wf * (double)v.w;
    }
    // the three tests at once, after the values they need (W = 0 gives NaN,
    // which fails them): a test on W and phi alone before G is formed would let
    // the compiler load the corners' G only after it, a second round trip
    const double iW = 1.0 / W;
    phi *= iW;
    Gx *= iW;
    Gy *= iW;
    Gz *= iW;
    const double wgt = 1.0 - phi * phi;
    const double g = sqrt(Gx * Gx + Gy * Gy + Gz * Gz);
    if (!(W > 0.0) || !(wgt > 0.0) || !(g > (double)EPS_G)) continue;
    const double ig = 1.0 / g;
    const double nx_ = Gx * ig, ny_ = Gy * ig, nz_ = Gz * ig;
    const double a = nx_ * sh[0] + ny_ * sh[1] + nz_ * sh[2];
    const double mx = sh[0] - a * nx_, my = sh[1] - a * ny_, mz = sh[2] - a * nz_;
    const double mn = sqrt(mx * mx + my * my + mz * mz);
    if (!(mn > (double)EPS_T)) continue;
    const double dA = R * R * sa * da * da;
    const double coef = pref * wgt * dA / mn;
    const double dF[3] = {coef * mx, coef * my, coef * mz};
    const double arm[3] = {R * sh[0], R * sh[1], R * sh[2]};
    acc[0] += dF[0];
    acc[1] += dF[1];
    acc[2] += dF[2];
    acc[3] += arm[1] * dF[2] - arm[2] * dF[1];
    acc[4] += arm[2] * dF[0] - arm[0] * dF[2];
    acc[5] += arm[0] * dF[1] - arm[1] * dF[0];
  }
  __shared__ double red[6][256];
  for (int k = 0; k < 6; ++k) red[k][threadIdx.x] = acc[k];
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if ((int)threadIdx.x < o)
      for (int k = 0; k < 6; ++k) red[k][threadIdx.x] += red[k][threadIdx.x + o];
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    for (int k = 0; k < 3; ++k) {
      atomicAdd(&P.Fca[k], red[k][0]);
      atomicAdd(&P.Tca[k], red[3 + k][0]);
    }
  }
}

// -------------------------------------------------------------------- DEM
__device__ inline void cross3(const double* a, const double* b, double* o) {
  o[0] = a[1] * b[2] - a[2] * b[1];
  o[1] = a[2] * b[0] - a[0] * b[2];
  o[2] = a[0] * b[1] - a[1] * b[0];
}
__device__ inline double dot3(const double* a, const double* b) {
  return a[0] * b[0] + a[1] * b[1] + a[2] * b[2];
}

// Slot of `partner` in a particle's contact table (created if asked and free
// slots remain).  ids holds the table's partner ids in registers (the caller
// loads them once per contact phase) and is kept in step with the table.
__device__ __forceinline__ Contact* find_slot(Contact* t, int* ids, int partner, bool create,
                                              uint32_t* status) {
  int found = -1, freek = -1;
#pragma unroll
  for (int k = MAXC - 1; k >= 0; --k) {
    const int pk = ids[k];
    if (pk == partner) found = k;
    if (pk == -100) freek = k;
  }
  if (found >= 0) return &t[found];
  if (!create) return nullptr;
  if (freek >= 0) {
    t[freek].partner = partner;
#pragma unroll
    for (int k = 0; k < MAXC; ++k)
      if (k == freek) ids[k] = partner;
    for (int d = 0; d < 3; ++d) t[freek].xt[d] = t[freek].xr[d] = 0.0;
    return &t[freek];
  }
  atomicOr(status, (uint32_t)ST_CONTACT_FULL);
  return nullptr;
}

// spring with a Coulomb cap (sliding friction eqs.; rolling uses the same rule)
__device__ inline void capped_spring(double k, double gam, double cap, double* xi, const double* v,
                                     double dt, double* F) {
  double F0[3];
  for (int d = 0; d < 3; ++d) F0[d] = -k * xi[d] - gam * v[d];
  const double f0 = sqrt(dot3(F0, F0));
  if (f0 <= cap) {
    for (int d = 0; d < 3; ++d) {
      F[d] = F0[d];
      xi[d] += v[d] * dt;
    }
  } else {
    for (int d = 0; d < 3; ++d) F[d] = cap * F0[d] / f0;
    for (int d = 0; d < 3; ++d) xi[d] = (k > 0.0) ? -(F[d] + gam * v[d]) / k : 0.0;
  }
}

// Contact of particle i with one partner (normal spring-dashpot, sliding and
// rolling friction after Luding's model as the paper describes it).
__device__ __forceinline__ bool contact(const SimDev& s, Contact* tab, int* ids, int partner,
                                        double delta, const double* nh, const double* vi,
                                        const double* wi, const double* vj, const double* wj,
                                        double Rci, double Rcj, const double* armj, double mu,
                                        double mur, double dt, double* Fo, double* To) {
  if (!(delta > 0.0)) {
    Contact* sl = find_slot(tab, ids, partner, false, &s.counters[1]);
    if (sl) {
      sl->partner = -100;
#pragma unroll
      for (int k = 0; k < MAXC; ++k)
        if (ids[k] == partner) ids[k] = -100;
    }
    return false;
  }
  Contact* sl = find_slot(tab, ids, partner, true, &s.counters[1]);
  if (!sl) return false;
  double vrel[3];
  for (int d = 0; d < 3; ++d) vrel[d] = vi[d] - vj[d];
  const double ddot = -dot3(vrel, nh);
  const double Fn = s.kn * delta + s.gn * ddot;
  double ri[3], rj[3], t1[3], t2[3], vc[3];
  for (int d = 0; d < 3; ++d) ri[d] = -(Rci - 0.5 * delta) * nh[d];
  for (int d = 0; d < 3; ++d) rj[d] = ri[d] + armj[d];
  cross3(wi, ri, t1);
  cross3(wj, rj, t2);
  for (int d = 0; d < 3; ++d) vc[d] = vrel[d] + t1[d] - t2[d];
  const double vn = dot3(vc, nh);
  double vt[3];
  for (int d = 0; d < 3; ++d) vt[d] = vc[d] - vn * nh[d];
  double xn = dot3(sl->xt, nh);
  for (int d = 0; d < 3; ++d) sl->xt[d] -= xn * nh[d];
  xn = dot3(sl->xr, nh);
  for (int d = 0; d < 3; ++d) sl->xr[d] -= xn * nh[d];
  const double Fcap = mu * (Fn > 0.0 ? Fn : 0.0);
  double Ft[3];
  capped_spring(s.kt, s.gt, Fcap, sl->xt, vt, dt, Ft);
  const double ap = (Rcj > 0.0) ? Rci * Rcj / (Rci + Rcj) : Rci;
  double nwi[3], nwj[3], vr[3], Fr[3];
  cross3(nh, wi, nwi);
  cross3(nh, wj, nwj);
  for (int d = 0; d < 3; ++d) vr[d] = -ap * (nwi[d] - nwj[d]);
  const double Rcap = mur * (Fn > 0.0 ? Fn : 0.0);
  capped_spring(s.kr, s.gr, Rcap, sl->xr, vr, dt, Fr);
  double Tt[3], Tr[3];
  cross3(ri, Ft, Tt);
  cross3(nh, Fr, Tr);
  for (int d = 0; d < 3; ++d) {
    Fo[d] = Fn * nh[d] + Ft[d];
    To[d] = Tt[d] + ap * Tr[d];
  }
  return true;
}

__device__ inline void rel_vec(const SimDev& s, const double* a, const double* b, double* d) {
  d[0] = wrapd(a[0] - b[0], (double)s.nx);
  d[1] = wrapd(a[1] - b[1], (double)s.ny);
  d[2] = wrapd(a[2] - b[2], (double)s.nz);
}

__device__ void quat_rotate(double* q, const double* th) {
  const double a = sqrt(dot3(th, th));
  if (!(a > 0.0)) return;
  const double h = 0.5 * a, sh = sin(h) / a;
  const double dq[4] = {cos(h), th[0] * sh, th[1] * sh, th[2] * sh};
  double r[4] = {dq[0] * q[0] - dq[1] * q[1] - dq[2] * q[2] - dq[3] * q[3],
                 dq[0] * q[1] + dq[1] * q[0] + dq[2] * q[3] - dq[3] * q[2],
                 dq[0] * q[2] - dq[1] * q[3] + dq[2] * q[0] + dq[3] * q[1],
                 dq[0] * q[3] + dq[1] * q[2] - dq[2] * q[1] + dq[3] * q[0]};
  const double nq = sqrt(r[0] * r[0] + r[1] * r[1] + r[2] * r[2] + r[3] * r[3]);
  for (int k = 0; k < 4; ++k) q[k] = r[k] / nq;
}

// dst[0, n1 + n2) = src1[0, n1) followed by src2[0, n2), by the whole
// workgroup: 20 loads per thread issued before their stores, so that a small
// box's particle records and contact tables arrive in one memory round trip
__device__ __forceinline__ void stage_in(double* dst, const double* src1, int n1,
                                         const double* src2, int n2) {
  constexpr int U = 20;
  const int nt = (int)blockDim.x, n = n1 + n2;
  for (int base = (int)threadIdx.x; base < n; base += U * nt) {
    double v[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int k = base + u * nt;
      v[u] = k < n1 ? src1[k] : (k < n ? src2[k - n1] : 0.0);
    }
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int k = base + u * nt;
      if (k < n) dst[k] = v[u];
    }
  }
}

// Contact geometry of a particle at x with the static wall: partner -1 is the
// plane's top face (normal +z, surface z = 1/2) or the tube (the cylinder
// r = R_t, normal from the wall to the centre, towards the axis), -2 the
// plane's underside seen through the periodic z direction (normal -z, surface
// z = nz - 1/2).  delta is the overlap with the mechanical radius Rc; false if
// the simulation has no such wall face.
__device__ __forceinline__ bool wall_geom(const SimDev& s, const double* x, double Rc, int partner,
                                          double& delta, double* nh) {
  nh[0] = nh[1] = nh[2] = 0.0;
  if (s.has_wall == 3 && partner <= -3) {
    // box -3 - b of a textured wall: its nearest surface point; no contact
    // while the centre is inside the box
    const int b = -3 - partner;
    if (b >= s.n_boxes) return false;
    const int* B = s.boxes[b];
    double d[3];
    for (int k = 0; k < 3; ++k) {
      const double lo = B[k] - 0.5, hi = B[3 + k] + 0.5;
      d[k] = x[k] - (x[k] < lo ? lo : (x[k] > hi ? hi : x[k]));
    }
    const double dn = sqrt(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]);
    if (!(dn > 0.0)) {
      delta = -1.0;
      return true;
    }
    for (int k = 0; k < 3; ++k) nh[k] = d[k] / dn;
    delta = Rc - dn;
    return true;
  }
  if (s.has_wall == 1 || s.has_wall == 3) {
    if (partner == -1) {
      delta = Rc - (x[2] - 0.5);
      nh[2] = 1.0;
    } else {
      delta = Rc - (((double)s.nz - 0.5) - x[2]);
      nh[2] = -1.0;
    }
    return true;
  }
  if (s.has_wall == 2 && partner == -1) {
    const double dy = x[1] - s.tube_yc, dz = x[2] - s.tube_zc;
    const double r = sqrt(dy * dy + dz * dz);
    if (r > 0.0) {
      nh[1] = -dy / r;
      nh[2] = -dz / r;
    }
    delta = Rc - (sqrt(s.tube_R2) - r);
    return true;
  }
  return false;
}

// Contact forces and torques on one particle from the walls and from its
// candidates.  T is the record type the particle data is read from (DevParticle
// or DemView: the same field names); cand(q) is the q-th candidate or -1 past
// the last; rec(j) is particle j's record.
template <class T, class Cand, class Rec>
__device__ __forceinline__ void dem_contacts(const SimDev& s, Contact* tab, const T& me,
                                             Cand cand, Rec rec, double dt, double* Fs,
                                             double* Ts) {
  const double Rci = me.Rc;
  const double zero[3] = {0, 0, 0};
  double Fo[3], To[3];
  // partner ids of the contact table in registers for the whole phase (the
  // table is written only by this thread): one memory round trip, not one per
  // contact evaluated
  int ids[MAXC];
#pragma unroll
  for (int k = 0; k < MAXC; ++k) ids[k] = tab[k].partner;
  for (int w = -1; w >= -2 - (s.has_wall == 3 ? s.n_boxes : 0); --w) {
    double dw, nw[3];
    if (!wall_geom(s, me.x, Rci, w, dw, nw)) continue;
    if (contact(s, tab, ids, w, dw, nw, me.vp, me.wp, zero, zero, Rci, 0.0, zero, me.mu_s,
                me.mu_r, dt, Fo, To))
      for (int d = 0; d < 3; ++d) {
        Fs[d] += Fo[d];
        Ts[d] += To[d];
      }
  }
  for (int q = 0; q < MAXNB; ++q) {
    const int j = cand(q);
    if (j < 0) break;
    const T& pj = rec(j);
    const double Rcj = pj.Rc;
    double dx[3];
    rel_vec(s, me.x, pj.x, dx);
    const double dist = sqrt(dot3(dx, dx));
    const double delta = Rci + Rcj - dist;
    double nh[3] = {0, 0, 0};
    if (dist > 0.0)
      for (int d = 0; d < 3; ++d) nh[d] = dx[d] / dist;
    if (contact(s, tab, ids, j, delta, nh, me.vp, me.wp, pj.vp, pj.wp, Rci, Rcj, dx,
                0.5 * (me.mu_s + pj.mu_s), 0.5 * (me.mu_r + pj.mu_r), dt, Fo, To))
      for (int d = 0; d < 3; ++d) {
        Fs[d] += Fo[d];
        Ts[d] += To[d];
      }
  }
}

// The pair tests of the DEM's candidate search spread over the GPU (boxes with
// up to 32 MAXNB particles): the tests of particle i against partners
// 32 w .. 32 w + 31 (centre distance, minimum image, below Rc_i + Rc_j + skin)
// form the hit mask stored as word w of row i of the candidate-list buffer
// (MAXNB words per particle), which k_dem_setup turns into the candidate list.
// Positions and contact radii are those the step starts from.  Grid
// (ceil(32 np_max ceil(np_max / 32) / 256), nsim).
__global__ __launch_bounds__(256) void k_dem_search(Batch bt) {
  // one thread per (particle i, partner j): half a wave takes the 32 partners
  // of one hit word and a ballot forms the word (one round of loads)
  const SimDev& s = bt.tab[blockIdx.y];
  const int np = s.np;
  const int nw = (np + 31) / 32;
  const long long t = (long long)blockIdx.x * 256 + threadIdx.x;
  const long long r = t / 32;  // word index (i, w)
  const int u = (int)(t & 31);
  const bool inr = r < (long long)np * nw;
  const int i = inr ? (int)(r / nw) : 0, w = inr ? (int)(r % nw) : 0;
  const int j = 32 * w + u;
  bool hit = false;
  if (inr && j < np && j != i) {
    const DevParticle* PP = s.P;
    const double skin = 1.5;
    const double xi[3] = {PP[i].x[0], PP[i].x[1], PP[i].x[2]};
    const double xj[3] = {PP[j].x[0], PP[j].x[1], PP[j].x[2]};
    double dx[3];
    rel_vec(s, xi, xj, dx);
    const double lim = PP[i].Rc + PP[j].Rc + skin;
    hit = dot3(dx, dx) < lim * lim;
  }
  const unsigned long long b = __ballot(hit);
  const uint32_t word = (uint32_t)(b >> (threadIdx.x & 32));
  if (inr && u == 0) ((uint32_t*)s.nb)[(long long)i * MAXNB + w] = word;
}

// Boxes with few particles (their records, contact tables and candidate
// lists fit 64 KB of LDS): one workgroup per simulation, everything staged in
// LDS for the whole lattice step (the dependent FP64 chains then wait on LDS,
// not on L2/HBM) and written back at the end.  Fluid forces (momentum exchange
// + capillary) are held over n_sub velocity-Verlet sub-steps; contacts are
// evaluated at the new positions with the predicted velocities; gravity is the
// downward g_p.
__global__ __launch_bounds__(256) void k_dem(Batch bt) {
  const SimDev& s = bt.tab[blockIdx.x];
  if (s.np == 0) return;
  extern __shared__ double dem_lds[];
  const int np = s.np;
  const int nt = blockDim.x;
  const size_t wP = (size_t)np * sizeof(DevParticle) / 8;
  const size_t wC = (size_t)np * MAXC * sizeof(Contact) / 8;
  double* lp = dem_lds;
  double* lc = lp + wP;
  DevParticle* PP = (DevParticle*)lp;
  Contact* CT = (Contact*)lc;
  int* NB = (int*)(lc + wC);
  // records and contact tables in one pass (lc follows lp)
  stage_in(lp, (const double*)s.P, (int)wP, (const double*)s.ct, (int)wC);
  __syncthreads();
  const double dt = 1.0 / s.n_sub;
  const double skin = 1.5;
  // per-step set-up: fluid force and torque, the mean of this and the previous
  // lattice step (the averaging of the Verlet update over the previous and
  // current step)
  for (int i = threadIdx.x; i < np; i += nt) {
    DevParticle& P = PP[i];
    for (int d = 0; d < 3; ++d) {
      P.Fcap[d] = P.Fca[d];
      P.Tcap[d] = P.Tca[d];
      P.Fca[d] = 0.0;
      P.Tca[d] = 0.0;
      const double fc = P.Fh[d] + P.Fcap[d], tc = P.Th[d] + P.Tcap[d];
      const double fp = P.havep ? P.Ffp[d] : fc, tp = P.havep ? P.Tfp[d] : tc;
      P.Ff[d] = 0.5 * (fc + fp);
      P.Tf[d] = 0.5 * (tc + tp);
      P.Ffp[d] = fc;
      P.Tfp[d] = tc;
      P.Fh_last[d] = P.Fh[d];
      P.Th_last[d] = P.Th[d];
      P.Fh[d] = 0.0;
      P.Th[d] = 0.0;
      P.xo[d] = P.x[d];
      P.Facc[d] = 0.0;
      P.Tacc[d] = 0.0;
    }
    P.Ff[2] -= P.g_p;
    P.Ro = P.R;
    P.havep = 1;
    P.cap_on = 0;
  }
  __syncthreads();
  // pair candidates within Rc_i + Rc_j + skin (ascending index)
  for (int i = threadIdx.x; i < np; i += nt) {
    const DevParticle& me = PP[i];
    int* nb = NB + (long long)i * MAXNB;
    int c = 0;
    // 32 partners per pass: the tests only set bits (no stores between the
    // loads), then the hits are appended in ascending order
    for (int j0 = 0; j0 < np; j0 += 32) {
      const int jn = min(32, np - j0);
      uint32_t hit = 0;
#pragma unroll 4
      for (int u = 0; u < jn; ++u) {
        const int j = j0 + u;
        double dx[3];
        rel_vec(s, me.x, PP[j].x, dx);
        const double lim = me.Rc + PP[j].Rc + skin;
        if (j != i && dot3(dx, dx) < lim * lim) hit |= 1u << u;
      }
      while (hit) {
        const int j = j0 + __builtin_ctz(hit);
        hit &= hit - 1;
        if (c < MAXNB)
          nb[c++] = j;
        else
          atomicOr(&s.counters[1], (uint32_t)ST_CONTACT_FULL);
      }
    }
    if (c < MAXNB) nb[c] = -1;
    // free pair springs whose partner is out of range
    Contact* tab = CT + (long long)i * MAXC;
    for (int k = 0; k < MAXC; ++k) {
      const int pt = tab[k].partner;
      if (pt < 0) continue;
      bool found = false;
      for (int q = 0; q < c && q < MAXNB; ++q) found |= nb[q] == pt;
      if (!found) tab[k].partner = -100;
    }
  }
  __syncthreads();
  for (int sub = 0; sub < s.n_sub; ++sub) {
    for (int i = threadIdx.x; i < np; i += nt) {
      DevParticle& P = PP[i];
      double th[3];
      for (int d = 0; d < 3; ++d) {
        if (P.kin) {
          P.ao[d] = 0.0;
          P.bo[d] = 0.0;
        } else {
          P.ao[d] = (P.Ff[d] + P.Fcp[d]) / P.mass;
          P.bo[d] = (P.Tf[d] + P.Tcp[d]) / P.inertia;
        }
        P.x[d] += P.v[d] * dt + 0.5 * P.ao[d] * dt * dt;
        th[d] = P.w[d] * dt + 0.5 * P.bo[d] * dt * dt;
        P.vp[d] = P.v[d] + P.ao[d] * dt;
        P.wp[d] = P.w[d] + P.bo[d] * dt;
      }
      quat_rotate(P.q, th);
      const double L[3] = {(double)s.nx, (double)s.ny, (double)s.nz};
      for (int d = 0; d < 3; ++d) {
        if ((d == 2 && s.has_wall) || (d == 0 && s.open_x)) continue;
        if (P.x[d] >= L[d])
          P.x[d] -= L[d];
        else if (P.x[d] < 0.0)
          P.x[d] += L[d];
      }
    }
    __syncthreads();
    for (int i = threadIdx.x; i < np; i += nt) {
      DevParticle& P = PP[i];
      Contact* tab = CT + (long long)i * MAXC;
      double Fs[3] = {0, 0, 0}, Ts[3] = {0, 0, 0};
      const int* nb = NB + (long long)i * MAXNB;
      dem_contacts(
          s, tab, P, [&](int q) { return nb[q]; },
          [&](int j) -> const DevParticle& { return PP[j]; }, dt, Fs, Ts);
      for (int d = 0; d < 3; ++d) {
        P.Fcn[d] = Fs[d];
        P.Tcn[d] = Ts[d];
      }
    }
    __syncthreads();
    for (int i = threadIdx.x; i < np; i += nt) {
      DevParticle& P = PP[i];
      for (int d = 0; d < 3; ++d) {
        if (!P.kin) {
          const double an = (P.Ff[d] + P.Fcn[d]) / P.mass;
          const double bn = (P.Tf[d] + P.Tcn[d]) / P.inertia;
          P.v[d] += 0.5 * (P.ao[d] + an) * dt;
          P.w[d] += 0.5 * (P.bo[d] + bn) * dt;
        }
        P.Fcp[d] = P.Fcn[d];
        P.Tcp[d] = P.Tcn[d];
        P.Facc[d] += P.Fcn[d];
        P.Tacc[d] += P.Tcn[d];
      }
    }
    __syncthreads();
  }
  const unsigned long long step = *s.step_counter;
  for (int i = threadIdx.x; i < np; i += nt) {
    DevParticle& P = PP[i];
    for (int d = 0; d < 3; ++d) {
      P.Fcon[d] = P.Facc[d] / s.n_sub;
      P.Tcon[d] = P.Tacc[d] / s.n_sub;
    }
    if (near_open_end(s, P.x[0], P.R)) atomicOr(&s.counters[1], (uint32_t)ST_OPEN_END);
    if (s.hist_cap > 0) {
      double* h = s.hist + ((long long)(step % (unsigned long long)s.hist_cap) * np + i) *
                               LBM_HIST_DOUBLES_DEV;
      for (int d = 0; d < 3; ++d) {
        h[d] = P.Fh_last[d];
        h[3 + d] = P.Th_last[d];
        h[6 + d] = P.Fcap[d];
        h[9 + d] = P.Tcap[d];
        h[12 + d] = P.Fcon[d];
        h[15 + d] = P.Tcon[d];
        h[18 + d] = P.x[d];
        h[21 + d] = P.v[d];
        h[24 + d] = P.w[d];
      }
    }
  }
  __syncthreads();
  for (size_t k = threadIdx.x; k < wP; k += blockDim.x) ((double*)s.P)[k] = dem_lds[k];
  for (size_t k = threadIdx.x; k < wC; k += blockDim.x) ((double*)s.ct)[k] = dem_lds[wP + k];
  if (threadIdx.x == 0) *s.step_counter = step + 1;
}

// ---------------------------------------------- DEM over the whole GPU
// Boxes with more particles than the LDS variants hold well: each lattice step
// runs k_dem_setup (one thread per particle: fluid force mean, candidate list,
// predictor of the first sub-step), then per DEM sub-step one launch of
// k_dem_sub with a wave per particle: lane q < MAXNB evaluates the contact
// with candidate q, lanes MAXNB and MAXNB + 1 the wall and its underside; the
// contact forces are summed over the wave, and lane 0 applies the corrector and
// the predictor of the next sub-step.  The positions and predicted velocities
// the contacts read are the view of the sub-step (two buffers, so that a
// sub-step's predictor does not overwrite what its contacts still read), and
// a particle's contact table is written only by its own wave.

// Predictor of a sub-step (velocity Verlet, held fluid force, contact force of
// the last sub-step): new centre, orientation and predicted velocities, into
// the record and the view.
__device__ void dem_predict(const SimDev& s, DevParticle& P, DemView& v, double dt) {
  // every field read before the first store (a load behind a store to the
  // record would wait for it)
  const int kin = P.kin;
  const double mass = P.mass, inertia = P.inertia;
  const int nx = s.nx, ny = s.ny, nz = s.nz, has_wall = s.has_wall, open_x = s.open_x;
  double Ff[3], Fcp[3], Tf[3], Tcp[3], X[3], V[3], W[3];
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    Ff[d] = P.Ff[d];
    Fcp[d] = P.Fcp[d];
    Tf[d] = P.Tf[d];
    Tcp[d] = P.Tcp[d];
    X[d] = P.x[d];
    V[d] = P.v[d];
    W[d] = P.w[d];
  }
  double th[3], ao[3], bo[3], vp[3], wp[3];
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    if (kin) {
      ao[d] = 0.0;
      bo[d] = 0.0;
    } else {
      ao[d] = (Ff[d] + Fcp[d]) / mass;
      bo[d] = (Tf[d] + Tcp[d]) / inertia;
    }
    X[d] += V[d] * dt + 0.5 * ao[d] * dt * dt;
    th[d] = W[d] * dt + 0.5 * bo[d] * dt * dt;
    vp[d] = V[d] + ao[d] * dt;
    wp[d] = W[d] + bo[d] * dt;
  }
  const double L[3] = {(double)nx, (double)ny, (double)nz};
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    if ((d == 2 && has_wall) || (d == 0 && open_x)) continue;
    if (X[d] >= L[d])
      X[d] -= L[d];
    else if (X[d] < 0.0)
      X[d] += L[d];
  }
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    P.ao[d] = ao[d];
    P.bo[d] = bo[d];
    P.x[d] = X[d];
    P.vp[d] = vp[d];
    P.wp[d] = wp[d];
    v.x[d] = X[d];
    v.vp[d] = vp[d];
    v.wp[d] = wp[d];
  }
  quat_rotate(P.q, th);
}

// Pair candidates of every particle within Rc_i + Rc_j + skin by a full loop
// (boxes too large for the hit masks of k_dem_search), ascending, as lists
// of the candidate-list buffer (-1 after the last).
__global__ __launch_bounds__(64) void k_dem_lists(Batch bt, int np_rows) {
  const int r = blockIdx.x * 64 + threadIdx.x;
  if (r >= np_rows) return;
  const int2 sp = batch_particle(bt, r);
  const SimDev& s = bt.tab[sp.x];
  const int i = sp.y, np = s.np;
  const DevParticle* PP = s.P;
  const double skin = 1.5;
  const double xi[3] = {PP[i].x[0], PP[i].x[1], PP[i].x[2]};
  const double Rci = PP[i].Rc;
  int* nb = s.nb + (long long)i * MAXNB;
  int c = 0;
  for (int j = 0; j < np; ++j) {
    if (j == i) continue;
    const double xj[3] = {PP[j].x[0], PP[j].x[1], PP[j].x[2]};
    double dx[3];
    rel_vec(s, xi, xj, dx);
    const double lim = Rci + PP[j].Rc + skin;
    if (dot3(dx, dx) < lim * lim) {
      if (c < MAXNB)
        nb[c++] = j;
      else
        atomicOr(&s.counters[1], (uint32_t)ST_CONTACT_FULL);
    }
  }
  if (c < MAXNB) nb[c] = -1;
}

// Per-step set-up of one particle (thread): held fluid force and torque (mean
// of this and the previous lattice step) and gravity, its candidate list (from
// k_dem_search's hit masks when `masks`, else the lists of k_dem_lists), the
// springs of partners that left it freed, the predictor of the first
// sub-step into view 0, and the constant view fields in both views.
__global__ __launch_bounds__(64) void k_dem_setup(Batch bt, int np_rows, int masks) {
  const int r = blockIdx.x * 64 + threadIdx.x;
  if (r >= np_rows) return;
  const int2 sp = batch_particle(bt, r);
  const SimDev& s = bt.tab[sp.x];
  const int i = sp.y, np = s.np;
  DevParticle& P = s.P[i];
  // every field read before the first store (a load behind a store to the
  // record waits for it: one round trip per component otherwise)
  double Fca[3], Tca[3], Fh[3], Th[3], Ffp[3], Tfp[3], X[3];
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    Fca[d] = P.Fca[d];
    Tca[d] = P.Tca[d];
    Fh[d] = P.Fh[d];
    Th[d] = P.Th[d];
    Ffp[d] = P.Ffp[d];
    Tfp[d] = P.Tfp[d];
    X[d] = P.x[d];
  }
  const int havep = P.havep;
  const double g_p = P.g_p, R = P.R;
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    P.Fcap[d] = Fca[d];
    P.Tcap[d] = Tca[d];
    P.Fca[d] = 0.0;
    P.Tca[d] = 0.0;
    const double fc = Fh[d] + Fca[d], tc = Th[d] + Tca[d];
    const double fp = havep ? Ffp[d] : fc, tp = havep ? Tfp[d] : tc;
    P.Ff[d] = 0.5 * (fc + fp) - (d == 2 ? g_p : 0.0);
    P.Tf[d] = 0.5 * (tc + tp);
    P.Ffp[d] = fc;
    P.Tfp[d] = tc;
    P.Fh_last[d] = Fh[d];
    P.Th_last[d] = Th[d];
    P.Fh[d] = 0.0;
    P.Th[d] = 0.0;
    P.xo[d] = X[d];
    P.Facc[d] = 0.0;
    P.Tacc[d] = 0.0;
  }
  P.Ro = R;
  P.havep = 1;
  P.cap_on = 0;
  // the step counter advances here (the sub-steps' history record takes the
  // value before it)
  if (i == 0) *s.step_counter += 1;
  int* nb = s.nb + (long long)i * MAXNB;
  int c = 0;
  // membership of a partner in this step's candidate list, from registers (a
  // re-read of the list just written would wait for its stores, per slot)
  uint32_t words[MAXNB];
  int lst[MAXNB];
  int jlast = -1;  // masks: the last partner the list took (it is capped at MAXNB)
  if (masks) {
    // row i holds one hit mask per 32 partners: all words read before the
    // list overwrites them
    const int nw = (np + 31) / 32;
#pragma unroll
    for (int w = 0; w < MAXNB; ++w) words[w] = w < nw ? ((const uint32_t*)nb)[w] : 0u;
#pragma unroll
    for (int w = 0; w < MAXNB; ++w) {
      uint32_t hit = words[w];
      while (hit) {
        const int j = 32 * w + __builtin_ctz(hit);
        hit &= hit - 1;
        if (c < MAXNB) {
          nb[c++] = j;
          jlast = j;
        } else {
          atomicOr(&s.counters[1], (uint32_t)ST_CONTACT_FULL);
        }
      }
    }
    if (c < MAXNB) nb[c] = -1;
  } else {
    // the list as k_dem_lists wrote it: entries up to the first negative one
    bool end = false;
#pragma unroll
    for (int w = 0; w < MAXNB; ++w) {
      lst[w] = nb[w];
      end |= lst[w] < 0;
      c += end ? 0 : 1;
    }
  }
  auto listed = [&](int pt) {
    bool r = false;
    if (masks) {
      // the list holds the set bits in increasing order up to jlast
#pragma unroll
      for (int w = 0; w < MAXNB; ++w) r |= (w == (pt >> 5)) && ((words[w] >> (pt & 31)) & 1u);
      return r && pt <= jlast;
    }
#pragma unroll
    for (int w = 0; w < MAXNB; ++w) r |= w < c && lst[w] == pt;
    return r;
  };
  // free pair springs whose partner is out of range
  Contact* tab = s.ct + (long long)i * MAXC;
  for (int k = 0; k < MAXC; ++k) {
    const int pt = tab[k].partner;
    if (pt < 0) continue;
    if (!listed(pt)) tab[k].partner = -100;
  }
  DemView* V0 = s.view;
  DemView* V1 = s.view + np;
  V0[i].Rc = V1[i].Rc = P.Rc;
  V0[i].mu_s = V1[i].mu_s = P.mu_s;
  V0[i].mu_r = V1[i].mu_r = P.mu_r;
  dem_predict(s, P, V0[i], 1.0 / s.n_sub);
}

// The contact force of one active contact whose spring slot sl is known
// (normal spring-dashpot, sliding and rolling friction after Luding's model as
// the paper describes it); the same arithmetic as contact().
__device__ __forceinline__ void contact_force(const SimDev& s, Contact* sl, double delta,
                                              const double* nh, const double* vi,
                                              const double* wi, const double* vj,
                                              const double* wj, double Rci, double Rcj,
                                              const double* armj, double mu, double mur,
                                              double dt, double* Fo, double* To) {
  double vrel[3];
  for (int d = 0; d < 3; ++d) vrel[d] = vi[d] - vj[d];
  const double ddot = -dot3(vrel, nh);
  const double Fn = s.kn * delta + s.gn * ddot;
  double ri[3], rj[3], t1[3], t2[3], vc[3];
  for (int d = 0; d < 3; ++d) ri[d] = -(Rci - 0.5 * delta) * nh[d];
  for (int d = 0; d < 3; ++d) rj[d] = ri[d] + armj[d];
  cross3(wi, ri, t1);
  cross3(wj, rj, t2);
  for (int d = 0; d < 3; ++d) vc[d] = vrel[d] + t1[d] - t2[d];
  const double vn = dot3(vc, nh);
  double vt[3];
  for (int d = 0; d < 3; ++d) vt[d] = vc[d] - vn * nh[d];
  double xt[3], xr[3];
  for (int d = 0; d < 3; ++d) {
    xt[d] = sl->xt[d];
    xr[d] = sl->xr[d];
  }
  double xn = dot3(xt, nh);
  for (int d = 0; d < 3; ++d) xt[d] -= xn * nh[d];
  xn = dot3(xr, nh);
  for (int d = 0; d < 3; ++d) xr[d] -= xn * nh[d];
  const double Fcap = mu * (Fn > 0.0 ? Fn : 0.0);
  double Ft[3];
  capped_spring(s.kt, s.gt, Fcap, xt, vt, dt, Ft);
  const double ap = (Rcj > 0.0) ? Rci * Rcj / (Rci + Rcj) : Rci;
  double nwi[3], nwj[3], vr[3], Fr[3];
  cross3(nh, wi, nwi);
  cross3(nh, wj, nwj);
  for (int d = 0; d < 3; ++d) vr[d] = -ap * (nwi[d] - nwj[d]);
  const double Rcap = mur * (Fn > 0.0 ? Fn : 0.0);
  capped_spring(s.kr, s.gr, Rcap, xr, vr, dt, Fr);
  for (int d = 0; d < 3; ++d) {
    sl->xt[d] = xt[d];
    sl->xr[d] = xr[d];
  }
  double Tt[3], Tr[3];
  cross3(ri, Ft, Tt);
  cross3(nh, Fr, Tr);
  for (int d = 0; d < 3; ++d) {
    Fo[d] = Fn * nh[d] + Ft[d];
    To[d] = Tt[d] + ap * Tr[d];
  }
}

// One DEM sub-step of every particle: a wave per particle (four per block).
__global__ __launch_bounds__(256) void k_dem_sub(Batch bt, int np_rows, int sub) {
  // the particle row is the same for the whole wave; declared uniform, it lets
  // the simulation record and the particle's own data be read by scalar loads
  const int r = __builtin_amdgcn_readfirstlane(blockIdx.x * 4 + ((int)threadIdx.x >> 6));
  const int lane = (int)threadIdx.x & 63;
  if (r >= np_rows) return;  // the whole wave
  const int2 sp = batch_particle(bt, r);
  const SimDev& s = bt.tab[sp.x];
  if (sub >= s.n_sub) return;
  const int i = sp.y, np = s.np;
  const double dt = 1.0 / s.n_sub;
  const DemView* V = s.view + (sub & 1) * np;
  const DemView& me = V[i];
  Contact* tab = s.ct + (long long)i * MAXC;
  int ids[MAXC];
#pragma unroll
  for (int k = 0; k < MAXC; ++k) ids[k] = tab[k].partner;
  // this lane's partner: candidate `lane`, or the wall (-1) or its underside (-2)
  int partner = -100;
  // lanes past the list's end stay idle (a list shorter than MAXNB ends at -1):
  // a lane is past it when a lower lane holds a negative entry (one ballot)
  const int j = lane < MAXNB ? s.nb[(long long)i * MAXNB + lane] : 0;
  const unsigned long long neg = __ballot(j < 0);
  if (lane < MAXNB) {
    partner = (j >= 0 && (neg & ((1ull << lane) - 1ull)) == 0ull) ? j : -100;
  } else if (lane == MAXNB && s.has_wall) {
    partner = -1;
  } else if (lane == MAXNB + 1 && s.has_wall) {
    partner = -2;
  } else if (lane >= MAXNB + 2 && s.has_wall == 3 && lane - (MAXNB + 2) < s.n_boxes) {
    partner = -3 - (lane - (MAXNB + 2));  // a box of the textured wall
  }
  // the partner's velocities by value (a pointer that may also point at a
  // local array of zeros puts that array in scratch and makes the loads generic)
  double delta = 0.0, nh[3] = {0.0, 0.0, 0.0}, arm[3] = {0.0, 0.0, 0.0};
  double vj[3] = {0.0, 0.0, 0.0}, wj[3] = {0.0, 0.0, 0.0};
  double Rcj = 0.0, mu = me.mu_s, mur = me.mu_r;
  if (partner >= 0) {
    const DemView& pj = V[partner];
    rel_vec(s, me.x, pj.x, arm);  // X_i - X_j, min image
    const double dist = sqrt(dot3(arm, arm));
    Rcj = pj.Rc;
    delta = me.Rc + Rcj - dist;
    if (dist > 0.0)
      for (int d = 0; d < 3; ++d) nh[d] = arm[d] / dist;
    for (int d = 0; d < 3; ++d) {
      vj[d] = pj.vp[d];
      wj[d] = pj.wp[d];
    }
    mu = 0.5 * (me.mu_s + pj.mu_s);
    mur = 0.5 * (me.mu_r + pj.mu_r);
  } else if (partner != -100) {
    if (!wall_geom(s, me.x, me.Rc, partner, delta, nh)) partner = -100;
  }
  const bool has = partner != -100;
  const bool active = has && delta > 0.0;
  int found = -1, nfree = 0;
#pragma unroll
  for (int k = MAXC - 1; k >= 0; --k)
    if (has && ids[k] == partner) found = k;
  // new contacts take the free slots in lane order (free before this pass)
  const unsigned long long need = __ballot(active && found < 0);
  const int rank = __popcll(need & ((1ull << lane) - 1ull));
  int slot = found;
  if (active && found < 0) {
    slot = -1;
#pragma unroll
    for (int k = 0; k < MAXC; ++k)
      if (ids[k] == -100) {
        if (nfree == rank) slot = k;
        ++nfree;
      }
    if (slot < 0) {
      atomicOr(&s.counters[1], (uint32_t)ST_CONTACT_FULL);
    } else {
      tab[slot].partner = partner;
      for (int d = 0; d < 3; ++d) tab[slot].xt[d] = tab[slot].xr[d] = 0.0;
    }
  }
  double acc[6] = {0, 0, 0, 0, 0, 0};
  if (active && slot >= 0) {
    double Fo[3], To[3];
    contact_force(s, &tab[slot], delta, nh, me.vp, me.wp, vj, wj, me.Rc, Rcj, arm, mu, mur, dt,
                  Fo, To);
    for (int d = 0; d < 3; ++d) {
      acc[d] = Fo[d];
      acc[3 + d] = To[d];
    }
  } else if (has && !active && found >= 0) {
    tab[found].partner = -100;  // the contact ended: its springs are released
  }
#pragma unroll
  for (int c = 0; c < 6; ++c)
    for (int off = 32; off > 0; off >>= 1) acc[c] += __shfl_xor(acc[c], off, 64);
  if (lane != 0) return;
  DevParticle& P = s.P[i];
  // every field read before the first store (a load behind a store to the
  // record would wait for it)
  const int kin = P.kin;
  const double mass = P.mass, inertia = P.inertia;
  double Ff[3], Tf[3], ao[3], bo[3], Vv[3], Ww[3], Fa[3], Ta[3];
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    Ff[d] = P.Ff[d];
    Tf[d] = P.Tf[d];
    ao[d] = P.ao[d];
    bo[d] = P.bo[d];
    Vv[d] = P.v[d];
    Ww[d] = P.w[d];
    Fa[d] = P.Facc[d];
    Ta[d] = P.Tacc[d];
  }
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    if (!kin) {
      const double an = (Ff[d] + acc[d]) / mass;
      const double bn = (Tf[d] + acc[3 + d]) / inertia;
      P.v[d] = Vv[d] + 0.5 * (ao[d] + an) * dt;
      P.w[d] = Ww[d] + 0.5 * (bo[d] + bn) * dt;
    }
    P.Fcp[d] = acc[d];
    P.Tcp[d] = acc[3 + d];
    P.Facc[d] = Fa[d] + acc[d];
    P.Tacc[d] = Ta[d] + acc[3 + d];
  }
  if (sub + 1 < s.n_sub) {
    dem_predict(s, P, s.view[((sub + 1) & 1) * np + i], dt);
    return;
  }
  // the last sub-step: contact means and the history record
  for (int d = 0; d < 3; ++d) {
    P.Fcon[d] = P.Facc[d] / s.n_sub;
    P.Tcon[d] = P.Tacc[d] / s.n_sub;
  }
  if (near_open_end(s, P.x[0], P.R)) atomicOr(&s.counters[1], (uint32_t)ST_OPEN_END);
  if (s.hist_cap > 0) {
    const unsigned long long step = *s.step_counter - 1;  // advanced by k_dem_setup
    double* h = s.hist + ((long long)(step % (unsigned long long)s.hist_cap) * np + i) *
                             LBM_HIST_DOUBLES_DEV;
    for (int d = 0; d < 3; ++d) {
      h[d] = P.Fh_last[d];
      h[3 + d] = P.Th_last[d];
      h[6 + d] = P.Fcap[d];
      h[9 + d] = P.Tcap[d];
      h[12 + d] = P.Fcon[d];
      h[15 + d] = P.Tcon[d];
      h[18 + d] = P.x[d];
      h[21 + d] = P.v[d];
      h[24 + d] = P.w[d];
    }
  }
}

// ------------------------------------------------------------ host launchers
static inline unsigned box_blocks(int B) {
  const int v = B * B * B;
  return (unsigned)((v + 255) / 256);
}

hipError_t launch_mask_update(const Batch& b, int np_rows, int Bmax, bool with_release,
                              hipStream_t st) {
  if (np_rows == 0) return hipSuccess;
  dim3 grid(box_blocks(Bmax), np_rows);
  hipLaunchKernelGGL(k_claim, grid, dim3(256), 0, st, b);
  if (with_release) hipLaunchKernelGGL(k_release, grid, dim3(256), 0, st, b);
  hipLaunchKernelGGL(k_cover, grid, dim3(256), 0, st, b);
  return hipGetLastError();
}

// fresh_cap_max: the largest fresh-list capacity of the batch; np_max: the
// most particles of one simulation; mode REFILL_STEP (in a step) or
// REFILL_BOUNDARY (between steps).  The grid row takes two blocks of 14 fresh
// nodes per particle (128 to 1,024): the fresh nodes of a step scale with the
// moving particles, and a block that must take a second round of them doubles
// the kernel's dependent chain (500 spheres: 196 -> 185 us for the particle
// phase with 1,000 blocks instead of 128)
hipError_t launch_refill(const Batch& b, int storage, size_t fresh_cap_max, int np_max, int mode,
                         hipStream_t st) {
  if (fresh_cap_max == 0) return hipSuccess;
  unsigned nb = (unsigned)((fresh_cap_max + 13) / 14);
  const unsigned cap = (unsigned)std::min(1024, std::max(128, 2 * np_max));
  if (nb > cap) nb = cap;
  if (nb == 0) nb = 1;
  const dim3 grid(nb, b.nsim);
  if (storage == 0) {
    if (mode == REFILL_STEP)
      hipLaunchKernelGGL((k_refill<0, REFILL_STEP>), grid, dim3(256), 0, st, b);
    else
      hipLaunchKernelGGL((k_refill<0, REFILL_BOUNDARY>), grid, dim3(256), 0, st, b);
  } else {
    if (mode == REFILL_STEP)
      hipLaunchKernelGGL((k_refill<1, REFILL_STEP>), grid, dim3(256), 0, st, b);
    else
      hipLaunchKernelGGL((k_refill<1, REFILL_BOUNDARY>), grid, dim3(256), 0, st, b);
  }
  return hipGetLastError();
}

// cap_B: the largest capillary-box side; npts: Lagrangian points per particle
hipError_t launch_capillary(const Batch& b, int np_rows, int cap_B, int npts, hipStream_t st) {
  if (np_rows == 0) return hipSuccess;
  hipLaunchKernelGGL(k_capbox, dim3(box_blocks(cap_B), np_rows), dim3(256), 0, st, b);
  // workgroups per particle: four points per thread, or down to one where
  // few particles leave the GPU idle (about 2,048 workgroups in all)
  const int wide = std::min(npts / 256, (2048 + np_rows - 1) / np_rows);
  const int many = std::max(1, (4096 + np_rows - 1) / np_rows);
  const unsigned split = (unsigned)std::max(1, std::min(64, std::max(std::min(npts / (256 * 4), many), wide)));
  hipLaunchKernelGGL(k_capillary, dim3(split, np_rows), dim3(256), 0, st, b);
  return hipGetLastError();
}

// np_max: the most particles of one simulation in the batch; np_rows: particle
// rows of the batch; n_sub_max: the most DEM sub-steps of one simulation
hipError_t launch_dem(const Batch& b, int np_max, int np_rows, int n_sub_max, hipStream_t st) {
  if (np_max == 0) return hipSuccess;
  static int max_lds = -1;
  if (max_lds < 0) {
    int dev = 0, v = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&v, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) != hipSuccess)
      v = 0;
    max_lds = v;
  }
  const size_t need = (size_t)np_max * (sizeof(DevParticle) + MAXC * sizeof(Contact)) +
                      (size_t)np_max * MAXNB * sizeof(int);
  if (need <= (size_t)max_lds && need <= 64 * 1024) {
    // few particles: one workgroup per simulation, everything in LDS (256
    // threads: a single wave was slower, C2 DEM 44 against 35 us)
    hipLaunchKernelGGL(k_dem, dim3(b.nsim), dim3(256), need, st, b);
    return hipGetLastError();
  }
  // many particles: set-up, then a launch per sub-step with a wave per particle
  const unsigned g64 = (unsigned)((np_rows + 63) / 64);
  if (np_max <= 32 * MAXNB) {
    // the pair tests on many CUs; the hit masks fit the list buffer
    const long long nw = (np_max + 31) / 32;
    const unsigned gx = (unsigned)(((long long)np_max * nw * 32 + 255) / 256);
    hipLaunchKernelGGL(k_dem_search, dim3(gx, b.nsim), dim3(256), 0, st, b);
    hipLaunchKernelGGL(k_dem_setup, dim3(g64), dim3(64), 0, st, b, np_rows, 1);
  } else {
    hipLaunchKernelGGL(k_dem_lists, dim3(g64), dim3(64), 0, st, b, np_rows);
    hipLaunchKernelGGL(k_dem_setup, dim3(g64), dim3(64), 0, st, b, np_rows, 0);
  }
  const unsigned g4 = (unsigned)((np_rows + 3) / 4);
  for (int sub = 0; sub < n_sub_max; ++sub)
    hipLaunchKernelGGL(k_dem_sub, dim3(g4), dim3(256), 0, st, b, np_rows, sub);
  return hipGetLastError();
}

}  // namespace lbm
