/*
 * lbm_oracle.c -- plain FP64 CPU reference of the coupled colour-gradient
 * lattice Boltzmann + discrete element time step of Naga, Zhang, Yang and
 * Kusumaatmaja, "Modelling droplet-particle interactions on solid surfaces by
 * coupling the lattice Boltzmann and discrete element methods" (arXiv 2505.10171).
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product library links, loads or
 * calls this file; only the test suite, the smoke check and the CPU-baseline leg
 * of the benchmark do.  It shares no code, header, table or constant generator
 * with the HIP path.
 *
 * Design rules: FP64 throughout, array-of-structures colour populations fa[n][19]
 * and fb[n][19] (the paper's own variables), the literal MRT matrix form of the
 * collision, push streaming, and the paper's order of operations.  OpenMP is used
 * only over independent nodes; every reduction (momentum exchange, capillary
 * force, mass) is a serial loop in a fixed order, so results do not depend on the
 * thread count.  Build with -O2 -fno-fast-math -ffp-contract=off.
 *
 * Per time step (section "Lattice Boltzmann model for fluid dynamics" and
 * section "Coupling between fluid and particles"; the flow-chart figure is not
 * available, so the order below is the reading of the text):
 *   S1  moments rho_a, rho_b, rho, phi                  (order-parameter eq.)
 *   S2  colour gradient G = grad phi (isotropic stencil)
 *   S3  geometric wetting: rotate G at fluid nodes next to a solid  (n_pm eq.)
 *   S4  unit normal n = G/|G|
 *   S5  curvature kappa = div n
 *   S6  force F = -sigma kappa G / 2 + body force on fluid a (CSF eq.)
 *   S7  velocity rho u = sum c f + F/2
 *   S8  local relaxation from the harmonic-mean viscosity
 *   S9  MRT collision with Guo forcing on the total f
 *   S10 recolouring into fa, fb
 *   S11 capillary force on particles from Lagrangian surface points
 *   S12 push streaming, half-way bounce-back with moving walls
 *   S13 momentum exchange on particle links (Galilean invariant form)
 *   S14 DEM: contacts, sliding and rolling friction, Verlet integration
 *   S15 new solid mask, refilling of fresh fluid nodes
 *
 * Geometry: the static solid is the node plane z = 0 (has_wall 1), a tube
 * along x (has_wall 2: nodes with (y - yc)^2 + (z - zc)^2 >= R_t^2 are solid,
 * yc = (ny - 1)/2, zc = (nz - 1)/2, section "Benchmarking hydrodynamic force"),
 * the plane with up to 8 boxes of solid nodes standing on it or above it
 * (has_wall 3: a textured wall, the paper's stated future work; box b holds
 * the nodes lo_b <= x <= hi_b in every axis, its solid surface is the box
 * grown by half a node, [lo_b - 1/2, hi_b + 1/2], as half-way bounce-back
 * places it), or nothing (has_wall 0).  With open_x the x direction is not periodic: the
 * planes x = -1/2 and x = nx - 1/2 are pressure boundaries held by the
 * anti-bounce-back rule of that section (pressure inlet/outlet eq.).
 *
 * Readings of passages that are silent, ambiguous or garbled are listed where
 * they are used; each is marked "reading:".
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define Q 19
#define MAXC 16

/* D3Q19 velocities: rest, +-x, +-y, +-z, then (+-1,+-1,0), (+-1,0,+-1),
 * (0,+-1,+-1), each group in ++, +-, -+, -- order. */
static const int CV[Q][3] = {
    {0, 0, 0},  {1, 0, 0},  {-1, 0, 0}, {0, 1, 0},  {0, -1, 0},
    {0, 0, 1},  {0, 0, -1}, {1, 1, 0},  {1, -1, 0}, {-1, 1, 0},
    {-1, -1, 0}, {1, 0, 1}, {1, 0, -1}, {-1, 0, 1}, {-1, 0, -1},
    {0, 1, 1},  {0, 1, -1}, {0, -1, 1}, {0, -1, -1}};

static double WT[Q];
static int OPPD[Q];
static double MM[Q][Q];   /* MRT transformation matrix (rows = moments) */
static double MINV[Q][Q]; /* its inverse, by Gauss-Jordan elimination     */
static int tables_ready = 0;

/* ------------------------------------------------------------------ structs */
typedef struct {
  int32_t nx, ny, nz, has_wall;
  double rho0, tau_a, tau_b, sigma, beta;
  double theta_wall_deg;
  double body_force[3];
  double kn, kt, kr, gn, gt, gr, delta_R;
  double cap_k, cap_dang_deg;
  int32_t n_particles, pad0;
  int32_t open_x, pad1;    /* 1: pressure boundaries at both ends of x      */
  double rho_in, rho_out;  /* their densities (pressure rho / 3)            */
  double tube_R;           /* radius of the tube (has_wall 2)               */
  int32_t n_boxes, pad2;   /* boxes of the textured wall (has_wall 3)       */
  int32_t boxes[8][6];     /* per box: lo x, y, z, hi x, y, z (node indices) */
} orc_config;

typedef struct {
  double x[3], v[3], w[3], q[4];
  double R, rho_p, theta_deg, mu_s, mu_r, g_p;
  int32_t kinematic, pad0;
  double F_hyd[3], T_hyd[3], F_cap[3], T_cap[3], F_con[3], T_con[3];
} orc_particle;

typedef struct {
  int partner; /* -1 bottom wall surface, -2 wall underside, >=0 particle, -100 free */
  double xt[3], xr[3];
} orc_contact;

typedef struct {
  orc_config c;
  int64_t N;
  double *fa, *fb;         /* N*Q current (post-stream) colour populations   */
  double *fa_new, *fb_new; /* N*Q streaming targets                           */
  uint16_t *mask;          /* 0 fluid, 1 wall, 2+p particle p                 */
  uint16_t *mask_new;
  double *rho_a, *rho_b, *phi; /* N */
  double *G, *nrm, *F, *u;     /* N*3 */
  orc_particle *P;
  orc_contact *ct;             /* n_particles * MAXC */
  double *Fc_prev, *Tc_prev;   /* contact force/torque of the last DEM sub-step */
  double *Ff_prev, *Tf_prev;   /* fluid force/torque of the previous lattice step */
  int have_prev;
  int n_sub;
  int64_t n_fresh;
  int status;
} orc_sim;

/* ------------------------------------------------------------ lattice tables */
static void build_tables(void) {
  if (tables_ready) return;
  for (int i = 0; i < Q; ++i) {
    int c2 = CV[i][0] * CV[i][0] + CV[i][1] * CV[i][1] + CV[i][2] * CV[i][2];
    WT[i] = (c2 == 0) ? 1.0 / 3.0 : (c2 == 1 ? 1.0 / 18.0 : 1.0 / 36.0);
    for (int j = 0; j < Q; ++j)
      if (CV[j][0] == -CV[i][0] && CV[j][1] == -CV[i][1] && CV[j][2] == -CV[i][2])
        OPPD[i] = j;
  }
  /* d'Humieres' D3Q19 moment basis, written as polynomials of c; the order
   * (rho, e, eps, jx, qx, jy, qy, jz, qz, 3pxx, 3pixx, pww, piww, pxy, pyz,
   * pxz, mx, my, mz) is the one the relaxation vector S is printed in. */
  for (int i = 0; i < Q; ++i) {
    double cx = CV[i][0], cy = CV[i][1], cz = CV[i][2];
    double c2 = cx * cx + cy * cy + cz * cz;
    double r[Q] = {1.0,
                   19.0 * c2 - 30.0,
                   (21.0 * c2 * c2 - 53.0 * c2 + 24.0) / 2.0,
                   cx,
                   (5.0 * c2 - 9.0) * cx,
                   cy,
                   (5.0 * c2 - 9.0) * cy,
                   cz,
                   (5.0 * c2 - 9.0) * cz,
                   3.0 * cx * cx - c2,
                   (3.0 * c2 - 5.0) * (3.0 * cx * cx - c2),
                   cy * cy - cz * cz,
                   (3.0 * c2 - 5.0) * (cy * cy - cz * cz),
                   cx * cy,
                   cy * cz,
                   cx * cz,
                   (cy * cy - cz * cz) * cx,
                   (cz * cz - cx * cx) * cy,
                   (cx * cx - cy * cy) * cz};
    for (int k = 0; k < Q; ++k) MM[k][i] = r[k];
  }
  /* Gauss-Jordan inversion with partial pivoting. */
  double A[Q][2 * Q];
  for (int r = 0; r < Q; ++r)
    for (int c = 0; c < 2 * Q; ++c) A[r][c] = (c < Q) ? MM[r][c] : (c - Q == r ? 1.0 : 0.0);
  for (int col = 0; col < Q; ++col) {
    int piv = col;
    for (int r = col + 1; r < Q; ++r)
      if (fabs(A[r][col]) > fabs(A[piv][col])) piv = r;
    if (piv != col)
      for (int c = 0; c < 2 * Q; ++c) {
        double t = A[col][c];
        A[col][c] = A[piv][c];
        A[piv][c] = t;
      }
    double d = A[col][col];
    for (int c = 0; c < 2 * Q; ++c) A[col][c] /= d;
    for (int r = 0; r < Q; ++r)
      if (r != col) {
        double m = A[r][col];
        if (m != 0.0)
          for (int c = 0; c < 2 * Q; ++c) A[r][c] -= m * A[col][c];
      }
  }
  for (int r = 0; r < Q; ++r)
    for (int c = 0; c < Q; ++c) MINV[r][c] = A[r][Q + c];
  tables_ready = 1;
}

/* ---------------------------------------------------------------- helpers */
static inline int wrapi(int a, int n) {
  a %= n;
  return a < 0 ? a + n : a;
}
/* reading: minimum image, a coordinate difference wrapped once into (-L/2, L/2] */
static inline double wrapd(double d, double L) {
  if (d > 0.5 * L)
    d -= L;
  else if (d <= -0.5 * L)
    d += L;
  return d;
}
static inline int64_t nidx(const orc_sim *s, int x, int y, int z) {
  return (int64_t)x + (int64_t)s->c.nx * ((int64_t)y + (int64_t)s->c.ny * z);
}
static inline void ncoord(const orc_sim *s, int64_t n, int *x, int *y, int *z) {
  *x = (int)(n % s->c.nx);
  int64_t r = n / s->c.nx;
  *y = (int)(r % s->c.ny);
  *z = (int)(r / s->c.ny);
}
/* direction i leaves the domain through an open end of x */
static inline int outside(const orc_sim *s, int x, int i) {
  return s->c.open_x && (x + CV[i][0] < 0 || x + CV[i][0] >= s->c.nx);
}
static inline int64_t neighbour(const orc_sim *s, int x, int y, int z, int i) {
  return nidx(s, wrapi(x + CV[i][0], s->c.nx), wrapi(y + CV[i][1], s->c.ny),
              wrapi(z + CV[i][2], s->c.nz));
}
static inline void cross3(const double a[3], const double b[3], double o[3]) {
  o[0] = a[1] * b[2] - a[2] * b[1];
  o[1] = a[2] * b[0] - a[0] * b[2];
  o[2] = a[0] * b[1] - a[1] * b[0];
}
static inline double dot3(const double a[3], const double b[3]) {
  return a[0] * b[0] + a[1] * b[1] + a[2] * b[2];
}
static inline double norm3(const double a[3]) { return sqrt(dot3(a, a)); }

/* min-image vector from particle centre X to point p */
static void rel_vec(const orc_sim *s, const double p[3], const double X[3], double d[3]) {
  d[0] = wrapd(p[0] - X[0], (double)s->c.nx);
  d[1] = wrapd(p[1] - X[1], (double)s->c.ny);
  d[2] = wrapd(p[2] - X[2], (double)s->c.nz);
}

/* surface velocity u_w = V + Omega x (x_w - X) of particle p at point xw */
static void wall_velocity(const orc_sim *s, int p, const double xw[3], double uw[3]) {
  const orc_particle *P = &s->P[p];
  double r[3], wr[3];
  rel_vec(s, xw, P->x, r);
  cross3(P->w, r, wr);
  for (int k = 0; k < 3; ++k) uw[k] = P->v[k] + wr[k];
}

/* Second-order equilibrium (refilling eq.; the collision uses the same form). */
static void equilibrium(double rho, const double u[3], double feq[Q]) {
  double uu = dot3(u, u);
  for (int i = 0; i < Q; ++i) {
    double cu = CV[i][0] * u[0] + CV[i][1] * u[1] + CV[i][2] * u[2];
    feq[i] = rho * WT[i] * (1.0 + 3.0 * cu + 4.5 * cu * cu - 1.5 * uu);
  }
}

/* Guo forcing source F-bar (force eq. with c_s^2 = 1/3). */
static void guo_source(const double u[3], const double F[3], double Fb[Q]) {
  double uF = dot3(u, F);
  for (int i = 0; i < Q; ++i) {
    double cF = CV[i][0] * F[0] + CV[i][1] * F[1] + CV[i][2] * F[2];
    double cu = CV[i][0] * u[0] + CV[i][1] * u[1] + CV[i][2] * u[2];
    Fb[i] = WT[i] * (3.0 * cF + 9.0 * cu * cF - 3.0 * uF);
  }
}

/* Literal MRT collision with Guo forcing (collision-step eq., MRT operator eq.,
 * relaxation vector S and forcing eq.):
 *   f* = f - M^-1 S M (f - feq) + M^-1 (I - S/2) M Fbar.                      */
static void mrt_collide(const double f[Q], const double feq[Q], const double Fb[Q],
                        double omega, double fstar[Q]) {
  double om2 = 8.0 * (2.0 - omega) / (8.0 - omega);
  double S[Q] = {0, omega, omega, 0, om2, 0, om2, 0, om2, omega,
                 omega, omega, omega, omega, omega, omega, om2, om2, om2};
  double m[Q], mF[Q], r[Q];
  for (int k = 0; k < Q; ++k) {
    double a = 0.0, b = 0.0;
    for (int i = 0; i < Q; ++i) {
      a += MM[k][i] * (f[i] - feq[i]);
      b += MM[k][i] * Fb[i];
    }
    m[k] = a;
    mF[k] = b;
  }
  for (int k = 0; k < Q; ++k) r[k] = -S[k] * m[k] + (1.0 - 0.5 * S[k]) * mF[k];
  for (int i = 0; i < Q; ++i) {
    double a = 0.0;
    for (int k = 0; k < Q; ++k) a += MINV[i][k] * r[k];
    fstar[i] = f[i] + a;
  }
}

/* reading: relaxation time from the harmonic mean of the kinematic
 * viscosities of the two (equal-density) fluids, nu = (tau - 1/2)/3. */
static double local_omega(const orc_config *c, double phi) {
  double nua = (c->tau_a - 0.5) / 3.0, nub = (c->tau_b - 0.5) / 3.0;
  double inv = (1.0 + phi) / (2.0 * nua) + (1.0 - phi) / (2.0 * nub);
  double tau = 0.5 + 3.0 / inv;
  return 1.0 / tau;
}

/* ------------------------------------------------------------------ masks */
/* reading: node x is inside particle p iff ((dx*dx)+(dy*dy))+(dz*dz) < R*R in
 * FP64 without fused multiply-add, with d = x - X wrapped once into (-L/2,L/2];
 * equality counts as fluid.  The static wall is as above (a tube node is solid
 * iff its squared distance from the axis is at least R_t^2).  A node inside
 * several particles belongs to the lowest index. */
static int static_wall(const orc_config *c, int x, int y, int z) {
  if (c->has_wall == 1) return z == 0;
  if (c->has_wall == 3) {
    if (z == 0) return 1;
    for (int b = 0; b < c->n_boxes; ++b) {
      const int32_t *B = c->boxes[b];
      if (x >= B[0] && x <= B[3] && y >= B[1] && y <= B[4] && z >= B[2] && z <= B[5]) return 1;
    }
    return 0;
  }
  if (c->has_wall == 2) {
    double dy = y - 0.5 * (c->ny - 1), dz = z - 0.5 * (c->nz - 1);
    return (dy * dy) + (dz * dz) >= c->tube_R * c->tube_R;
  }
  return 0;
}

/* d = p - (the point of box b's solid surface nearest to p): zero inside */
static void box_offset(const int32_t *B, const double p[3], double d[3]) {
  for (int k = 0; k < 3; ++k) {
    double lo = B[k] - 0.5, hi = B[3 + k] + 0.5;
    double q = p[k] < lo ? lo : (p[k] > hi ? hi : p[k]);
    d[k] = p[k] - q;
  }
}

static void build_mask(const orc_sim *s, uint16_t *m) {
  const orc_config *c = &s->c;
#pragma omp parallel for schedule(static)
  for (int64_t n = 0; n < s->N; ++n) {
    int x, y, z;
    ncoord(s, n, &x, &y, &z);
    m[n] = static_wall(c, x, y, z) ? 1 : 0;
  }
  for (int p = 0; p < c->n_particles; ++p) {
    const orc_particle *P = &s->P[p];
    int L[3] = {c->nx, c->ny, c->nz}, lo[3], w[3];
    for (int k = 0; k < 3; ++k) {
      lo[k] = (int)floor(P->x[k] - P->R) - 1;
      w[k] = (int)floor(P->x[k] + P->R) + 1 - lo[k] + 1;
      if (w[k] > L[k]) {
        lo[k] = 0;
        w[k] = L[k];
      }
    }
    double RR = P->R * P->R;
    for (int dz = 0; dz < w[2]; ++dz)
      for (int dy = 0; dy < w[1]; ++dy)
        for (int dx = 0; dx < w[0]; ++dx) {
          int x = wrapi(lo[0] + dx, L[0]), y = wrapi(lo[1] + dy, L[1]), z = wrapi(lo[2] + dz, L[2]);
          int64_t n = nidx(s, x, y, z);
          if (m[n] != 0) continue; /* wall, or a lower-index particle */
          double ddx = wrapd((double)x - P->x[0], (double)L[0]);
          double ddy = wrapd((double)y - P->x[1], (double)L[1]);
          double ddz = wrapd((double)z - P->x[2], (double)L[2]);
          double d2 = ((ddx * ddx) + (ddy * ddy)) + (ddz * ddz);
          if (d2 < RR) m[n] = (uint16_t)(2 + p);
        }
  }
}

/* ------------------------------------------------------- S1 .. S7 (prepare) */
static void moments_node(const orc_sim *s, int64_t n) {
  const double *a = s->fa + n * Q, *b = s->fb + n * Q;
  double ra = 0.0, rb = 0.0;
  for (int i = 0; i < Q; ++i) {
    ra += a[i];
    rb += b[i];
  }
  s->rho_a[n] = ra;
  s->rho_b[n] = rb;
  s->phi[n] = (ra - rb) / (ra + rb);
}

/* reading: the interface normal is n = G / max(|G|, eps_g).  Inside the
 * diffuse interface (|G| > eps_g, within about five nodes of its centre) this
 * is the unit normal; outside it fades continuously to zero with G, so that
 * rounding noise in a nearly uniform phi cannot turn into an O(1) normal.
 * reading: the wetting rotation turns G about the direction of its tangential
 * part G_t = G - (G.n_s) n_s; where |G_t| <= eps_gt (the interface parallel to
 * the solid, or G_t below what single precision resolves) the axis is not
 * defined and G is left unrotated.  The rotation fades in between the
 * thresholds and twice their value (see wetting_node), so that G stays a
 * continuous function of phi: a switch at a hard threshold would let a
 * last-bit difference in |G_t| or |G| turn G by up to 90 degrees.
 * The paper itself normalises G without a threshold and rotates it at every
 * boundary node of the interface.  orc_set_regularisation replaces these
 * values, so that the tests can run that plain method (thresholds near zero,
 * no fade-in) beside the regularised one and bound the difference. */
static double eps_g = 1e-4, eps_gt = 1e-4;
static int wet_blend = 1;
/* capillary direction m = n_s - (n.n_s) n is skipped below this length */
#define EPS_T 1e-3

/* S3, geometric wetting (wetting-condition eq. for n_pm).
 * reading: it is applied at every fluid node that has at least one solid
 * D3Q19 neighbour and lies in the diffuse interface, |G| > eps_g.  The solid is the lowest-index particle
 * among the neighbours, else the wall.  theta is measured through fluid a
 * (phi = +1), so with n_s the outward solid normal the target is
 * n.n_s = -cos(theta): the paper's n_+ with theta -> pi - theta.  Writing
 * n* = cos(a*) n_s + sin(a*) t^, n_+ = cos(theta) n_s + sin(theta) t^ is always
 * at least as close to n* as n_-, so n_+ is taken; if |G_t| <= eps_gt the
 * direction is left unchanged.  |G| is kept where the rotation applies in full
 * (|G_t| >= 2 eps_gt and |G| >= 2 eps_g, or always without the fade-in); below that, G moves from the
 * unrotated towards the rotated vector in proportion to the weight w. */
static void wetting_node(const orc_sim *s, int64_t n, int x, int y, int z, double G[3]) {
  int solid_p = -1, has_wall = 0;
  for (int i = 1; i < Q; ++i) {
    if (outside(s, x, i)) continue; /* an open end is no solid */
    uint16_t mv = s->mask[neighbour(s, x, y, z, i)];
    if (mv >= 2) {
      int p = mv - 2;
      if (solid_p < 0 || p < solid_p) solid_p = p;
    } else if (mv == 1) {
      has_wall = 1;
    }
  }
  if (solid_p < 0 && !has_wall) return;
  double g = norm3(G);
  if (!(g > eps_g)) return;
  double ns[3], theta;
  if (solid_p >= 0) {
    double xp[3] = {(double)x, (double)y, (double)z}, d[3];
    rel_vec(s, xp, s->P[solid_p].x, d);
    double dn = norm3(d);
    for (int k = 0; k < 3; ++k) ns[k] = d[k] / dn;
    theta = s->P[solid_p].theta_deg * M_PI / 180.0;
  } else if (s->c.has_wall == 1) {
    /* the wall plane z = 0 is below node z = 1 and, through the periodic
     * z direction, above node z = nz - 1 */
    ns[0] = ns[1] = 0.0;
    ns[2] = (z == 1) ? 1.0 : -1.0;
    theta = s->c.theta_wall_deg * M_PI / 180.0;
  } else if (s->c.has_wall == 3) {
    /* reading: the normal of the nearest point of the solid surface (the
     * plane's top face z = 1/2 or, through the periodic z direction, its
     * underside z = nz - 1/2; the boxes grown by half a node), from it to the
     * node; on ties the plane, then the lowest box index */
    double dt = z - 0.5, du = ((double)s->c.nz - 0.5) - z;
    double best = dt <= du ? dt : du;
    ns[0] = ns[1] = 0.0;
    ns[2] = dt <= du ? 1.0 : -1.0;
    const double xp[3] = {(double)x, (double)y, (double)z};
    for (int b = 0; b < s->c.n_boxes; ++b) {
      double d[3];
      box_offset(s->c.boxes[b], xp, d);
      double dn = norm3(d);
      if (dn > 0.0 && dn < best) {
        best = dn;
        for (int k = 0; k < 3; ++k) ns[k] = d[k] / dn;
      }
    }
    theta = s->c.theta_wall_deg * M_PI / 180.0;
  } else {
    /* tube: the wall's outward normal points from the node to the axis */
    double dy = y - 0.5 * (s->c.ny - 1), dz = z - 0.5 * (s->c.nz - 1);
    double r = sqrt(dy * dy + dz * dz);
    if (!(r > 0.0)) return;
    ns[0] = 0.0;
    ns[1] = -dy / r;
    ns[2] = -dz / r;
    theta = s->c.theta_wall_deg * M_PI / 180.0;
  }
  double a = dot3(G, ns);
  double t[3] = {G[0] - a * ns[0], G[1] - a * ns[1], G[2] - a * ns[2]};
  double tn = norm3(t);
  if (!(tn > eps_gt)) return;
  double ct = -cos(theta), st = sin(theta);
  /* weight of the rotated gradient: 0 at the thresholds, 1 from twice them */
  double wt = tn / eps_gt - 1.0, wg = g / eps_g - 1.0;
  double w = wet_blend ? (wt < 1.0 ? wt : 1.0) * (wg < 1.0 ? wg : 1.0) : 1.0;
  for (int k = 0; k < 3; ++k) {
    double r = g * (ct * ns[k] + st * t[k] / tn);
    G[k] = w >= 1.0 ? r : G[k] + w * (r - G[k]);
  }
}

static void prepare(orc_sim *s) {
  const orc_config *c = &s->c;
  const int64_t N = s->N;
  /* S1 */
#pragma omp parallel for schedule(static)
  for (int64_t n = 0; n < N; ++n) {
    if (s->mask[n] == 0)
      moments_node(s, n);
    else
      s->rho_a[n] = s->rho_b[n] = s->phi[n] = 0.0;
  }
  /* S2 - S4
   * reading: isotropic gradient G = 3 sum_i w_i c_i phi(x + c_i); a solid
   * neighbour, or one beyond an open end, contributes the value at x
   * (zero-gradient closure). */
#pragma omp parallel for schedule(static)
  for (int64_t n = 0; n < N; ++n) {
    double *G = s->G + 3 * n, *nr = s->nrm + 3 * n;
    G[0] = G[1] = G[2] = 0.0;
    nr[0] = nr[1] = nr[2] = 0.0;
    if (s->mask[n] != 0) continue;
    int x, y, z;
    ncoord(s, n, &x, &y, &z);
    double p0 = s->phi[n];
    for (int i = 1; i < Q; ++i) {
      int64_t m = neighbour(s, x, y, z, i);
      double pv = (!outside(s, x, i) && s->mask[m] == 0) ? s->phi[m] : p0;
      for (int k = 0; k < 3; ++k) G[k] += 3.0 * WT[i] * CV[i][k] * pv;
    }
    wetting_node(s, n, x, y, z, G);
    double g = norm3(G);
    double den = g > eps_g ? g : eps_g;
    for (int k = 0; k < 3; ++k) nr[k] = G[k] / den;
  }
  /* S5 - S7
   * reading: kappa = div n with the same stencil and closure, so that the CSF
   * force -sigma kappa G / 2 points into a drop of fluid a and produces the
   * Laplace jump 2 sigma / R.  reading: the body force acts on fluid a only,
   * weighted by its local fraction (1 + phi)/2. */
#pragma omp parallel for schedule(static)
  for (int64_t n = 0; n < N; ++n) {
    double *F = s->F + 3 * n, *u = s->u + 3 * n;
    F[0] = F[1] = F[2] = 0.0;
    u[0] = u[1] = u[2] = 0.0;
    if (s->mask[n] != 0) continue;
    int x, y, z;
    ncoord(s, n, &x, &y, &z);
    const double *n0 = s->nrm + 3 * n;
    double kappa = 0.0;
    for (int i = 1; i < Q; ++i) {
      int64_t m = neighbour(s, x, y, z, i);
      const double *nv = (!outside(s, x, i) && s->mask[m] == 0) ? s->nrm + 3 * m : n0;
      kappa += 3.0 * WT[i] * (CV[i][0] * nv[0] + CV[i][1] * nv[1] + CV[i][2] * nv[2]);
    }
    double phi = s->phi[n];
    for (int k = 0; k < 3; ++k)
      F[k] = -0.5 * c->sigma * kappa * s->G[3 * n + k] + c->body_force[k] * 0.5 * (1.0 + phi);
    double rho = s->rho_a[n] + s->rho_b[n];
    const double *a = s->fa + n * Q, *b = s->fb + n * Q;
    double j[3] = {0, 0, 0};
    for (int i = 0; i < Q; ++i)
      for (int k = 0; k < 3; ++k) j[k] += CV[i][k] * (a[i] + b[i]);
    for (int k = 0; k < 3; ++k) u[k] = (j[k] + 0.5 * F[k]) / rho;
  }
}

/* ------------------------------------------------------- S8 .. S10 collide */
static void collide_all(orc_sim *s) {
  const orc_config *c = &s->c;
#pragma omp parallel for schedule(static)
  for (int64_t n = 0; n < s->N; ++n) {
    if (s->mask[n] != 0) continue;
    double *a = s->fa + n * Q, *b = s->fb + n * Q;
    double f[Q], feq[Q], Fb[Q], fs[Q];
    double ra = s->rho_a[n], rb = s->rho_b[n], rho = ra + rb;
    for (int i = 0; i < Q; ++i) f[i] = a[i] + b[i];
    equilibrium(rho, s->u + 3 * n, feq);
    guo_source(s->u + 3 * n, s->F + 3 * n, Fb);
    mrt_collide(f, feq, Fb, local_omega(c, s->phi[n]), fs);
    /* S10 recolouring.  reading: the segregation term enters fluid a with a
     * plus sign when n points toward fluid a; the printed sign with this n
     * would mix the fluids.  Post-collision values overwrite fa, fb in place. */
    const double *nr = s->nrm + 3 * n;
    double seg = c->beta * ra * rb / rho;
    for (int i = 0; i < Q; ++i) {
      double cn = CV[i][0] * nr[0] + CV[i][1] * nr[1] + CV[i][2] * nr[2];
      a[i] = (ra / rho) * fs[i] + seg * WT[i] * cn;
      b[i] = (rb / rho) * fs[i] - seg * WT[i] * cn;
    }
  }
}

/* ------------------------------------------------------------ S11 capillary */
/* Capillary force model (capillary-force eq.).
 * reading: F = sigma * sum_j 9/2 k beta max(0, 1 - phi^2) dA sin(theta_p) m^,
 * over all points of a 2-degree polar/azimuthal grid at radius R, polar
 * angles (j + 1/2) dalpha, azimuth k dphi; phi and G at a point by trilinear
 * interpolation over the fluid corners with renormalised weights (skipped if all
 * corners are solid); m^ = normalise((n x n_s) x n) = normalise(n_s - (n.n_s) n);
 * torque arm R n_s.  (The printed formula has no sigma; a force needs it.) */
static void capillary(orc_sim *s) {
  const orc_config *c = &s->c;
  const double da = c->cap_dang_deg * M_PI / 180.0;
  const int na = (int)llround(180.0 / c->cap_dang_deg), nph = (int)llround(360.0 / c->cap_dang_deg);
  const int L[3] = {c->nx, c->ny, c->nz};
  for (int p = 0; p < c->n_particles; ++p) {
    orc_particle *P = &s->P[p];
    double Fs[3] = {0, 0, 0}, Ts[3] = {0, 0, 0};
    double pref = c->sigma * 4.5 * c->cap_k * c->beta * sin(P->theta_deg * M_PI / 180.0);
    for (int j = 0; j < na; ++j) {
      double al = (j + 0.5) * da;
      double dA = P->R * P->R * sin(al) * da * da;
      for (int k = 0; k < nph; ++k) {
        double ph = k * da;
        double sh[3] = {sin(al) * cos(ph), sin(al) * sin(ph), cos(al)};
        double xp[3];
        for (int d = 0; d < 3; ++d) xp[d] = P->x[d] + P->R * sh[d];
        int i0[3];
        double fr[3];
        for (int d = 0; d < 3; ++d) {
          double fl = floor(xp[d]);
          i0[d] = (int)fl;
          fr[d] = xp[d] - fl;
        }
        double W = 0.0, ph_i = 0.0, Gi[3] = {0, 0, 0};
        for (int cz = 0; cz < 2; ++cz)
          for (int cy = 0; cy < 2; ++cy)
            for (int cx = 0; cx < 2; ++cx) {
              int64_t m = nidx(s, wrapi(i0[0] + cx, L[0]), wrapi(i0[1] + cy, L[1]),
                               wrapi(i0[2] + cz, L[2]));
              if (s->mask[m] != 0) continue;
              double w = (cx ? fr[0] : 1.0 - fr[0]) * (cy ? fr[1] : 1.0 - fr[1]) *
                         (cz ? fr[2] : 1.0 - fr[2]);
              W += w;
              ph_i += w * s->phi[m];
              for (int d = 0; d < 3; ++d) Gi[d] += w * s->G[3 * m + d];
            }
        if (!(W > 0.0)) continue;
        ph_i /= W;
        for (int d = 0; d < 3; ++d) Gi[d] /= W;
        double wgt = 1.0 - ph_i * ph_i;
        if (!(wgt > 0.0)) continue;
        double g = norm3(Gi);
        if (!(g > eps_g)) continue;
        double nn[3] = {Gi[0] / g, Gi[1] / g, Gi[2] / g};
        double a = dot3(nn, sh);
        double mv[3] = {sh[0] - a * nn[0], sh[1] - a * nn[1], sh[2] - a * nn[2]};
        double mn = norm3(mv);
        if (!(mn > EPS_T)) continue;
        double dF[3], arm[3] = {P->R * sh[0], P->R * sh[1], P->R * sh[2]}, dT[3];
        for (int d = 0; d < 3; ++d) dF[d] = pref * wgt * dA * mv[d] / mn;
        cross3(arm, dF, dT);
        for (int d = 0; d < 3; ++d) {
          Fs[d] += dF[d];
          Ts[d] += dT[d];
        }
      }
    }
    for (int d = 0; d < 3; ++d) {
      P->F_cap[d] = Fs[d];
      P->T_cap[d] = Ts[d];
    }
  }
}

/* ------------------------------------------------- S12 + S13 stream, bounce */
/* Half-way bounce-back with a moving wall (bounce-back eqs.).
 * reading: the reflected population is f_opp(x) = f*_i(x) + 2 w_i rho^{a,b}(x)
 * (c_opp . u_w)/c_s^2 (the printed factor 6 w_i ... / c_s^2 would triple the
 * moving-wall term), with u_w taken at the link midpoint x + c_i/2.
 * Momentum exchange (hydrodynamic force eqs.): per link to particle p,
 * dP = (c_i - u_w) f*_i(x) - (c_opp - u_w) f_opp(x) is the momentum given to
 * the particle; torque arm x + c_i/2 - X_p. */
static void stream_bounce(orc_sim *s) {
  const int64_t N = s->N;
#pragma omp parallel for schedule(static)
  for (int64_t n = 0; n < N; ++n) {
    if (s->mask[n] != 0) continue;
    int x, y, z;
    ncoord(s, n, &x, &y, &z);
    const double *a = s->fa + n * Q, *b = s->fb + n * Q;
    double ra = s->rho_a[n], rb = s->rho_b[n];
    s->fa_new[n * Q] = a[0];
    s->fb_new[n * Q] = b[0];
    for (int i = 1; i < Q; ++i) {
      if (outside(s, x, i)) {
        /* Anti-bounce-back at the pressure boundary (pressure inlet/outlet
         * eq.): f_opp(x) = -f*_i(x) + 2 w_i rho_w [1 + (c_i.u_w)^2/(2 cs^4)
         * - u_w^2/(2 cs^2)] with p_w = cs^2 rho_w.  reading: u_w is the
         * velocity of the boundary node itself; the rule is applied to each
         * fluid with its share rho_w (1 +- phi)/2 of rho_w, phi that of the
         * boundary node (the colour leaving and entering is the node's). */
        int o = OPPD[i];
        double rw = (x + CV[i][0] < 0) ? s->c.rho_in : s->c.rho_out;
        const double *uw = s->u + 3 * n;
        double cu = CV[i][0] * uw[0] + CV[i][1] * uw[1] + CV[i][2] * uw[2];
        double e = 2.0 * WT[i] * rw * (1.0 + 4.5 * cu * cu - 1.5 * dot3(uw, uw));
        double ph = s->phi[n];
        s->fa_new[n * Q + o] = -a[i] + 0.5 * (1.0 + ph) * e;
        s->fb_new[n * Q + o] = -b[i] + 0.5 * (1.0 - ph) * e;
        continue;
      }
      int64_t m = neighbour(s, x, y, z, i);
      uint16_t mv = s->mask[m];
      if (mv == 0) {
        s->fa_new[m * Q + i] = a[i];
        s->fb_new[m * Q + i] = b[i];
      } else {
        int o = OPPD[i];
        double uw[3] = {0, 0, 0};
        if (mv >= 2) {
          double xw[3] = {x + 0.5 * CV[i][0], y + 0.5 * CV[i][1], z + 0.5 * CV[i][2]};
          wall_velocity(s, mv - 2, xw, uw);
        }
        double cu = CV[o][0] * uw[0] + CV[o][1] * uw[1] + CV[o][2] * uw[2];
        s->fa_new[n * Q + o] = a[i] + 6.0 * WT[i] * ra * cu;
        s->fb_new[n * Q + o] = b[i] + 6.0 * WT[i] * rb * cu;
      }
    }
  }
  /* S13, serial in node order */
  for (int p = 0; p < s->c.n_particles; ++p)
    for (int k = 0; k < 3; ++k) s->P[p].F_hyd[k] = s->P[p].T_hyd[k] = 0.0;
  for (int64_t n = 0; n < N; ++n) {
    if (s->mask[n] != 0) continue;
    int x, y, z;
    ncoord(s, n, &x, &y, &z);
    for (int i = 1; i < Q; ++i) {
      if (outside(s, x, i)) continue;
      uint16_t mv = s->mask[neighbour(s, x, y, z, i)];
      if (mv < 2) continue;
      int p = mv - 2, o = OPPD[i];
      double xw[3] = {x + 0.5 * CV[i][0], y + 0.5 * CV[i][1], z + 0.5 * CV[i][2]};
      double uw[3], arm[3], dP[3], dT[3];
      wall_velocity(s, p, xw, uw);
      double fin = s->fa[n * Q + i] + s->fb[n * Q + i];
      double fout = s->fa_new[n * Q + o] + s->fb_new[n * Q + o];
      for (int k = 0; k < 3; ++k) dP[k] = (CV[i][k] - uw[k]) * fin - (CV[o][k] - uw[k]) * fout;
      rel_vec(s, xw, s->P[p].x, arm);
      cross3(arm, dP, dT);
      for (int k = 0; k < 3; ++k) {
        s->P[p].F_hyd[k] += dP[k];
        s->P[p].T_hyd[k] += dT[k];
      }
    }
  }
  double *t = s->fa;
  s->fa = s->fa_new;
  s->fa_new = t;
  t = s->fb;
  s->fb = s->fb_new;
  s->fb_new = t;
}

/* ------------------------------------------------------------------ S14 DEM */
static double pmass(const orc_particle *P) { return P->rho_p * 4.0 / 3.0 * M_PI * P->R * P->R * P->R; }

/* Collision duration t_c = pi / omega_c (collision-duration eq.) for the
 * lightest contact pair; reading: the DEM runs n_sub = ceil(45 / t_c) sub-steps
 * per lattice step, so that its step is about t_c / 45 at every particle size. */
static int dem_substeps(const orc_sim *s, int *ok) {
  const orc_config *c = &s->c;
  *ok = 1;
  if (c->n_particles == 0) return 1;
  double m1 = INFINITY, m2 = INFINITY;
  for (int p = 0; p < c->n_particles; ++p) {
    double m = pmass(&s->P[p]);
    if (m < m1) {
      m2 = m1;
      m1 = m;
    } else if (m < m2)
      m2 = m;
  }
  double meff = (c->n_particles >= 2) ? m1 * m2 / (m1 + m2) : m1;
  double eta = c->gn / (2.0 * meff);
  double w2 = c->kn / meff - eta * eta;
  if (!(w2 > 0.0)) {
    *ok = 0;
    return 1;
  }
  double tc = M_PI / sqrt(w2);
  int ns = (int)ceil(45.0 / tc);
  return ns < 1 ? 1 : ns;
}

static orc_contact *find_slot(orc_sim *s, int i, int partner, int create) {
  orc_contact *t = s->ct + (int64_t)i * MAXC;
  for (int k = 0; k < MAXC; ++k)
    if (t[k].partner == partner) return &t[k];
  if (!create) return NULL;
  for (int k = 0; k < MAXC; ++k)
    if (t[k].partner == -100) {
      memset(&t[k], 0, sizeof(orc_contact));
      t[k].partner = partner;
      return &t[k];
    }
  s->status = -5; /* contact table full */
  return NULL;
}

/* Spring with a Coulomb cap (sliding-friction eqs.; rolling friction uses the
 * same switch on the rolling velocity). */
static void capped_spring(double k, double gam, double cap, double xi[3], const double v[3],
                          double dt, double Fout[3]) {
  double F0[3];
  for (int d = 0; d < 3; ++d) F0[d] = -k * xi[d] - gam * v[d];
  double f0 = norm3(F0);
  if (f0 <= cap) {
    for (int d = 0; d < 3; ++d) {
      Fout[d] = F0[d];
      xi[d] += v[d] * dt;
    }
  } else {
    for (int d = 0; d < 3; ++d) Fout[d] = cap * F0[d] / f0;
    for (int d = 0; d < 3; ++d) xi[d] = (k > 0.0) ? -(Fout[d] + gam * v[d]) / k : 0.0;
  }
}

/* Contact of particle i with a partner, after Luding (2008) as the paper
 * cites it.  nh points from the partner to particle i; vj, wj, Xj are the
 * partner's velocity, spin and centre (wall: zero, zero, unused); Rcj is the
 * partner's mechanical radius (wall: 0).  Returns 1 if the contact is active. */
static int contact(orc_sim *s, int i, int partner, double delta, const double nh[3],
                   const double vi[3], const double wi[3], const double vj[3],
                   const double wj[3], double Rci, double Rcj, const double armj_rel[3],
                   double mu, double mur, double dt, double Fo[3], double To[3]) {
  const orc_config *c = &s->c;
  if (!(delta > 0.0)) {
    orc_contact *sl = find_slot(s, i, partner, 0);
    if (sl) sl->partner = -100;
    return 0;
  }
  orc_contact *sl = find_slot(s, i, partner, 1);
  if (!sl) return 0;
  double vrel[3];
  for (int d = 0; d < 3; ++d) vrel[d] = vi[d] - vj[d];
  double ddot = -dot3(vrel, nh);
  /* reading: F_n = k_n delta + gamma_n d(delta)/dt, signed, along nh */
  double Fn = c->kn * delta + c->gn * ddot;
  /* contact point relative to particle i's centre, and to the partner's */
  double ri[3], rj[3], t1[3], t2[3], vc[3];
  for (int d = 0; d < 3; ++d) ri[d] = -(Rci - 0.5 * delta) * nh[d];
  for (int d = 0; d < 3; ++d) rj[d] = ri[d] + armj_rel[d];
  cross3(wi, ri, t1);
  cross3(wj, rj, t2);
  for (int d = 0; d < 3; ++d) vc[d] = vrel[d] + t1[d] - t2[d];
  double vn = dot3(vc, nh), vt[3];
  for (int d = 0; d < 3; ++d) vt[d] = vc[d] - vn * nh[d];
  /* springs are kept in the tangent plane */
  double xn = dot3(sl->xt, nh);
  for (int d = 0; d < 3; ++d) sl->xt[d] -= xn * nh[d];
  xn = dot3(sl->xr, nh);
  for (int d = 0; d < 3; ++d) sl->xr[d] -= xn * nh[d];
  double Fcap = mu * (Fn > 0.0 ? Fn : 0.0);
  double Ft[3];
  capped_spring(c->kt, c->gt, Fcap, sl->xt, vt, dt, Ft);
  /* rolling: v_r = -a' (n x w_i - n x w_j), torque a' n x F_r, no force */
  double ap = (Rcj > 0.0) ? Rci * Rcj / (Rci + Rcj) : Rci;
  double nwi[3], nwj[3], vr[3], Fr[3];
  cross3(nh, wi, nwi);
  cross3(nh, wj, nwj);
  for (int d = 0; d < 3; ++d) vr[d] = -ap * (nwi[d] - nwj[d]);
  double Rcap = mur * (Fn > 0.0 ? Fn : 0.0);
  capped_spring(c->kr, c->gr, Rcap, sl->xr, vr, dt, Fr);
  double Tt[3], Tr[3];
  cross3(ri, Ft, Tt);
  cross3(nh, Fr, Tr);
  for (int d = 0; d < 3; ++d) {
    Fo[d] = Fn * nh[d] + Ft[d];
    To[d] = Tt[d] + ap * Tr[d];
  }
  return 1;
}

/* contact force and torque on every particle at the current positions, with
 * predicted velocities vp, wp */
static void contacts_all(orc_sim *s, const double *vp, const double *wp, double dt, double *Fc,
                         double *Tc) {
  const orc_config *c = &s->c;
  const int np = c->n_particles;
  const double zero[3] = {0, 0, 0};
  for (int i = 0; i < np; ++i) {
    orc_particle *P = &s->P[i];
    double Rci = P->R + c->delta_R;
    double Fsum[3] = {0, 0, 0}, Tsum[3] = {0, 0, 0}, Fo[3], To[3];
    if (c->has_wall == 2) {
      /* reading: the tube's surface is the cylinder r = R_t (a node is solid
       * from r >= R_t on); the contact normal points from the wall to the
       * centre, towards the axis */
      double dy = P->x[1] - 0.5 * (c->ny - 1), dz = P->x[2] - 0.5 * (c->nz - 1);
      double r = sqrt(dy * dy + dz * dz);
      double nw[3] = {0.0, r > 0.0 ? -dy / r : 0.0, r > 0.0 ? -dz / r : 0.0};
      double dw = Rci - (c->tube_R - r);
      if (contact(s, i, -1, dw, nw, vp + 3 * i, wp + 3 * i, zero, zero, Rci, 0.0, zero, P->mu_s,
                  P->mu_r, dt, Fo, To))
        for (int d = 0; d < 3; ++d) {
          Fsum[d] += Fo[d];
          Tsum[d] += To[d];
        }
    } else if (c->has_wall) {
      double nb[3] = {0, 0, 1}, nt[3] = {0, 0, -1};
      double db = Rci - (P->x[2] - 0.5);
      if (contact(s, i, -1, db, nb, vp + 3 * i, wp + 3 * i, zero, zero, Rci, 0.0, zero, P->mu_s,
                  P->mu_r, dt, Fo, To))
        for (int d = 0; d < 3; ++d) {
          Fsum[d] += Fo[d];
          Tsum[d] += To[d];
        }
      double dtp = Rci - (((double)c->nz - 0.5) - P->x[2]);
      if (contact(s, i, -2, dtp, nt, vp + 3 * i, wp + 3 * i, zero, zero, Rci, 0.0, zero, P->mu_s,
                  P->mu_r, dt, Fo, To))
        for (int d = 0; d < 3; ++d) {
          Fsum[d] += Fo[d];
          Tsum[d] += To[d];
        }
      /* reading: each box of a textured wall is a contact partner of its own
       * (id -3 - b) at the nearest point of its grown surface, the normal from
       * there to the centre; no contact while the centre is inside it */
      for (int b = 0; c->has_wall == 3 && b < c->n_boxes; ++b) {
        double d[3], nbx[3] = {0, 0, 0};
        box_offset(c->boxes[b], P->x, d);
        double dn = norm3(d);
        if (dn > 0.0)
          for (int k = 0; k < 3; ++k) nbx[k] = d[k] / dn;
        double db2 = dn > 0.0 ? Rci - dn : -1.0;
        if (contact(s, i, -3 - b, db2, nbx, vp + 3 * i, wp + 3 * i, zero, zero, Rci, 0.0, zero,
                    P->mu_s, P->mu_r, dt, Fo, To))
          for (int k = 0; k < 3; ++k) {
            Fsum[k] += Fo[k];
            Tsum[k] += To[k];
          }
      }
    }
    for (int j = 0; j < np; ++j) {
      if (j == i) continue;
      const orc_particle *Pj = &s->P[j];
      double Rcj = Pj->R + c->delta_R, dx[3];
      rel_vec(s, P->x, Pj->x, dx); /* X_i - X_j, min image */
      double dist = norm3(dx);
      double delta = Rci + Rcj - dist;
      double nh[3] = {0, 0, 0};
      if (dist > 0.0)
        for (int d = 0; d < 3; ++d) nh[d] = dx[d] / dist;
      /* partner arm: contact point relative to X_j = r_i + (X_i - X_j) */
      /* reading: pair friction coefficients are the means of the two particles' */
      if (contact(s, i, j, delta, nh, vp + 3 * i, wp + 3 * i, vp + 3 * j, wp + 3 * j, Rci, Rcj, dx,
                  0.5 * (P->mu_s + Pj->mu_s), 0.5 * (P->mu_r + Pj->mu_r), dt, Fo, To))
        for (int d = 0; d < 3; ++d) {
          Fsum[d] += Fo[d];
          Tsum[d] += To[d];
        }
    }
    for (int d = 0; d < 3; ++d) {
      Fc[3 * i + d] = Fsum[d];
      Tc[3 * i + d] = Tsum[d];
    }
  }
}

static void quat_rotate(double q[4], const double th[3]) {
  double a = norm3(th);
  if (!(a > 0.0)) return;
  double h = 0.5 * a, sh = sin(h) / a;
  double dq[4] = {cos(h), th[0] * sh, th[1] * sh, th[2] * sh};
  double r[4] = {dq[0] * q[0] - dq[1] * q[1] - dq[2] * q[2] - dq[3] * q[3],
                 dq[0] * q[1] + dq[1] * q[0] + dq[2] * q[3] - dq[3] * q[2],
                 dq[0] * q[2] - dq[1] * q[3] + dq[2] * q[0] + dq[3] * q[1],
                 dq[0] * q[3] + dq[1] * q[2] - dq[2] * q[1] + dq[3] * q[0]};
  double nq = sqrt(r[0] * r[0] + r[1] * r[1] + r[2] * r[2] + r[3] * r[3]);
  for (int k = 0; k < 4; ++k) q[k] = r[k] / nq;
}

/* Newton-Euler with velocity Verlet (translational and rotational Newton eqs.;
 * reading of "average of the forces in the previous and current step"): per
 * sub-step, X += V dt + a_old dt^2/2, contacts at the new X with predicted
 * velocities V + a_old dt, then V += (a_old + a_new) dt / 2.  The fluid force and
 * torque (hydrodynamic + capillary) are held over the sub-steps; gravity is the
 * downward force g_p.  Kinematic particles keep V, Omega. */
static void dem(orc_sim *s, const double *Fext) {
  const orc_config *c = &s->c;
  const int np = c->n_particles;
  if (np == 0) return;
  const double dt = 1.0 / s->n_sub;
  double *vp = malloc(sizeof(double) * 3 * np), *wp = malloc(sizeof(double) * 3 * np);
  double *Fc = malloc(sizeof(double) * 3 * np), *Tc = malloc(sizeof(double) * 3 * np);
  double *Ff = malloc(sizeof(double) * 3 * np), *Tf = malloc(sizeof(double) * 3 * np);
  double *ao = malloc(sizeof(double) * 3 * np), *bo = malloc(sizeof(double) * 3 * np);
  double *Facc = calloc(3 * np, sizeof(double)), *Tacc = calloc(3 * np, sizeof(double));
  /* reading of the Verlet passage ("an average of the forces/torques in the
   * previous and current time step"): the fluid force and torque (momentum
   * exchange + capillary) applied over this lattice step are the means of the
   * values computed at this and at the previous lattice step. */
  for (int i = 0; i < np; ++i) {
    orc_particle *P = &s->P[i];
    for (int d = 0; d < 3; ++d) {
      double fc = P->F_hyd[d] + P->F_cap[d], tc = P->T_hyd[d] + P->T_cap[d];
      double fp = s->have_prev ? s->Ff_prev[3 * i + d] : fc;
      double tp = s->have_prev ? s->Tf_prev[3 * i + d] : tc;
      Ff[3 * i + d] = 0.5 * (fc + fp) + (Fext ? Fext[3 * i + d] : 0.0);
      Tf[3 * i + d] = 0.5 * (tc + tp);
      s->Ff_prev[3 * i + d] = fc;
      s->Tf_prev[3 * i + d] = tc;
    }
    Ff[3 * i + 2] -= P->g_p;
  }
  s->have_prev = 1;
  for (int sub = 0; sub < s->n_sub; ++sub) {
    for (int i = 0; i < np; ++i) {
      orc_particle *P = &s->P[i];
      double m = pmass(P), I = 0.4 * m * P->R * P->R;
      double th[3];
      for (int d = 0; d < 3; ++d) {
        if (P->kinematic) {
          ao[3 * i + d] = bo[3 * i + d] = 0.0;
        } else {
          ao[3 * i + d] = (Ff[3 * i + d] + s->Fc_prev[3 * i + d]) / m;
          bo[3 * i + d] = (Tf[3 * i + d] + s->Tc_prev[3 * i + d]) / I;
        }
        P->x[d] += P->v[d] * dt + 0.5 * ao[3 * i + d] * dt * dt;
        th[d] = P->w[d] * dt + 0.5 * bo[3 * i + d] * dt * dt;
        vp[3 * i + d] = P->v[d] + ao[3 * i + d] * dt;
        wp[3 * i + d] = P->w[d] + bo[3 * i + d] * dt;
      }
      quat_rotate(P->q, th);
      /* periodic axes keep the centre in [0, L) */
      double L[3] = {(double)c->nx, (double)c->ny, (double)c->nz};
      for (int d = 0; d < 3; ++d) {
        if (d == 2 && c->has_wall) continue;
        if (d == 0 && c->open_x) continue;
        if (P->x[d] >= L[d])
          P->x[d] -= L[d];
        else if (P->x[d] < 0.0)
          P->x[d] += L[d];
      }
    }
    contacts_all(s, vp, wp, dt, Fc, Tc);
    for (int i = 0; i < np; ++i) {
      orc_particle *P = &s->P[i];
      double m = pmass(P), I = 0.4 * m * P->R * P->R;
      for (int d = 0; d < 3; ++d) {
        if (!P->kinematic) {
          double an = (Ff[3 * i + d] + Fc[3 * i + d]) / m;
          double bn = (Tf[3 * i + d] + Tc[3 * i + d]) / I;
          P->v[d] += 0.5 * (ao[3 * i + d] + an) * dt;
          P->w[d] += 0.5 * (bo[3 * i + d] + bn) * dt;
        }
        s->Fc_prev[3 * i + d] = Fc[3 * i + d];
        s->Tc_prev[3 * i + d] = Tc[3 * i + d];
        Facc[3 * i + d] += Fc[3 * i + d];
        Tacc[3 * i + d] += Tc[3 * i + d];
      }
    }
  }
  for (int i = 0; i < np; ++i)
    for (int d = 0; d < 3; ++d) {
      s->P[i].F_con[d] = Facc[3 * i + d] / s->n_sub;
      s->P[i].T_con[d] = Tacc[3 * i + d] / s->n_sub;
    }
  /* a particle must keep R + 4 nodes from an open end: the lattice work
   * around it (mask box, links, capillary points, refill) never reaches the
   * boundary planes then */
  if (c->open_x)
    for (int i = 0; i < np; ++i) {
      const orc_particle *P = &s->P[i];
      if (P->x[0] < P->R + 4.0 || P->x[0] > (double)(c->nx - 1) - P->R - 4.0) s->status = -5;
    }
  free(vp); free(wp); free(Fc); free(Tc); free(Ff); free(Tf); free(ao); free(bo);
  free(Facc); free(Tacc);
}

/* --------------------------------------------------- S15 mask and refilling */
/* Refilling of fresh fluid nodes (refilling eqs.).
 * reading: the densities are the means over the D3Q19 neighbours that are
 * fluid in the new mask and not fresh, of the moments of their post-stream
 * populations; if there is none, rho0/2 each.  u is the surface velocity of the
 * particle that uncovered the node, at the node, after the DEM update. */
static void update_mask_and_refill(orc_sim *s) {
  build_mask(s, s->mask_new);
  const int64_t N = s->N;
  /* fresh nodes: particle before, fluid now */
  int64_t nf = 0;
  for (int64_t n = 0; n < N; ++n)
    if (s->mask[n] >= 2 && s->mask_new[n] == 0) ++nf;
  int64_t *fl = malloc(sizeof(int64_t) * (nf ? nf : 1));
  int *fo = malloc(sizeof(int) * (nf ? nf : 1));
  nf = 0;
  for (int64_t n = 0; n < N; ++n)
    if (s->mask[n] >= 2 && s->mask_new[n] == 0) {
      fl[nf] = n;
      fo[nf] = s->mask[n] - 2;
      ++nf;
    }
  s->n_fresh = nf;
  double *fa_r = malloc(sizeof(double) * Q * (nf ? nf : 1));
  double *fb_r = malloc(sizeof(double) * Q * (nf ? nf : 1));
  for (int64_t k = 0; k < nf; ++k) {
    int64_t n = fl[k];
    int x, y, z;
    ncoord(s, n, &x, &y, &z);
    double sa = 0.0, sb = 0.0;
    int cnt = 0;
    for (int i = 1; i < Q; ++i) {
      if (outside(s, x, i)) continue;
      int64_t m = neighbour(s, x, y, z, i);
      if (s->mask_new[m] != 0) continue;
      if (s->mask[m] >= 2) continue; /* also fresh */
      double ra = 0.0, rb = 0.0;
      for (int q = 0; q < Q; ++q) {
        ra += s->fa[m * Q + q];
        rb += s->fb[m * Q + q];
      }
      sa += ra;
      sb += rb;
      ++cnt;
    }
    double rba = cnt ? sa / cnt : 0.5 * s->c.rho0, rbb = cnt ? sb / cnt : 0.5 * s->c.rho0;
    double xp[3] = {(double)x, (double)y, (double)z}, uw[3];
    wall_velocity(s, fo[k], xp, uw);
    equilibrium(rba, uw, fa_r + Q * k);
    equilibrium(rbb, uw, fb_r + Q * k);
  }
  for (int64_t k = 0; k < nf; ++k)
    for (int q = 0; q < Q; ++q) {
      s->fa[fl[k] * Q + q] = fa_r[Q * k + q];
      s->fb[fl[k] * Q + q] = fb_r[Q * k + q];
    }
  /* covered nodes (fluid before, solid now) lose their populations */
  for (int64_t n = 0; n < N; ++n)
    if (s->mask[n] == 0 && s->mask_new[n] != 0)
      for (int q = 0; q < Q; ++q) s->fa[n * Q + q] = s->fb[n * Q + q] = 0.0;
  uint16_t *t = s->mask;
  s->mask = s->mask_new;
  s->mask_new = t;
  free(fl); free(fo); free(fa_r); free(fb_r);
}

/* ------------------------------------------------------------ public C API */
void orc_destroy(orc_sim *s);

orc_sim *orc_create(const orc_config *cfg, const float *phi0, const orc_particle *parts) {
  build_tables();
  if (cfg->nx < 1 || cfg->ny < 1 || cfg->nz < 3) return NULL;
  if (cfg->has_wall < 0 || cfg->has_wall > 3) return NULL;
  if (cfg->has_wall == 3) {
    if (cfg->n_boxes < 0 || cfg->n_boxes > 8 || cfg->open_x) return NULL;
    const int L[3] = {cfg->nx, cfg->ny, cfg->nz};
    for (int b = 0; b < cfg->n_boxes; ++b)
      for (int k = 0; k < 3; ++k)
        if (cfg->boxes[b][k] < 0 || cfg->boxes[b][k] > cfg->boxes[b][3 + k] ||
            cfg->boxes[b][3 + k] >= L[k])
          return NULL;
  }
  if (cfg->has_wall == 2 && !(cfg->tube_R > 0.0)) return NULL;
  if (cfg->open_x && (!(cfg->rho_in > 0.0) || !(cfg->rho_out > 0.0) || cfg->nx < 2)) return NULL;
  orc_sim *s = calloc(1, sizeof(orc_sim));
  s->c = *cfg;
  s->N = (int64_t)cfg->nx * cfg->ny * cfg->nz;
  const int64_t N = s->N;
  s->fa = calloc(N * Q, sizeof(double));
  s->fb = calloc(N * Q, sizeof(double));
  s->fa_new = calloc(N * Q, sizeof(double));
  s->fb_new = calloc(N * Q, sizeof(double));
  s->mask = calloc(N, sizeof(uint16_t));
  s->mask_new = calloc(N, sizeof(uint16_t));
  s->rho_a = calloc(N, sizeof(double));
  s->rho_b = calloc(N, sizeof(double));
  s->phi = calloc(N, sizeof(double));
  s->G = calloc(3 * N, sizeof(double));
  s->nrm = calloc(3 * N, sizeof(double));
  s->F = calloc(3 * N, sizeof(double));
  s->u = calloc(3 * N, sizeof(double));
  int np = cfg->n_particles;
  s->P = calloc(np ? np : 1, sizeof(orc_particle));
  s->ct = calloc((np ? np : 1) * MAXC, sizeof(orc_contact));
  s->Fc_prev = calloc(3 * (np ? np : 1), sizeof(double));
  s->Tc_prev = calloc(3 * (np ? np : 1), sizeof(double));
  s->Ff_prev = calloc(3 * (np ? np : 1), sizeof(double));
  s->Tf_prev = calloc(3 * (np ? np : 1), sizeof(double));
  if (!s->fa || !s->fb || !s->fa_new || !s->fb_new || !s->G || !s->u) {
    orc_destroy(s);
    return NULL;
  }
  for (int p = 0; p < np; ++p) s->P[p] = parts[p];
  for (int64_t k = 0; k < (int64_t)np * MAXC; ++k) s->ct[k].partner = -100;
  int ok;
  s->n_sub = dem_substeps(s, &ok);
  if (!ok) {
    orc_destroy(s);
    return NULL;
  }
  build_mask(s, s->mask);
  /* initial state at rest: fa = w rho0 (1 + phi0)/2, fb = w rho0 (1 - phi0)/2 */
#pragma omp parallel for schedule(static)
  for (int64_t n = 0; n < N; ++n) {
    if (s->mask[n] != 0) continue;
    double p0 = phi0 ? (double)phi0[n] : 1.0;
    for (int i = 0; i < Q; ++i) {
      s->fa[n * Q + i] = WT[i] * cfg->rho0 * 0.5 * (1.0 + p0);
      s->fb[n * Q + i] = WT[i] * cfg->rho0 * 0.5 * (1.0 - p0);
    }
  }
  return s;
}

void orc_destroy(orc_sim *s) {
  if (!s) return;
  free(s->fa); free(s->fb); free(s->fa_new); free(s->fb_new);
  free(s->mask); free(s->mask_new);
  free(s->rho_a); free(s->rho_b); free(s->phi);
  free(s->G); free(s->nrm); free(s->F); free(s->u);
  free(s->P); free(s->ct); free(s->Fc_prev); free(s->Tc_prev); free(s->Ff_prev); free(s->Tf_prev);
  free(s);
}

/* instability check: NaN, rho <= 0 or |u| > 0.3 at a fluid node */
static int unstable(const orc_sim *s) {
  int bad = 0;
#pragma omp parallel for schedule(static) reduction(| : bad)
  for (int64_t n = 0; n < s->N; ++n) {
    if (s->mask[n] != 0) continue;
    double rho = s->rho_a[n] + s->rho_b[n];
    const double *u = s->u + 3 * n;
    double uu = u[0] * u[0] + u[1] * u[1] + u[2] * u[2];
    if (!(rho > 0.0) || !(uu <= 0.09)) bad = 1;
  }
  return bad;
}

/* One step per iteration; returns 0, or -4 if the flow became unstable, -5 if
 * a contact table overflowed or a particle came within R + 4 of an open end. */
int orc_step(orc_sim *s, int nsteps) {
  for (int t = 0; t < nsteps; ++t) {
    prepare(s);            /* S1 - S7 */
    if (unstable(s)) return -4;
    collide_all(s);        /* S8 - S10 (in place) */
    capillary(s);          /* S11 from phi, G of this step */
    stream_bounce(s);      /* S12 - S13 */
    dem(s, NULL);          /* S14 */
    update_mask_and_refill(s); /* S15 */
    if (s->status) return s->status;
  }
  return 0;
}

/* DEM only (no fluid): nsteps lattice steps with an extra constant force per
 * particle (3 doubles each, may be NULL) and zero fluid force. */
int orc_dem_run(orc_sim *s, int nsteps, const double *Fext) {
  for (int t = 0; t < nsteps; ++t) {
    for (int p = 0; p < s->c.n_particles; ++p)
      for (int k = 0; k < 3; ++k)
        s->P[p].F_hyd[k] = s->P[p].T_hyd[k] = s->P[p].F_cap[k] = s->P[p].T_cap[k] = 0.0;
    dem(s, Fext);
    if (s->status) return s->status;
  }
  return 0;
}

int orc_n_sub(const orc_sim *s) { return s->n_sub; }
int64_t orc_n_fresh(const orc_sim *s) { return s->n_fresh; }

/* Fields of the current state: rho, u (3 planes, x-fastest), phi, mask.  Solid
 * nodes report rho = phi = 0 and u = u_w (0 on the wall).  Any pointer may be
 * NULL.  The velocity includes half the force (velocity eq.). */
void orc_fields(orc_sim *s, double *rho, double *u, double *phi, uint16_t *mask) {
  prepare(s);
  const int64_t N = s->N;
  for (int64_t n = 0; n < N; ++n) {
    uint16_t mv = s->mask[n];
    if (rho) rho[n] = (mv == 0) ? s->rho_a[n] + s->rho_b[n] : 0.0;
    if (phi) phi[n] = (mv == 0) ? s->phi[n] : 0.0;
    if (mask) mask[n] = mv;
    if (u) {
      double uw[3] = {0, 0, 0};
      if (mv == 0) {
        for (int k = 0; k < 3; ++k) uw[k] = s->u[3 * n + k];
      } else if (mv >= 2) {
        int x, y, z;
        ncoord(s, n, &x, &y, &z);
        double xp[3] = {(double)x, (double)y, (double)z};
        wall_velocity(s, mv - 2, xp, uw);
      }
      for (int k = 0; k < 3; ++k) u[k * N + n] = uw[k];
    }
  }
}

/* colour gradient after wetting and force of the current state (N*3 each) */
void orc_grad_force(orc_sim *s, double *G, double *F) {
  prepare(s);
  if (G) memcpy(G, s->G, sizeof(double) * 3 * s->N);
  if (F) memcpy(F, s->F, sizeof(double) * 3 * s->N);
}

/* populations, as N*19 arrays (node-major) */
void orc_get_pops(const orc_sim *s, double *fa, double *fb) {
  if (fa) memcpy(fa, s->fa, sizeof(double) * Q * s->N);
  if (fb) memcpy(fb, s->fb, sizeof(double) * Q * s->N);
}
void orc_set_pops(orc_sim *s, const double *fa, const double *fb) {
  if (fa) memcpy(s->fa, fa, sizeof(double) * Q * s->N);
  if (fb) memcpy(s->fb, fb, sizeof(double) * Q * s->N);
}

void orc_get_particles(const orc_sim *s, orc_particle *out) {
  memcpy(out, s->P, sizeof(orc_particle) * s->c.n_particles);
}
/* replace the particle state; the mask is rebuilt and fresh nodes refilled */
void orc_set_particles(orc_sim *s, const orc_particle *in) {
  memcpy(s->P, in, sizeof(orc_particle) * s->c.n_particles);
  update_mask_and_refill(s);
}

/* Links (x fluid, x + c_i inside particle p), packed as (node << 5) | dir,
 * in particle, node, direction order; writes up to max entries and returns the
 * total count.  pid receives the particle of each link (may be NULL). */
int64_t orc_links(const orc_sim *s, uint32_t *out, int32_t *pid, int64_t max) {
  int64_t cnt = 0;
  for (int p = 0; p < s->c.n_particles; ++p)
    for (int64_t n = 0; n < s->N; ++n) {
      if (s->mask[n] != 0) continue;
      int x, y, z;
      ncoord(s, n, &x, &y, &z);
      for (int i = 1; i < Q; ++i)
        if (s->mask[neighbour(s, x, y, z, i)] == 2 + p) {
          if (cnt < max) {
            out[cnt] = (uint32_t)((n << 5) | i);
            if (pid) pid[cnt] = p;
          }
          ++cnt;
        }
    }
  return cnt;
}

/* Sensitivity probe (not part of the method): round every colour population's
 * departure from its rest value w_i rho0 / 2 to single precision, in place, as
 * a store of the state in FP32 would; tests use it to measure how far the
 * method's trajectory moves under storage rounding alone. */
void orc_round_state_f32(orc_sim *s) {
  const double h = 0.5 * s->c.rho0;
#pragma omp parallel for schedule(static)
  for (int64_t n = 0; n < s->N; ++n) {
    if (s->mask[n] != 0) continue;
    for (int i = 0; i < Q; ++i) {
      const double r = WT[i] * h;
      s->fa[n * Q + i] = r + (double)(float)(s->fa[n * Q + i] - r);
      s->fb[n * Q + i] = r + (double)(float)(s->fb[n * Q + i] - r);
    }
  }
}

/* Round x to the nearest binary16 value (round half to even), subnormals
 * included; |x| stays far below the binary16 range here. */
static double round_binary16(double x) {
  if (x == 0.0 || !isfinite(x)) return x;
  const double sub = ldexp(1.0, -24); /* spacing of the subnormals */
  if (fabs(x) < ldexp(1.0, -14)) return nearbyint(x / sub) * sub;
  int e;
  const double m = frexp(x, &e); /* x = m 2^e, 0.5 <= |m| < 1 */
  return ldexp(nearbyint(ldexp(m, 11)), e - 11);
}

/* Sensitivity probe, not the method: the total population of every fluid node
 * rounded as a 16-bit store relative to the node's density would round it,
 * h = (f - w_i rho)/(w_i rho0) to binary16, the colour difference fa - fb
 * kept. */
void orc_round_state_f16(orc_sim *s) {
  const double r0 = s->c.rho0;
#pragma omp parallel for schedule(static)
  for (int64_t n = 0; n < s->N; ++n) {
    if (s->mask[n] != 0) continue;
    double *a = s->fa + n * Q, *b = s->fb + n * Q;
    double rho = 0.0;
    for (int i = 0; i < Q; ++i) rho += a[i] + b[i];
    for (int i = 0; i < Q; ++i) {
      const double f = a[i] + b[i], g = a[i] - b[i];
      const double h = round_binary16((f - WT[i] * rho) / (WT[i] * r0));
      const double fr = WT[i] * rho + WT[i] * r0 * h;
      a[i] = 0.5 * (fr + g);
      b[i] = 0.5 * (fr - g);
    }
  }
}

/* Global mass of each fluid, sums in node order. */
void orc_mass(const orc_sim *s, double out[2]) {
  double a = 0.0, b = 0.0;
  for (int64_t n = 0; n < s->N; ++n) {
    if (s->mask[n] != 0) continue;
    for (int i = 0; i < Q; ++i) {
      a += s->fa[n * Q + i];
      b += s->fb[n * Q + i];
    }
  }
  out[0] = a;
  out[1] = b;
}

/* Single-node kernels exposed for the identity tests. */
void orc_lattice(int32_t *c, double *w, int32_t *opp) {
  build_tables();
  for (int i = 0; i < Q; ++i) {
    for (int k = 0; k < 3; ++k) c[3 * i + k] = CV[i][k];
    w[i] = WT[i];
    opp[i] = OPPD[i];
  }
}
void orc_mrt_matrix(double *M, double *Minv) {
  build_tables();
  for (int r = 0; r < Q; ++r)
    for (int c = 0; c < Q; ++c) {
      M[r * Q + c] = MM[r][c];
      Minv[r * Q + c] = MINV[r][c];
    }
}
void orc_equilibrium(double rho, const double *u, double *feq) {
  build_tables();
  equilibrium(rho, u, feq);
}
void orc_guo_source(const double *u, const double *F, double *Fb) {
  build_tables();
  guo_source(u, F, Fb);
}
void orc_collide(const double *f, const double *feq, const double *Fb, double omega, double *out) {
  build_tables();
  mrt_collide(f, feq, Fb, omega, out);
}
double orc_omega(const orc_config *c, double phi) { return local_omega(c, phi); }
/* thresholds of the normal and the wetting rotation, and whether the rotation
 * fades in (1) or switches on at once (0); see the readings at eps_g */
void orc_set_regularisation(double g, double gt, int blend) {
  eps_g = g;
  eps_gt = gt;
  wet_blend = blend ? 1 : 0;
}
void orc_get_regularisation(double *g, double *gt, int *blend) {
  *g = eps_g;
  *gt = eps_gt;
  *blend = wet_blend;
}
int orc_num_threads(void) {
#ifdef _OPENMP
  return omp_get_max_threads();
#else
  return 1;
#endif
}
void orc_set_num_threads(int n) {
#ifdef _OPENMP
  if (n > 0) omp_set_num_threads(n);
#else
  (void)n;
#endif
}
