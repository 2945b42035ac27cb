/*
 * lbm.h -- C ABI of the MI355X (gfx950) hot path of the coupled
 * colour-gradient lattice Boltzmann / discrete element method of
 * Naga, Zhang, Yang and Kusumaatmaja, arXiv 2505.10171.
 *
 * One context holds one or more independent simulations (an ensemble); each is
 * a periodic box of nx*ny*nz lattice nodes whose node plane z = 0 is a solid
 * wall (unless has_wall = 0), filled with two immiscible equal-density fluids
 * (a: phi = +1, the drop liquid; b: phi = -1) and holding rigid frictional
 * spheres.  lbm_step advances both fluids and the particles; the other calls
 * move state across the host/device boundary.  The method's steps are those of
 * the paper's sections on the lattice Boltzmann model (colour-gradient
 * populations, MRT collision with Guo forcing, CSF surface tension,
 * recolouring, streaming), the fluid-particle coupling (half-way bounce-back
 * with moving walls, momentum exchange, refilling, geometric wetting,
 * capillary force) and the DEM (normal, sliding and rolling contact, Verlet).
 *
 * Conventions
 *  - Every function returns LBM_OK (0) or a negative lbm_status.  Errors are
 *    sticky: after any error every call on that context returns LBM_ESTATE
 *    until lbm_destroy; lbm_last_error gives the message.  Nothing throws.
 *  - Fields are x-fastest: node n = x + nx*(y + ny*z).  Vector fields are 3
 *    planes of N values (u_x, then u_y, then u_z).
 *  - D3Q19 order: 0 rest; 1..6 +x,-x,+y,-y,+z,-z; 7..10 (+-1,+-1,0),
 *    11..14 (+-1,0,+-1), 15..18 (0,+-1,+-1), each group in ++,+-,-+,-- order.
 *  - Mask codes: 0 fluid, 1 static wall (lbm_wall), 2+p inside particle p.  A node is inside
 *    particle p iff ((dx*dx)+(dy*dy))+(dz*dz) < R*R in FP64 without fused
 *    multiply-add, d = x - X wrapped once into (-L/2, L/2]; ties are fluid;
 *    the lowest particle index wins.
 *  - Memory: the caller owns every host buffer and the device workspace (for
 *    instance a torch uint8 CUDA tensor); the workspace must outlive the
 *    context.  The library allocates no device memory.  All device work is
 *    issued on the caller's HIP stream.
 *  - Threading: one context per stream; a context is not thread-safe.
 */
#ifndef LBM_H
#define LBM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct lbm_ctx lbm_ctx;

enum lbm_status {
  LBM_OK = 0,
  LBM_EINVAL = -1,    /* invalid argument or configuration                   */
  LBM_ENOMEM = -2,    /* workspace too small / host allocation failed        */
  LBM_EHIP = -3,      /* a HIP runtime call failed                           */
  LBM_EUNSTABLE = -4, /* NaN, rho <= 0 or |u| > 0.3 met at a fluid node      */
  LBM_ERANGE = -5,    /* index out of range, or a fixed capacity exceeded    */
  LBM_ESTATE = -6     /* the context is in the error state                   */
};

enum lbm_storage {
  LBM_STORE_FP32 = 0, /* total populations stored as FP32 deviations f - w rho0 */
  LBM_STORE_FP16 = 1  /* FP16: h = (f - w R)/(w rho0) with R the node's density
                         of the previous state; FP32 arithmetic.  Either way
                         the colour is held as the per-node order parameter:
                         the colour populations after the recolouring are a
                         function of f, rho, phi and the interface normal of
                         the node they left, and are rebuilt from them      */
};

/* Static solid of a simulation (lbm_config.has_wall). */
enum lbm_wall {
  LBM_WALL_NONE = 0,  /* fully periodic box                                   */
  LBM_WALL_PLANE = 1, /* the node plane z = 0 (the substrate of the drop runs)  */
  LBM_WALL_TUBE = 2,  /* a tube along x: node (x, y, z) is solid iff
                         (y - (ny-1)/2)^2 + (z - (nz-1)/2)^2 >= tube_R^2 (the
                         hydrodynamic benchmark of the section "Benchmarking
                         hydrodynamic force"); wetting and DEM contact use the
                         cylinder's normal, from the wall towards the axis     */
  LBM_WALL_BOXES = 3  /* a textured wall (the future work of the paper's
                         conclusions): the plane z = 0 and n_boxes boxes of
                         solid nodes; box b holds the nodes with
                         boxes[b][k] <= x_k <= boxes[b][3+k]; its solid surface
                         is the box grown by half a node.  Wetting takes the
                         normal of the nearest surface point (ties: the plane,
                         then the lowest box); each box is a DEM contact
                         partner of its own at its nearest surface point.
                         Needs open_x = 0                                    */
};
#define LBM_MAX_BOXES 8

enum lbm_field_bits {
  LBM_F_RHO = 1u,  /* total density rho                              (float) */
  LBM_F_U = 2u,    /* velocity with half the force (velocity eq.)   (float) */
  LBM_F_PHI = 4u,  /* order parameter (order-parameter eq.)         (float) */
  LBM_F_MASK = 8u, /* solid mask                                 (uint16_t) */
  LBM_F_POPS = 16u, /* raw stored populations, 19 per node in the storage
                       type, in blocks of 64 nodes: value i of node n at
                       (n / 64) 19 64 + 64 i + n % 64, the last block padded
                       (19 ceil(N / 64) 64 values).  FP32: f - w rho0.
                       FP16: the encoded h of LBM_STORE_FP16 (the reference
                       densities are internal)                             */
  LBM_F_FORCE = 32u  /* force per volume: CSF surface tension (CSF eq.) plus
                       the body force on fluid a                    (float) */
};

/* One simulation, in lattice units.  Defaults in brackets follow the paper's
 * parameter table. */
typedef struct {
  int32_t nx, ny, nz;   /* lattice size; nz >= 3, 19 (nx ny nz + 63) < 2^32 */
  int32_t has_wall;     /* lbm_wall [LBM_WALL_PLANE]                         */
  double rho0;          /* reference density [0.05]                          */
  double tau_a, tau_b;  /* relaxation times of fluids a and b (> 1/2) [1, 1] */
  double sigma;         /* surface tension [0.01]                            */
  double beta;          /* recolouring segregation parameter [0.7]           */
  double theta_wall_deg;/* wall contact angle through fluid a, (0, 180)      */
  double body_force[3]; /* force per volume on fluid a, times (1 + phi)/2    */
  double kn, kt, kr;    /* normal, sliding, rolling spring stiffness [2.5, 1, 0.5] */
  double gn, gt, gr;    /* normal, sliding, rolling damping [0, 0, 0]        */
  double delta_R;       /* mechanical minus hydrodynamic radius [1]          */
  double cap_k;         /* capillary geometric constant k [0.134]            */
  double cap_dang_deg;  /* Lagrangian grid spacing in degrees [2]            */
  int32_t storage;      /* lbm_storage                                       */
  int32_t n_particles;  /* spheres in this simulation (<= 4096)              */
  /* Open x ends (section "Benchmarking hydrodynamic force", pressure
   * inlet/outlet eq.): with open_x = 1 the x direction is not periodic; the
   * planes x = -1/2 and x = nx - 1/2 are pressure boundaries of density rho_in
   * and rho_out (p = rho / 3), held by anti-bounce-back with the boundary
   * node's own velocity; each fluid takes the node's colour share of rho_w.
   * Stencils take the node's own value beyond an open end.  Particles must keep
   * R + 4 nodes from both ends (LBM_ERANGE otherwise).  [0] */
  int32_t open_x;
  int32_t pad0;
  double rho_in, rho_out;
  double tube_R;        /* tube radius (LBM_WALL_TUBE)                       */
  int32_t n_boxes;      /* boxes of a textured wall (LBM_WALL_BOXES), <= 8   */
  int32_t pad1;
  int32_t boxes[LBM_MAX_BOXES][6]; /* lo x, y, z, hi x, y, z node indices  */
} lbm_config;

/* FP64 particle record, in and out. */
typedef struct {
  double x[3], v[3], w[3]; /* centre, velocity, angular velocity             */
  double q[4];             /* orientation quaternion (w, x, y, z)            */
  double R;                /* hydrodynamic radius R_p                        */
  double rho_p;            /* particle density (mass = rho_p 4/3 pi R^3)     */
  double theta_deg;        /* contact angle through fluid a                  */
  double mu_s, mu_r;       /* sliding and rolling friction coefficients      */
  double g_p;              /* downward force on the particle                 */
  int32_t kinematic;       /* 1: v and w are prescribed and never updated   */
  int32_t pad0;
  double F_hyd[3], T_hyd[3]; /* out: momentum-exchange force/torque, last step */
  double F_cap[3], T_cap[3]; /* out: capillary force/torque, last step       */
  double F_con[3], T_con[3]; /* out: contact force/torque (sub-step mean)    */
} lbm_particle;

/* Per-step history record: 27 doubles per particle per step, in the order
 * F_hyd[3], T_hyd[3], F_cap[3], T_cap[3], F_con[3], T_con[3], x[3], v[3], w[3]. */
#define LBM_HIST_DOUBLES 27

/* Device workspace needed for n_sims simulations (cfg[0..n_sims-1], with the
 * particles parts[s] that lbm_create will receive; the largest radius of each
 * simulation bounds the radii a later PUSH may set) and a per-step particle
 * history ring of history_steps entries.  Returns 0 if a configuration is
 * invalid. */
size_t lbm_workspace_bytes(const lbm_config* cfg, int32_t n_sims,
                           const lbm_particle* const* parts, int32_t history_steps);

/* Create a context: validates the configurations, carves the caller's device
 * workspace, uploads phi0 (per simulation a host float array of nx*ny*nz
 * values, or NULL for phi = +1 everywhere) and the particles (per simulation
 * cfg[s].n_particles host records, state at rest is allowed), sets the fluid at
 * rest with f_a = w rho0 (1+phi0)/2, f_b = w rho0 (1-phi0)/2 (the equilibrium
 * of the paper's lattice Boltzmann section at zero velocity, split by the
 * order-parameter eq.), builds the solid mask (coupling section: nodes inside
 * a sphere are solid) and the first moments (rho0, phi0).  The workspace must be 256-byte aligned
 * and at least lbm_workspace_bytes long (LBM_EINVAL / LBM_ENOMEM otherwise).
 * hip_stream is a hipStream_t (NULL: the null stream).  On success *out owns the
 * context. */
int lbm_create(const lbm_config* cfg, int32_t n_sims, const float* const* phi0,
               const lbm_particle* const* parts, int32_t history_steps,
               void* dev_workspace, size_t ws_bytes, void* hip_stream, lbm_ctx** out);

/* Advance every simulation by n_steps time steps (asynchronous on the stream).
 * Each step: collision + recolouring + streaming + bounce-back + momentum
 * exchange, capillary force, DEM, mask update, refilling, moments.  The
 * instability flag is checked by the next synchronising call. */
int lbm_step(lbm_ctx* ctx, int32_t n_steps);

/* Wait for the stream and report LBM_EUNSTABLE if the flow became unstable. */
int lbm_sync(lbm_ctx* ctx);

/* dir 0 (PULL): copy simulation sim's n particle records to parts, and, if
 * history is not NULL, up to max_steps most recent history records (oldest
 * first, LBM_HIST_DOUBLES * n doubles per step) to history; *n_hist (may be
 * NULL) receives the number of steps written.  The records carry the forces of
 * the paper's hydrodynamic force and torque eqs. (momentum exchange), the
 * capillary-force eq. and the DEM's net contact force.  dir 1 (PUSH): replace
 * the particle state (x, v, w, q and properties) from parts (a prescribed
 * path, as the detachment benchmark's); contact springs are kept; the mask is
 * rebuilt and fresh fluid nodes are refilled (refilling eqs.).  Synchronous. */
int lbm_particles_sync(lbm_ctx* ctx, int32_t sim, int32_t dir, lbm_particle* parts, int32_t n,
                       double* history, int32_t max_steps, int32_t* n_hist);

/* Copy fields of simulation sim (bits of lbm_field_bits).  rho, phi: N floats;
 * u: 3N floats; mask: N uint16; pops: 19 ceil(N/64) 64 values of the storage type.  Solid
 * nodes report rho = phi = 0 and u = the solid's surface velocity.  Buffers are
 * host memory unless dst_is_device.  Synchronous. */
int lbm_fields(lbm_ctx* ctx, int32_t sim, uint32_t what, float* rho, float* u, float* phi,
               uint16_t* mask, void* pops, int32_t dst_is_device);

/* As lbm_fields, with the force field (3N floats, LBM_F_FORCE) as well.  Solid
 * nodes report a zero force. */
int lbm_fields2(lbm_ctx* ctx, int32_t sim, uint32_t what, float* rho, float* u, float* phi,
                float* force, uint16_t* mask, void* pops, int32_t dst_is_device);

/* Links (x fluid, x + c_i inside particle p) of simulation sim, packed
 * (node << 5) | i, in particle, node, direction order; pid[k] = p.  Writes up
 * to max entries and stores the total in *count.  Synchronous. */
int lbm_links(lbm_ctx* ctx, int32_t sim, uint32_t* out, int32_t* pid, int64_t max,
              int64_t* count);

/* Global FP64 mass of fluids a and b of simulation sim: the sums over fluid
 * nodes of rho^a = rho (1 + phi)/2 and rho^b = rho (1 - phi)/2 (order-parameter
 * eq.).  Synchronous. */
int lbm_mass(lbm_ctx* ctx, int32_t sim, double out[2]);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the FP64
 * masses of fluids a and b of every simulation of the context, 2 doubles per
 * simulation in order, as lbm_mass computes them one simulation at a time.  It
 * allocates nothing: the accumulators live in a fixed device array of the
 * library, 2 * LBM_NOALLOC_MAX_SIMS doubles per GPU, held until the process
 * ends; a context of more simulations is rejected (LBM_ERANGE).  Every call on
 * a GPU shares that GPU's array, so calls that overlap on one GPU (two
 * streams, two threads) race; the array is cleared by a kernel at each call.
 * out: host memory (the call then waits for the stream), or device memory on
 * the context's device when dst_is_device (asynchronous on the stream, no
 * memset: it may be captured into a graph). */
#define LBM_NOALLOC_MAX_SIMS 1024
int lbm_mass_all_noalloc(lbm_ctx* ctx, double* out, int32_t dst_is_device);

/* Number of DEM sub-steps per lattice step of simulation sim (from the
 * collision-duration rule dt_DEM ~ t_c / 45). */
int lbm_dem_substeps(lbm_ctx* ctx, int32_t sim, int32_t* out);

/* Per-phase timing for benchmarks.  lbm_profile(ctx, k), k >= 1, starts (or
 * restarts) recording HIP events on the context's stream around the phases of
 * every k-th step (k = 1: every step):
 * kind 0 the fused collide-stream kernel, kind 1 the particle kernels other
 * than the link kernel (capillary, DEM, mask update, refill), kind 2 the
 * order-parameter kernel, kind 3 the interface kernels (normal and curvature),
 * kind 4 the link kernel (moving-wall terms and momentum exchange);
 * lbm_profile(ctx, 0) stops.  lbm_profile_read waits for the recorded steps and
 * writes, for the first n_kinds kinds, the summed GPU time in milliseconds and
 * the number of timed launches (per simulation and step). */
int lbm_profile(lbm_ctx* ctx, int32_t enable);
int lbm_profile_read(lbm_ctx* ctx, double* total_ms, int64_t* launches, int32_t n_kinds);

/* Block-shape autotuner for the per-node kernels (256 threads per block: 256
 * consecutive nodes, or x-y tiles of 256 x 1 .. 16 x 16 nodes; the moments pass
 * keeps its own tiling).  For each box class of the context it times `reps`
 * passes of the per-node kernels with every shape on the current state (each
 * pass the fluid part of a real step: interface, collide-and-stream, moments of
 * what was streamed) and keeps the fastest; results are identical with any
 * shape.  The state is left unchanged: the previous moments, which the timed
 * moments pass overwrites (8 bytes per node), and the status words are kept in
 * host memory meanwhile.  chosen (nullable, one per simulation) receives the
 * tile width (0 = consecutive nodes).  Choices are cached in the process per
 * (GPU architecture, box size, storage).  Synchronous. */
int lbm_autotune(lbm_ctx* ctx, int32_t reps, int32_t* chosen);

/* Set the block shape of one simulation by hand (tile width 0, 16, 32, 64,
 * 128 or 256; LBM_EINVAL otherwise). */
int lbm_set_tile(lbm_ctx* ctx, int32_t sim, int32_t tile_x);

/* Marching depth of the interface and moments passes of one simulation: each
 * block takes an x-y tile of 64 x 4, 32 x 8 or 16 x 16 nodes (the widest
 * whose whole tiles cover the box's width with at most 20 % to spare, else
 * 16 x 16) and marches up `planes` planes (1..256; 0 restores the default: 12 on planes
 * of at least 65,536 nodes unless that gives between 1,536 and 6,144 blocks,
 * else 6, or 8 where 6 gives more than 1,536 blocks and 8 at most 1,536; a
 * context of several simulations whose blocks at depth 24 number at least
 * 6,144 starts every simulation at 24).  Results are identical with any depth;
 * deeper blocks re-read fewer halo planes, shallower ones give more blocks
 * to fill the GPU. */
int lbm_set_march(lbm_ctx* ctx, int32_t sim, int32_t planes);

/* Graph replay of steps.  With enable = 1, lbm_step captures two consecutive
 * steps of every simulation into a HIP graph on the context's stream the first
 * time it runs at least two steps, and from then on replays that graph for each
 * pair of steps (an odd remaining step runs as ordinary launches).  The result
 * is the same as without the graph.  Needs a stream other than the null stream
 * (LBM_EINVAL otherwise); steps taken while lbm_profile is on are never
 * replayed from the graph.  enable = 0 releases the graph. */
int lbm_use_graph(lbm_ctx* ctx, int32_t enable);

void lbm_destroy(lbm_ctx* ctx);

/* Sticky error message of the context, or NULL if there is none. */
const char* lbm_last_error(const lbm_ctx* ctx);

#ifdef __cplusplus
}
#endif
#endif /* LBM_H */
