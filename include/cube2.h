/*
 * cube2.h -- C ABI of the MI355X (gfx950) implementation of the CUBE2 force
 * computation (Yu et al., "CUBE2: A Parallel N-Body Simulation Code for
 * Scalability, Accuracy, and Memory Efficiency", arXiv 2512.12629).
 *
 * What is computed (section 2.1, eqs. 3-4): the gravitational acceleration of
 * N equal-mass particles in a periodic cube, split into
 *   - a coarse PM level with softening b_coarse (eq. 4a, untruncated),
 *   - a fine PM level with softening b_fine truncated at b_coarse (eq. 4b),
 *   - a short-range particle-particle (PP) sum, softening b_pp, cut off at
 *     b_fine (eq. 4d with the finest PM level's softening as the cutoff),
 * where each PM level assigns mass with the cloud-in-cell kernel, solves
 * Poisson's equation by FFT with the optimized Green's function of eq. (11),
 * differentiates with the 4-point stencil of eq. (7) and interpolates with
 * the assignment kernel (section 2.1.2).  Leapfrog kick and drift act on
 * integer in-cell positions (IOS storage, section 2.3).  The *_backward
 * entry points are the adjoints (vector-Jacobian products) of the forward
 * ones; the paper has none, they are derived from the forward definitions.
 *
 * Units.  Inside the library lengths are in fine mesh cells (the fine mesh
 * has n_fine cells per side; the box side is n_fine).  Positions are integers
 * q in units of 2^-15 fine cells, q in [0, n_fine * 2^15).  The particle
 * "IOS" form stores, for particles sorted by their IOS cell (2x2x2 fine
 * cells), the low 16 bits of q per axis (uint16 SoA, pos[d*n + i]) and the
 * exclusive prefix count of particles per IOS cell (cell_start).  IOS cells
 * are ordered tile-major: tiles of 8^3 IOS cells, x fastest, and x fastest
 * inside a tile.  Velocities are fine cells per unit time, accelerations
 * fine cells per unit time^2, FP32 SoA (v[d*n + i]) in the particle order.
 *
 * Memory.  The caller owns all device memory.  cube2_sizes() gives the byte
 * sizes of two buffers: `tables` (persistent: Green's-function tables,
 * twiddles, the device status word; must outlive every call) and `work`
 * (scratch reused by every call; its contents are undefined between calls).
 * The library never allocates device memory.  Pointers marked (device) are
 * device addresses; pointers marked (host) are host addresses.
 *
 * Streams.  Every call enqueues work on `stream` (a hipStream_t, 0 = the
 * default stream) and returns without synchronising, except cube2_status
 * and cube2_reduce's host read-back.  One context must not be used from two
 * streams at once; calls sharing one `work` buffer must be serialised.
 *
 * Errors.  Every call returns 0 (CUBE2_OK) or a negative code.  Argument
 * errors are detected on the host before anything is enqueued.  Device-side
 * conditions (a deposit or codec accumulator that could overflow, a
 * kick-drift that met a non-finite velocity) set bits in the device status
 * word, which cube2_status() reports and clears.  Nothing is
 * printed and no exception crosses the ABI.
 */
#ifndef CUBE2_H
#define CUBE2_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* hipStream_t without requiring the HIP headers. */
typedef struct ihipStream_t *cube2_stream_t;

enum cube2_status_code {
    CUBE2_OK = 0,
    CUBE2_EINVAL = -1,        /* bad argument (null pointer, size, level) */
    CUBE2_EUNSUPPORTED = -2,  /* configuration outside the supported set */
    CUBE2_EWORKSPACE = -3,    /* tables or work buffer too small */
    CUBE2_EOVERFLOW = -4,     /* deposit accumulator could overflow (status) */
    CUBE2_EHIP = -5,          /* a HIP runtime call failed */
    CUBE2_ESTATE = -6,        /* tables not initialised */
    CUBE2_ENONFINITE = -7     /* kick-drift met a non-finite velocity (status) */
};

enum cube2_flags {
    CUBE2_PP_OFF = 1,         /* cube2_pp_force becomes a no-op (paper, sec. 4:
                                 PP may be disabled for fast runs) */
    CUBE2_FP64_FORM = 2,      /* also build the FP64 tables and size the work
                                 buffer for the *_f64 entry points */
    CUBE2_ASSIGN_TSC = 4,     /* TSC assignment (eq. 5) on every PM level instead
                                 of CIC: 16-bit fixed-point weights, density =
                                 accumulator * 2^-48, G with W = sinc^3 (eq. 9);
                                 the adjoints use the same weights and the
                                 slopes of eq. 5 */
    CUBE2_ISOLATED = 8        /* isolated boundaries (appendix A): the mesh is
                                 twice the isolation box, the particles must lie
                                 in [0, n_fine/2)^3 fine cells, and the
                                 untruncated level's target force is cut at
                                 r = n_fine/2 (its transform times
                                 1 - sinc(k L), eq. A2) */
};

/* Force parameters (section 2.1.1 and 2.2.2).  All lengths in fine cells. */
typedef struct cube2_config {
    int32_t n_fine;        /* fine cells per side: power of two, 16..1024 */
    int32_t coarse_ratio;  /* 0 = one PM level; else the coarse spacing in fine
                              cells: 2, 4 or 8, with n_fine/coarse_ratio >= 8 */
    double  b_coarse;      /* coarse softening b_1 (ignored with one level) */
    double  b_fine;        /* fine softening, also the PP cutoff; (0, 4]:
                              up to 2 PP pairs lie in adjacent IOS cells (27
                              neighbour cells), above 2 within two cells (125
                              neighbour cells, ~5x the PP work at equal
                              density) */
    double  b_pp;          /* PP softening b_PP, 0 < b_pp < b_fine */
    double  m_p;           /* particle mass */
    double  g_newton;      /* coupling constant G */
    int32_t alias_nmax;    /* alias sum |n_d| <= alias_nmax in eq. (11); the
                              paper truncates at 2 (section 2.1.2); 0..4 */
    int32_t flags;         /* cube2_flags */
} cube2_config;

typedef struct cube2_ctx cube2_ctx;

/* Validate `cfg` and create a host-side context (no device work).
 * Returns CUBE2_EUNSUPPORTED for sizes or ratios outside the set above, or
 * when no grid of K <= 128 equal intervals of [0, b_fine) has b_pp/2, b_pp
 * and b_fine/2 on its edges (the exact pair-law pieces of eq. 2 need that),
 * and CUBE2_EINVAL for non-positive softenings or b_pp >= b_fine. */
int cube2_create(const cube2_config *cfg, cube2_ctx **out);

/* Free a context (host memory only; device buffers belong to the caller). */
void cube2_destroy(cube2_ctx *ctx);

/* Byte sizes of the tables buffer and of the work buffer needed for up to
 * n_max particles. (host) outputs. */
int cube2_sizes(const cube2_ctx *ctx, int64_t n_max, size_t *table_bytes, size_t *work_bytes);

/* Host-only consistency check of the context's buffer layout for up to
 * n_max particles and of the index arithmetic the kernels derive from its
 * geometry, run on the host with the kernels' own index functions: the
 * velocity codec's bulk cells of every tile (section 2.3) and their per-tile
 * maxima, the PM adjoint's fixed-point coarse mesh and the concurrent PP
 * staging area stay inside their regions.  No device work; CUBE2_OK, or
 * CUBE2_EUNSUPPORTED / CUBE2_EWORKSPACE naming the failed check's kind. */
int cube2_self_check(const cube2_ctx *ctx, int64_t n_max);

/* Mesh geometry of level 0 (fine) or 1 (coarse): cells per side and the
 * complex row pitch P (in complex elements) of the half-spectrum layout
 * [kz][ky][kx], kx in [0, n/2] padded to P. */
int cube2_level_shape(const cube2_ctx *ctx, int level, int32_t *n, int32_t *pitch);

/* Build the Green's-function tables (eq. 11 with CIC W, eq. 10 D, eq. 12 R,
 * eq. 13 S; alias sum over |n_d| <= alias_nmax) in FP64 on the device and
 * store them in FP32 octant form, G[|mz|][|my|][mx], plus FFT twiddles, into
 * `tables` (device, table_bytes from cube2_sizes).  Runs once; the context
 * keeps the pointer. */
int cube2_init_tables(cube2_ctx *ctx, void *tables, size_t table_bytes, cube2_stream_t stream);

/* Copy the level's Green's table (FP32, (n/2+1)^3, [mz][my][mx]) to `out`
 * (device). */
int cube2_green_table(const cube2_ctx *ctx, int level, float *out, cube2_stream_t stream);

/* The FP32 pair law of the PP force (eqs. 2 and 4d: g = [R(r, b_pp) -
 * R(r, b_fine)] / r, so that a pair contributes g * D) exactly as the FP32
 * forward PP kernel evaluates it -- the same table, indexed by s = |D|^2,
 * and the same FP32 operations -- on the host, for inspecting its accuracy.
 * d (host, 3*n floats: d[k*n+i] is component k of separation i, fine
 * cells, each |component| < 4, or < 6 when b_fine > 2) in, g (host, n
 * floats) out.  No device work; CUBE2_EINVAL for a NULL pointer, n < 0 or a
 * component beyond that bound. */
int cube2_pair_law_f32(const cube2_ctx *ctx, const float *d, float *g, int64_t n);

/* The FP32 pair law and its derivative g_s = dg/ds (s = |D|^2) exactly as
 * the FP32 PP adjoint kernel evaluates them (its own table, the same FP32
 * operations), on the host; the pair Jacobian is d(g D)/dD = g I +
 * 2 g_s D D^T.  d as for cube2_pair_law_f32; g, gs (host, n floats) out. */
int cube2_pair_jacobian_f32(const cube2_ctx *ctx, const float *d, float *g, float *gs, int64_t n);

/* Quantise FP32 box-unit positions x (device, x[d*n+i] in [0,1)) to the
 * IOS form (section 2.3): q = floor(x * n_fine * 2^15) mod (n_fine * 2^15),
 * then sort stably by IOS cell.  Outputs (device): pos (3*n uint16 in-cell
 * offsets), cell_start ((n_fine/2)^3 + 1 prefix counts) and perm (n int32;
 * perm[i] = input index of sorted particle i). */
int cube2_pack(cube2_ctx *ctx, const float *x, int64_t n, uint16_t *pos, uint32_t *cell_start,
               int32_t *perm, void *work, size_t work_bytes, cube2_stream_t stream);

/* CIC mass assignment of one level (section 2.1.2 step 1, CIC kernel):
 * acc(node) = sum_i prod_d w_d, w = (2^15 - f, f), f the 15-bit in-cell
 * fraction of the particle on that level, summed exactly in uint64; the
 * FP32 density (particle masses per level cell) is acc rounded to nearest
 * times 2^-45.  With CUBE2_ASSIGN_TSC: TSC (eq. 5), three nodes per axis
 * around the nearest node with the 16-bit weights round((2^14 -/+ m)^2 /
 * 2^15) and 2^16 minus their sum (m the offset from the nearest node in
 * units of 2^-15), density = acc * 2^-48; the overflow guard then trips at
 * 2^17 particles in a tile's gathered box or 2^14 in a tile.  level 0 = fine (n_fine^3), 1 = coarse.  rho (device,
 * [z][y][x]) receives the FP32 density; rho_fx (device, optional, may be
 * NULL) receives the integer accumulator.  Bit-exact and order independent.
 * Sets CUBE2_EOVERFLOW in the status word if a tile holds 2^16 or more
 * particles (an accumulator could then exceed 64 bits). */
int cube2_deposit(cube2_ctx *ctx, const uint16_t *pos, const uint32_t *cell_start, int64_t n,
                  int level, float *rho, uint64_t *rho_fx, void *work, size_t work_bytes,
                  cube2_stream_t stream);

/* Forward unnormalised real-to-complex 3D FFT of a level mesh (device, n^3
 * FP32) into `spec` (device, n*n*P complex64 [kz][ky][kx]); entries beyond
 * kx = n/2 are zero.  Exposed for testing the transform. */
int cube2_fft_r2c(cube2_ctx *ctx, int level, const float *mesh, float *spec, void *work,
                  size_t work_bytes, cube2_stream_t stream);

/* Potential of a level (section 2.1.2 step 2): phi = IFFT(G * FFT(rho)),
 * inverse normalised by 1/n^3.  rho and phi (device, n^3 FP32) may alias. */
int cube2_potential(cube2_ctx *ctx, int level, const float *rho, float *phi, void *work,
                    size_t work_bytes, cube2_stream_t stream);

/* Finite-difference force and CIC interpolation (section 2.1.2 steps 3-4):
 * E = -D phi with the 4-point stencil of eq. (7), interpolated with the
 * deposit's integer weights; both levels are gathered in one particle sweep
 * (phi_coarse may be NULL with one level).  acc (device, 3*n FP32) receives
 * G m_p sum_levels H^-2 (W * E), H the level spacing; accumulate != 0 adds. */
int cube2_interp(cube2_ctx *ctx, const uint16_t *pos, const uint32_t *cell_start, int64_t n,
                 const float *phi_fine, const float *phi_coarse, float *acc, int accumulate,
                 cube2_stream_t stream);

/* The whole PM force of all levels: deposit, potential, interpolation.
 * acc (device, 3*n FP32), accumulate != 0 adds to it. */
int cube2_pm_force(cube2_ctx *ctx, const uint16_t *pos, const uint32_t *cell_start, int64_t n,
                   float *acc, int accumulate, void *work, size_t work_bytes,
                   cube2_stream_t stream);

/* The PM force of one level alone (section 2.1.2 steps 1-4 on that level):
 * level 0 = the fine level (eq. 4b, truncated at b_coarse when the context
 * has two levels), 1 = the coarse level (eq. 4a).  acc (device, 3*n FP32);
 * accumulate != 0 adds.  cube2_pm_force is the sum over the levels. */
int cube2_pm_level_force(cube2_ctx *ctx, const uint16_t *pos, const uint32_t *cell_start,
                         int64_t n, int level, float *acc, int accumulate, void *work,
                         size_t work_bytes, cube2_stream_t stream);

/* Local boxes of tiles (section 2.2.3).  The tile+buffer mode of the PM2
 * paragraph computes the fine level and PP of a tile on a local periodic box
 * holding the tile and a buffer zone around it: the fine level's force is
 * truncated at b_coarse, so a buffer of at least b_coarse + 3 fine cells
 * keeps every particle that acts on the tile's own particles and puts the
 * box's periodic images beyond the truncation; the coarse level stays global
 * (cube2_pm_level_force, level 1).  The PM3 level of the PM3 paragraph uses
 * the same boxes for subtiles, several of them packed into one box.
 *
 * cube2_tile_gather: for n_tiles tiles (origins, host, 3 ints per tile, x y
 * z, fine cells, even; 1 <= n_tiles <= 4096), the particles of the global
 * context's boxes of fine cells [origin - buffer, origin + tile + buffer)^3
 * (periodic; tile and buffer even; the slot side n_slot = tile + 2 buffer a
 * power of two, 32 <= n_slot <= n_fine).  Tile t is placed in slot t of a
 * k^3 grid of slots (k the smallest power of two with k^3 >= n_tiles, slot
 * t at (t mod k, (t / k) mod k, t / k^2) n_slot), and the packed box of
 * n_box = k n_slot <= 512 fine cells receives the positions in its box
 * units, x_local (device, (3, m) SoA at the front of a buffer of 3*m_max
 * floats; exact in FP32), with the particles' indices in the global order,
 * idx (device, m int32).  The order is fixed (tile by tile, region cells
 * z-major, x fastest, then the particle order within a cell), so the call is
 * deterministic.  *m (host) receives the count; the call synchronises the
 * stream to read it and returns CUBE2_EWORKSPACE, writing nothing, when it
 * exceeds m_max (or when n_tiles (n_slot/2)^3 exceeds the IOS cells of the
 * context).  Uses the fine-mesh and reduction areas of `work`.
 *
 * cube2_tile_scatter_add: for the m gathered particles after a cube2_pack on
 * the packed box's context (perm_local, device, m int32: gathered slot of
 * local particle i) and a force on it, acc_local (device, (3, m) in the
 * local particle order), adds scale * acc_local to acc (device, (3, n),
 * global order) at idx for the particles inside their tile proper (position
 * within the slot in [buffer, buffer + tile) fine cells on every axis).  A
 * box in units of H fine cells gives forces H^2 times those in fine units
 * (eq. 2 is homogeneous of degree -2), so scale = 1/H^2 there.  Each
 * particle lies in one tile of a tiling of the box, so the adds of one call
 * do not collide. */
int cube2_tile_gather(cube2_ctx *ctx, const uint16_t *pos, const uint32_t *cell_start, int64_t n,
                      const int32_t *origins, int32_t n_tiles, int32_t tile, int32_t buffer,
                      float *x_local, int32_t *idx, int64_t m_max, int64_t *m, void *work,
                      size_t work_bytes, cube2_stream_t stream);
int cube2_tile_scatter_add(int64_t m, const int32_t *perm_local, const float *x_local,
                           const int32_t *idx, int32_t n_tiles, int32_t tile, int32_t buffer,
                           float scale, const float *acc_local, float *acc, int64_t n,
                           cube2_stream_t stream);

/* cube2_pp_force restricted to the tiles (8^3 IOS cells) with skip_tiles[t]
 * == 0 (device, one byte per tile, t = (tz nt + ty) nt + tx with nt =
 * n_fine/16 tiles per side, may be NULL): the pair sums of the particles of a
 * skipped tile are neither computed nor written (their acc entries are left
 * as they are), as when the PM3 level of section 2.2.3 takes those
 * particles' short-range force with a shorter PP range. */
int cube2_pp_force_skip(cube2_ctx *ctx, const uint16_t *pos, const uint32_t *cell_start,
                        int64_t n, const uint8_t *skip_tiles, float *acc, int accumulate,
                        void *work, size_t work_bytes, cube2_stream_t stream);

/* PP force (eq. 4d): a_i += G m_p sum_{j != i, 0 < r < b_fine}
 * [R(r,b_pp) - R(r,b_fine)] (x_j - x_i)/r with R of eq. (2) and the exact
 * minimum-image integer separation, in FP32 with compensated summation.
 * acc (device, 3*n FP32), accumulate != 0 adds to it. */
int cube2_pp_force(cube2_ctx *ctx, const uint16_t *pos, const uint32_t *cell_start, int64_t n,
                   float *acc, int accumulate, void *work, size_t work_bytes,
                   cube2_stream_t stream);

/* cube2_pp_force without a work buffer, for callers that cannot allocate
 * (code under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc): the PP kernel's scratch (tile order, sort histogram and scan
 * temporaries, work counter: 4.3 MB at n_fine = 1024) lives in a fixed 5 MiB
 * device array of the library, one copy per device, held until the process
 * ends.  Same arguments and result as cube2_pp_force (bit for bit); the call
 * allocates nothing.  Every call on one device shares that array, so calls
 * that overlap on one device (two streams, two threads) race; the work
 * counter is cleared by a kernel at the start of each call.  CUBE2_EWORKSPACE
 * if the scratch does not fit the array (no supported n_fine). */
int cube2_pp_force_noalloc(cube2_ctx *ctx, const uint16_t *pos, const uint32_t *cell_start,
                           int64_t n, float *acc, int accumulate, cube2_stream_t stream);

/* The total force of eq. (4): the PM force of all levels plus the PP force,
 * acc = PM + PP (device, 3*n FP32, overwritten), equal bit for bit to
 * cube2_pm_force followed by cube2_pp_force with accumulate.  The PP part
 * runs on a stream of the context (made with its two events by
 * cube2_init_tables, default priority) beside the PM part on `stream`, with
 * its own tile queue and a 3*n FP32 staging area in `work`; `stream` waits
 * for both before the sum, so the call is ordered on `stream` like every
 * other.  Calls that share a context must not overlap (they share that
 * stream and the work regions). */
int cube2_force(cube2_ctx *ctx, const uint16_t *pos, const uint32_t *cell_start, int64_t n,
                float *acc, void *work, size_t work_bytes, cube2_stream_t stream);

/* Adjoint of cube2_force: x_bar = PM adjoint + PP adjoint for the cotangents
 * acc_bar (device, 3*n FP32 each; accumulate != 0 adds to x_bar), equal bit
 * for bit to cube2_pm_force_backward (with the same accumulate) followed by
 * cube2_pp_force_backward with accumulate (every adjoint scatter sums in
 * exact fixed point, so the result does not depend on the order of the
 * atomics), run the same way as cube2_force (PP adjoint on the context's
 * stream beside the PM adjoint on `stream`, joined before the sum). */
int cube2_force_backward(cube2_ctx *ctx, const uint16_t *pos, const uint32_t *cell_start,
                         int64_t n, const float *acc_bar, float *x_bar, int accumulate, void *work,
                         size_t work_bytes, cube2_stream_t stream);

/* Leapfrog kick and drift (sections 2.2.3, 2.3): v' = v + kick*a and
 * q' = q + rint(drift * v' * 2^15) (round half even, FP64 arithmetic),
 * wrapped periodically, then a stable re-sort by IOS cell.  Inputs (device):
 * pos_in, cell_start_in, vel_in (3*n), acc (3*n).  Outputs (device, must not
 * alias the inputs): pos_out, cell_start_out, vel_out, perm_out (perm_out[i] =
 * input slot of output particle i).  A component whose v' is not finite, or
 * whose displacement exceeds 2^62 position units, is not moved (its v' is
 * still stored) and the device status records CUBE2_ENONFINITE for
 * cube2_status; the call itself returns CUBE2_OK. */
int cube2_kick_drift(cube2_ctx *ctx, const uint16_t *pos_in, const uint32_t *cell_start_in,
                     const float *vel_in, const float *acc, int64_t n, double kick, double drift,
                     uint16_t *pos_out, uint32_t *cell_start_out, float *vel_out,
                     int32_t *perm_out, void *work, size_t work_bytes, cube2_stream_t stream);

/* FP64 diagnostics (device reductions, deterministic order): out8 (host) =
 * { m sum v_x, m sum v_y, m sum v_z, (m/2) sum |v|^2,
 *   m sum a_x, m sum a_y, m sum a_z, max |a| }.  vel may be NULL (zeros).
 * Synchronises the stream. */
int cube2_reduce(cube2_ctx *ctx, const float *vel, const float *acc, int64_t n, double *out8,
                 void *work, size_t work_bytes, cube2_stream_t stream);

/* IOS velocities (section 2.3: 16-bit velocities relative to a bulk
 * velocity field on a mesh; the paper defers the conversion formula, this
 * one is linear).  Bulk mesh: the coarse PM mesh, or cells of 4 fine cells
 * with one level; cube2_vel_bulk_side gives its side nb (host int out).
 *   v_bulk[d*nb^3 + (z*nb + y)*nb + x] = mean velocity of the particles in
 *     bulk cell (x, y, z) (0 for an empty cell), FP32, from exact 64-bit
 *     fixed-point sums;
 *   v_scale[0] = s = max_i |v_i - v_bulk(c_i)| / 32767 (1 if all are 0);
 *   vq[d*n+i] = rint((v - v_bulk(c_i)) / s), clamped to +-32767;
 * decode: vel = v_bulk(c_i) + s * vq (FP32, two roundings), so that the
 * round trip errs by at most s/2 plus FP32 rounding.  All arrays are device
 * memory in the IOS order of pos/cell_start; vel is 3*n floats, vq 3*n
 * int16, v_bulk 3*nb^3 floats, v_scale one float.  A bulk cell with 2^22
 * particles or more sets the overflow status. */
int cube2_vel_bulk_side(const cube2_ctx *ctx, int *side);
int cube2_vel_encode(cube2_ctx *ctx, const uint16_t *pos, const uint32_t *cell_start, int64_t n,
                     const float *vel, int16_t *vq, float *v_bulk, float *v_scale, void *work,
                     size_t work_bytes, cube2_stream_t stream);
int cube2_vel_decode(cube2_ctx *ctx, const uint16_t *pos, const uint32_t *cell_start, int64_t n,
                     const int16_t *vq, const float *v_bulk, const float *v_scale, float *vel,
                     cube2_stream_t stream);

/* Synchronise the stream and return the device status, clearing it:
 * CUBE2_OK, CUBE2_ENONFINITE (a kick-drift met a non-finite kicked velocity
 * or displacement; it has priority) or CUBE2_EOVERFLOW. */
int cube2_status(cube2_ctx *ctx, cube2_stream_t stream);

/* ---- adjoints ---------------------------------------------------------- */

/* Adjoint of cube2_deposit for the FP32 density of `level`: given rho_bar
 * (device, n^3), x_bar[d*n+i] (device, fine-cell units) = sum_nodes rho_bar
 * * d(W)/dx_d with the CIC weights' derivative (left-continuous at faces),
 * or with CUBE2_ASSIGN_TSC the TSC weights and the slopes of eq. 5 at the
 * particle's offset from its nearest node.  accumulate != 0 adds. */
int cube2_deposit_backward(cube2_ctx *ctx, const uint16_t *pos, const uint32_t *cell_start,
                           int64_t n, int level, const float *rho_bar, float *x_bar,
                           int accumulate, void *work, size_t work_bytes, cube2_stream_t stream);

/* Adjoint of cube2_pm_force: given acc_bar (device, 3*n), x_bar (device,
 * 3*n) = (d acc / d x)^T acc_bar.  Per level: scatter of acc_bar, FD
 * divergence (the transpose of eq. 7's stencil), the same FFT-G-IFFT (G is
 * real and even, so the operator is symmetric), the deposit adjoint, plus
 * the derivative of the interpolation weights.  The scatters sum in 64-bit
 * fixed point (scale 2^(41-e), 2^e > G m max|acc_bar| / H^2), so the result
 * is deterministic.  accumulate != 0 adds.  The fine scatter runs on a second
 * stream of the context (made by cube2_init_tables, default priority) beside
 * the recomputed forward potentials on `stream`, which waits for it: the call
 * is ordered on `stream` like every other, and calls that share a context
 * must not overlap. */
int cube2_pm_force_backward(cube2_ctx *ctx, const uint16_t *pos, const uint32_t *cell_start,
                            int64_t n, const float *acc_bar, float *x_bar, int accumulate,
                            void *work, size_t work_bytes, cube2_stream_t stream);

/* Adjoint of cube2_pp_force: x_bar_k = G m_p sum_j J(D_kj) (acc_bar_j -
 * acc_bar_k), J(D) = g(r) I + g'(r) D D^T / r.  accumulate != 0 adds. */
int cube2_pp_force_backward(cube2_ctx *ctx, const uint16_t *pos, const uint32_t *cell_start,
                            int64_t n, const float *acc_bar, float *x_bar, int accumulate,
                            void *work, size_t work_bytes, cube2_stream_t stream);

/* Adjoint of cube2_kick_drift with the rounding taken as identity:
 * given the output cotangents xbar_out, vbar_out (device, 3*n, output order)
 * and perm (from the forward), writes in input order
 * vbar_in = vbar_out + drift * xbar_out, xbar_in = xbar_out and
 * acc_bar = kick * vbar_in (all device, 3*n). */
int cube2_kick_drift_backward(cube2_ctx *ctx, int64_t n, const int32_t *perm,
                              const float *xbar_out, const float *vbar_out, double kick,
                              double drift, float *xbar_in, float *vbar_in, float *acc_bar,
                              cube2_stream_t stream);

/* ---- FP64 plain form ---------------------------------------------------
 * The same force evaluated in FP64 throughout on the device: the density is
 * the deposit's exact integer accumulator times 2^-45, the Green's tables
 * (eq. 11) and FFT twiddles are stored in FP64, the FFT-G-IFFT pipeline,
 * the eq. (7) stencil and the CIC interpolation run in FP64, and the PP pair
 * law (eqs. 2, 4d) is the same exact piecewise polynomial evaluated in FP64.
 * It is the reference the FP32 path is measured against on sizes the host
 * cannot evaluate.  All three return CUBE2_ESTATE unless the context was
 * created with CUBE2_FP64_FORM and its tables are initialised. */

/* FP64 potential of a level: phi = IFFT(G * FFT(rho)) / n^3; rho and phi
 * (device, n^3 FP64, [z][y][x]) may alias. */
int cube2_potential_f64(cube2_ctx *ctx, int level, const double *rho, double *phi, void *work,
                        size_t work_bytes, cube2_stream_t stream);

/* FP64 PM force of all levels (deposit, potential, interpolation) into acc
 * (device, 3*n FP64); accumulate != 0 adds. */
int cube2_pm_force_f64(cube2_ctx *ctx, const uint16_t *pos, const uint32_t *cell_start,
                       int64_t n, double *acc, int accumulate, void *work, size_t work_bytes,
                       cube2_stream_t stream);

/* FP64 PP force (eq. 4d) into acc (device, 3*n FP64); accumulate != 0 adds.
 * A no-op (or a zero fill) with CUBE2_PP_OFF, like cube2_pp_force. */
int cube2_pp_force_f64(cube2_ctx *ctx, const uint16_t *pos, const uint32_t *cell_start,
                       int64_t n, double *acc, int accumulate, void *work, size_t work_bytes,
                       cube2_stream_t stream);

/* Text of a status code. */
const char *cube2_strerror(int code);

#ifdef __cplusplus
}
#endif

#endif /* CUBE2_H */
