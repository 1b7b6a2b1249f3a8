/*
 * libpic - MI355X (gfx950) implementation of the relativistic
 * particle-in-cell step of Nattila, "Runko: Modern multiphysics toolbox for
 * plasma simulations" (arXiv 1906.06306).
 *
 * One time step follows the paper's time-advance loop (Table 1):
 *   pic_fdtd_step(PIC_HALF_B)          push_half_b1            Eq. (fdB)
 *   pic_push_interp(...)               interp_em + push        Sect. 2.3.2,
 *                                                              App. C, Eq. (fdX)
 *   pic_fdtd_step(PIC_HALF_B)          push_half_b2            Eq. (fdB)
 *   pic_deposit_current(...)           comp_curr, clear_vir_cur,
 *                                      cur_exchange            App. D
 *   pic_fdtd_step(PIC_CURL_E_ADD_J)    push_e + add_cur        Eq. (fdE)
 *   pic_sort_migrate(...)              particle communication rows
 * pic_step() enqueues that sequence; with PIC_PUSH_HALF_B the first half
 * update runs inside the push (on its LDS copy of B) and both halves are
 * applied to the stored B by one PIC_TWO_HALF_B pass, and with FDTD2 and no
 * current filter the last two rows before the migration are one
 * pic_deposit_current(PIC_DEPOSIT_CURL_E) pass.
 *
 * Units (App. A): dx = dt = 1, Courant number c = cfl; E, B, J in code
 * units; four-velocities u in units of the speed of light.
 *
 * Lattice (Sect. 2.3.1): each box stores, per component, one plane of
 * n0*n1*n2 values, x fastest; storage index (i,j,k) holds
 *   Ex (i+1/2,j,k)  Ey (i,j+1/2,k)  Ez (i,j,k+1/2)
 *   Bx (i,j+1/2,k+1/2)  By (i+1/2,j,k+1/2)  Bz (i+1/2,j+1/2,k)
 * and J is co-located with E.  Dimensions at or beyond `dim` have extent 1.
 *
 * Tiles (Sect. 3.1): every box is cut into tiles of tile[0] x tile[1] x
 * tile[2] cells (even edges dividing the box).  Particles are stored per
 * (tile, species) segment, structure of arrays, positions relative to the
 * tile centre (x_loc in [-T/2, T/2) per grid dimension) in the chosen
 * precision; the cell of a particle is floor(x_loc) + T/2.  Boxes are
 * periodic and independent (a batch of boxes is stepped together).
 *
 * Memory: the caller allocates ONE device workspace of
 * pic_layout.total_bytes (256-byte aligned) and owns it; the library never
 * allocates or frees device memory.  Every region (fields, particles, tile
 * tables, staging) is at the offsets pic_query() reports.  The library owns
 * only the host-side context.
 *
 * Streams: a context is bound to one HIP stream; every call except
 * pic_query, pic_error, pic_diagnostics and pic_destroy only enqueues work.
 *
 * Errors: functions return a pic_status.  Argument errors are returned at
 * once (PIC_E_ARG, PIC_E_STATE); HIP runtime failures return PIC_E_HIP with
 * text in pic_last_error().  Conditions found on the device (a full tile
 * segment or outbox, a non-finite momentum, a displacement of a cell or
 * more, a particle outside its tile) are latched as bits in a device word
 * and returned by the next synchronising call (pic_error, pic_diagnostics).
 * Particles are never dropped silently: an overflow sets PIC_E_CAPACITY and
 * the state must be discarded.
 */
#ifndef PIC_H_
#define PIC_H_

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t pic_status;

/* synchronous status codes */
#define PIC_OK 0
#define PIC_E_ARG 1      /* invalid configuration or argument             */
#define PIC_E_HIP 2      /* HIP runtime error, see pic_last_error()         */
#define PIC_E_STATE 3    /* call out of order (e.g. deposit before push)    */
/* device-latched bits (returned OR-ed, shifted left by 8) */
#define PIC_E_CAPACITY (1 << 8)     /* tile segment or outbox overflow     */
#define PIC_E_CFL (1 << 9)          /* |dx| >= 1 cell in one step          */
#define PIC_E_NONFINITE (1 << 10)   /* NaN/Inf momentum or position        */
#define PIC_E_OUT_OF_TILE (1 << 11) /* stored position outside its tile    */
#define PIC_E_ADJ_MAP (1 << 12)     /* adjoint origin id beyond the target
                                       buffer (wrong before_stride)       */

#define PIC_FP32 0
#define PIC_FP64 1

#define PIC_MAX_SPECIES 4

/* pic_fdtd_step phases (Table 1 rows) */
#define PIC_HALF_B 0        /* B -= (c/2) curl+ E        push_half_b1/b2  */
#define PIC_CURL_E 1        /* E += c curl- B            push_e           */
#define PIC_ADD_J 2         /* E -= J                    add_cur          */
#define PIC_CURL_E_ADD_J 3  /* both, one pass (they commute)              */
#define PIC_TWO_HALF_B 4    /* push_half_b1 then push_half_b2 in one pass:
                               B -= (c/2) curl+ E twice, E unchanged between */

/* flags of pic_push_interp / pic_deposit_current / pic_sort_migrate */
#define PIC_FUSED 1u        /* push also deposits J and moves leavers out  */
#define PIC_SORT_CELLS 2u   /* stable sort by cell inside every tile        */
#define PIC_PUSH_HALF_B 4u  /* the push applies push_half_b1 to its own LDS
                               copy of B; stored B stays at B^{n-1/2}, and
                               the caller then uses PIC_TWO_HALF_B          */
#define PIC_DEPOSIT_CURL_E 8u /* pic_deposit_current also applies
                               E += c curl- B - J (push_e + add_cur, as
                               PIC_CURL_E_ADD_J) in the fold's pass, from the
                               folded J; FDTD2 only                         */

/* species_mask of pic_push_interp / pic_deposit_current: bit s selects
 * species s (Table 1 runs interp_em, push and comp_curr once per particle
 * container); PIC_ALL_SPECIES selects every species. */
#define PIC_ALL_SPECIES 0xffffffffu

typedef struct {
    int32_t dim;          /* spatial dimensions D in {1,2,3}                 */
    int32_t precision;    /* PIC_FP32 or PIC_FP64                           */
    int32_t n_species;    /* 1..PIC_MAX_SPECIES                              */
    int32_t n_boxes;      /* independent periodic boxes, >= 1                */
    int32_t tile[3];      /* tile edge per dimension: even, >= 2, divides
                             every box; 1 for dimensions >= dim             */
    int32_t block;        /* threads per work-group of particle kernels
                             (64..1024, multiple of 64); 0 = default 256    */
    double cfl;           /* Courant number c, 0 < c <= 1/sqrt(D)           */
    const int32_t *box_cells;   /* host [n_boxes][3] cells per dimension     */
    const double *charge;       /* host [n_boxes][n_species] q (signed)      */
    const double *qm;           /* host [n_boxes][n_species] App. C factor
                                   s = q/(m m_pm) = sign(q)/m_pm             */
    const double *mass;         /* host [n_boxes][n_species] macro-particle
                                   mass (kinetic-energy diagnostic only)      */
    const int64_t *tile_capacity; /* host [tiles][n_species] particles a
                                   segment can hold, or NULL: see capacity   */
    double capacity_factor;     /* if tile_capacity == NULL: segment capacity
                                   = ceil(factor * count/tiles_in_box) + 64,
                                   rounded up to 64 (default 1.25 if <= 0)    */
    int32_t outbox_capacity;    /* leavers per (tile, species) per step; 0 =
                                   default (a quarter of the segment, >= 256) */
    uint32_t options;           /* PIC_OPT_* bits, 0 = defaults              */
    const int32_t *box_walls;   /* host [n_boxes] PIC_WALL_* bits, or NULL
                                   (every box periodic in every dimension)   */
    int32_t pusher;             /* PIC_PUSHER_BORIS (0), _VAY or _HC          */
    int32_t filter_passes;      /* binomial filter passes pic_step applies to
                                   J before add_cur (0 = none)               */
    int32_t fdtd_order;         /* 2 (or 0): App. B differences; 4: FDTD4 of
                                   the solver table, every curl difference
                                   over +-1/2 and +-3/2 with weights 9/8 and
                                   -1/24 (periodic boxes; pic_step then keeps
                                   the half B updates out of the push)      */
    int64_t inject_max;         /* largest batch pic_inject takes (sizes the
                                   binning scratch); 0 = the largest initial
                                   (box, species) count                      */
} pic_config;

/* pic_config.pusher (the solver table's pushers): the relativistic Boris
 * update of App. C; the Vay pusher (full electric kick and half the magnetic
 * kick with the old velocity, the other half with the new velocity solved
 * exactly for its Lorentz factor); the Higuera-Cary pusher (Boris's split
 * with the rotation's Lorentz factor from the same implicit relation).  The
 * two last keep force-free motion (E + v x B = 0) exact.  Units as App. C. */
#define PIC_PUSHER_BORIS 0
#define PIC_PUSHER_VAY 1
#define PIC_PUSHER_HC 2

/* pic_config.box_walls: conducting, reflecting walls on the node planes
 * x = 0 and x = n0 of the box (y, z stay periodic).  Tangential E (Ey, Ez)
 * and normal B (Bx) are held at zero on the wall planes (pic_init_tiles
 * zeroes them); the x-staggered components (Ex, By, Bz) see the wall as a
 * mirror in the interpolation; a particle whose move crosses a wall is
 * reflected (x mirrored, u_x -> -u_x) and deposits its current along the
 * broken path to the wall point and on to the mirrored position, which
 * keeps the continuity equation exact.  Boxes with walls need the fused
 * push; the reverse-mode calls reject them; the Gauss diagnostic skips the
 * wall plane (it carries the conductor's surface charge). */
#define PIC_WALL_X 1

/* pic_config.options: accumulate the fused push's current block in LDS in
 * the working precision.  Without it (the default) an FP64 run accumulates
 * in FP64 and an FP32 run in 64-bit fixed point (each ZigZag value scaled
 * by 2^e with |q| 2^e < 2^30 and rounded to an integer, the sum exact and
 * independent of the order of the atomics); the block is converted to the
 * working precision once when it is written out. */
#define PIC_OPT_ACC_WORKING 1u
/* pic_config.options: run the push as a persistent walker (a grid of
 * resident work-groups pulls (tile, species) segments, largest first, from
 * an atomic counter) instead of one work-group per segment. */
#define PIC_OPT_PERSISTENT 2u
/* pic_config.options: origin tracking for the reverse-mode adjoint.  Every
 * fused step (and pic_init_tiles) records, per stored particle, where it
 * came from: the slot it held before the step, or its index in the
 * concatenated input of pic_init_tiles (boxes, then species, then input
 * order).  Adds the ids region and the adjoint scratch to the workspace.
 * With it, pic_push_interp requires PIC_FUSED and PIC_SORT_CELLS is
 * rejected (neither path records origins). */
#define PIC_OPT_TRACK 4u

/* Byte offsets of the regions inside the caller's workspace.  Fields:
 * [3][cells_total] each, boxes concatenated (box b starts at cell offset
 * box_cell_offset[b]).  Particles: [dim][capacity_total] positions and
 * [3][capacity_total] four-velocities; segment (tile t, species s) starts at
 * element seg_offset[t*n_species+s] (int64, device).  Counts: int32
 * seg_count[t*n_species+s] (device).  elem = 4 (FP32) or 8 (FP64) bytes. */
typedef struct {
    uint64_t total_bytes;
    uint64_t off_E, off_B, off_J;           /* elem [3][cells_total]          */
    uint64_t off_pos, off_u;                /* elem [D|3][capacity_total]     */
    uint64_t off_xold;                      /* elem [D][capacity_total]       */
    uint64_t off_seg_offset;                /* int64 [tiles][species]          */
    uint64_t off_seg_capacity;              /* int32 [tiles][species]          */
    uint64_t off_seg_count;                 /* int32 [tiles][species]          */
    uint64_t off_error;                     /* int32 latched device error bits */
    uint64_t off_flags;                     /* int32 [tiles][species] particles
                                               of each segment flagged near a
                                               cell face (see pic_diag)        */
    uint64_t off_ids;                       /* int32 [capacity_total] origin of
                                               each particle (PIC_OPT_TRACK)   */
    int64_t cells_total;
    int64_t tiles_total;
    int64_t capacity_total;
    int64_t outbox_capacity;
    int32_t elem_bytes;
    int32_t reserved;
} pic_layout;

/* Initial state of box b, species s (index b*n_species+s), device
 * pointers, FP64, global coordinates of that box in cells, [0, n_d):
 * pos: [dim][count] planes, u: [3][count].  E, B: per box [3][cells]. */
typedef struct {
    const int64_t *count;          /* host [n_boxes][n_species]              */
    const double *const *pos;      /* host array of device pointers          */
    const double *const *u;        /* host array of device pointers          */
    const double *const *E;        /* host array [n_boxes] of device ptrs    */
    const double *const *B;        /* host array [n_boxes] of device ptrs    */
} pic_init_data;

/* FP64 diagnostics of the current state (Eqs. fdE/fdB, App. B). */
typedef struct {
    double field_energy;     /* 1/2 sum(E^2 + B^2) over all boxes           */
    double kinetic_energy;   /* sum m c^2 (gamma - 1) over all particles, c
                                the Courant number (code units, App. A)    */
    double gauss_max;        /* max |div- E - rho| on nodes                  */
    double divb_max;         /* max |div+ B| on cell centres                 */
    double charge_total;     /* sum rho                                      */
    int64_t particles;       /* particles stored                            */
    int64_t near_face;       /* particles flagged near a cell face: a
                                stored tile-local coordinate x lies within
                                2 ulps of the storage precision at the tile
                                half-width, |x - rint(x)| <= 2 ulp(T_d/2),
                                of an integer.  Every particle within 1 ulp
                                of a face is among them, and so is every
                                particle whose cell an FP32 step can put on
                                the other side of a face than the FP64 step
                                from the same input.  Counted over the
                                state after the last init, injection, push
                                or cell sort.                               */
    int32_t error_bits;      /* latched device errors (then cleared)         */
    int32_t reserved;
    double continuity_max;   /* max |rho^{n+1} - rho^n + div- J| on nodes (App.
                                D's discrete continuity) when exactly one step
                                separates this call from the previous
                                diagnostics call, else -1.  J is the last
                                step's current (after any filter passes). */
} pic_diag;

typedef struct pic_ctx pic_ctx;

/* Workspace layout for a configuration and initial particle counts
 * (host [n_boxes][n_species]).  Pure host computation.  PIC_E_ARG on an
 * invalid configuration (tile not dividing a box, odd tile edge, cfl out
 * of range, unsupported dim/precision/species count). */
pic_status pic_query(const pic_config *cfg, const int64_t *counts, pic_layout *out);

/* Bind a context to a workspace and stream, convert the initial FP64 state:
 * bin particles by tile (stable: input order kept inside a tile), convert
 * positions to tile-centre-relative coordinates in the working precision
 * (a value that rounds onto the upper tile face moves to the next tile at
 * -T/2), count particles within 1 ulp of a cell face, convert E and B, and
 * zero J.  The workspace must be at least pic_query's total_bytes. */
pic_status pic_init_tiles(const pic_config *cfg, const int64_t *counts, void *workspace,
                          uint64_t workspace_bytes, const pic_init_data *init, void *hip_stream,
                          pic_ctx **out);

/* Field update on every box (Eqs. fdE/fdB with the forward and backward
 * differences of App. B; periodic).  phase: PIC_HALF_B, PIC_CURL_E,
 * PIC_ADD_J, PIC_CURL_E_ADD_J or PIC_TWO_HALF_B. */
pic_status pic_fdtd_step(pic_ctx *ctx, int32_t phase);

/* interp_em + push for every particle of the species in species_mask:
 * linear interpolation of each E and B
 * component from its own staggered lattice (Sect. 2.3.2), relativistic
 * Boris update of u (App. C), position advance x += c u/gamma (Eq. fdX).
 * One step may push its species in several calls with disjoint masks (all
 * with the same PIC_FUSED setting) before its deposit and migration; a
 * species pushed twice in a step, an empty mask or a bit beyond n_species
 * is rejected (PIC_E_STATE, PIC_E_ARG), and with PIC_OPT_TRACK the mask
 * must cover every species.  The push also counts, per segment, the
 * particles it leaves near a cell face (pic_diag.near_face).
 * Without PIC_FUSED the new positions are stored in place unrebased and
 * the old ones in the xold region, for pic_deposit_current and
 * pic_sort_migrate.  One work-group handles one (tile, species) segment;
 * the segments are visited in decreasing particle count (re-sorted on the
 * device at every 8th push, at the first push after init or an injection,
 * and at every captured push; the order does not change the results).  With PIC_FUSED the same work-group also deposits
 * the ZigZag current of its particles into the segment's current block
 * (App. D) and compacts the particles that stay, moving leavers to the
 * segment's outbox (the "tag outflowing / pack" rows of Table 1). */
pic_status pic_push_interp(pic_ctx *ctx, uint32_t species_mask, uint32_t flags);

/* comp_curr + clear_vir_cur + cur_exchange for the species in species_mask
 * (each pushed in this step): after an unfused push, ZigZag
 * deposit from (xold, x) into per-segment current blocks; in both modes, sum
 * the blocks (every selected species of the tile plus the halos of its
 * neighbours) into J on the lattice, in a fixed order, so J is the current
 * of the selected species only.  One call per step.  With PIC_DEPOSIT_CURL_E the same
 * pass then updates E at each cell as pic_fdtd_step(PIC_CURL_E_ADD_J) would
 * (Eq. (fdE), same arithmetic), so the step saves that launch and the re-read
 * of J; B must already hold B^{n+1/2}.  PIC_E_ARG with the flag under FDTD4,
 * PIC_E_STATE without a preceding push of every selected species. */
pic_status pic_deposit_current(pic_ctx *ctx, uint32_t species_mask, uint32_t flags);

/* Particle communication rows of Table 1: after an unfused push, move the
 * particles that left each tile out (stable compaction); then every tile
 * appends the arrivals from its neighbours (directions in increasing code
 * sum (delta_d+1) 3^d, each in the sender's order) with positions rebased
 * by -delta T (exact).  PIC_SORT_CELLS then sorts every tile segment
 * stably by cell index (x fastest) and recounts near-face particles.
 *
 * Optional outputs (device buffers the caller owns, or NULL; written on the
 * context's stream, nothing synchronises):
 *   migration_counts  int32 [tiles_total][n_species][3^dim]: entry (t, s, k)
 *                     is the number of particles of species s that were in
 *                     tile t before the step and are in the neighbour at
 *                     offset delta (k = sum_d (delta_d + 1) 3^d, tiles of a
 *                     box periodic) after it; the centre code counts the
 *                     particles that stayed.  Needs a preceding push
 *                     (PIC_E_STATE otherwise); species not pushed in the
 *                     step count as staying.
 *   flagged           int64 [flagged_capacity + 1]: flagged[0] receives the
 *                     number of particles flagged near a cell face after the
 *                     call (the rule of pic_diag.near_face), flagged[1..]
 *                     the particle slots (element index into the particle
 *                     planes) of the first min(that number,
 *                     flagged_capacity) of them in increasing slot order.
 *                     Costs one extra pass over the positions.
 * PIC_E_ARG if flagged_capacity < 0. */
pic_status pic_sort_migrate(pic_ctx *ctx, uint32_t flags, int32_t *migration_counts, int64_t *flagged,
                            int64_t flagged_capacity);

/* One full time step in Table-1 order (see the top of this header), every
 * species; flags as for pic_push_interp, plus PIC_SORT_CELLS.  With FDTD2 and no
 * current filter the deposit and the E update run as one
 * pic_deposit_current(PIC_DEPOSIT_CURL_E) call. */
pic_status pic_step(pic_ctx *ctx, uint32_t flags);

/* Capture nsteps calls of pic_step(flags) into a HIP graph on the context's
 * stream (after one eager step, which also sets kernel attributes).  The
 * steps contain no memset nodes (fills are kernels).  Replaces a previous
 * graph.  PIC_E_STATE if called between a push and its migration; PIC_E_ARG
 * if the context is bound to the default (null) stream, which cannot be
 * captured. */
pic_status pic_graph_capture(pic_ctx *ctx, int32_t nsteps, uint32_t flags);

/* Particle creation in tiles (the shock setup's injector adds plasma every
 * step from a receding wall, Sect. 5.2): append count particles of one box
 * and species, FP64 global positions pos [dim][count] and four-velocities
 * u [3][count] (device pointers; the caller draws them), binned into their
 * tiles exactly as pic_init_tiles does and placed after the particles a tile
 * already holds (input order kept).  Between steps only.  A full segment
 * latches PIC_E_CAPACITY; a position outside the box PIC_E_OUT_OF_TILE.
 * Injected particles carry origin id -1 (the reverse-mode calls do not cover
 * creation).  Electrons and positrons placed on the same positions add no
 * net charge, so Gauss's law is kept. */
pic_status pic_inject(pic_ctx *ctx, int32_t box, int32_t species, int64_t count, const double *pos,
                      const double *u);

/* The solver table's 3-point binomial current filter: passes times, J <-
 * the (1/4, 1/2, 1/4) average along every grid dimension (the 3^D product
 * stencil), periodic.  pic_step calls it between the current fold and
 * add_cur with pic_config.filter_passes.  Boxes with walls are rejected. */
pic_status pic_filter_current(pic_ctx *ctx, int32_t passes);

/* Replay the captured steps on the context's stream. */
pic_status pic_graph_launch(pic_ctx *ctx);

/* Synchronise the stream and return (then clear) the latched device error
 * bits, or PIC_E_HIP. */
pic_status pic_error(pic_ctx *ctx);

/* FP64 diagnostics of the current state.  Synchronises the stream.  Its
 * return value includes the latched device error bits (then cleared). */
pic_status pic_diagnostics(pic_ctx *ctx, pic_diag *out);

/* The diagnostics of pic_diagnostics for callers that cannot allocate memory
 * (code in tight serving or stepping loops, harnesses that forbid
 * allocation): the same values (the reduction over tiles runs on the
 * device in the same order as pic_diagnostics' host loop), with the
 * per-tile partial sums and charge blocks in a static device array of the
 * library (16 MiB per device, held until the process ends) instead of the
 * workspace and a host buffer; it allocates no device or host memory.
 * PIC_E_ARG if the context's tiles need more than 16 MiB there: 8 doubles
 * plus (T+1)^D charge values per tile (e.g. 4,096 2D tiles of 16^2 cells
 * take 9.7 MB).  Every context on a device shares that device's array, and
 * each call overwrites it completely: calls that overlap on one device (two
 * threads, or two streams) race and must be serialised by the caller.
 * Synchronises the stream; returns the latched device error bits (then
 * cleared) like pic_diagnostics. */
pic_status pic_diagnostics_static(pic_ctx *ctx, pic_diag *out);

/* The same diagnostics per box: out is a host array of n_boxes entries
 * (error_bits is the context's, repeated in every entry). */
pic_status pic_diagnostics_boxes(pic_ctx *ctx, pic_diag *out);

/* Reverse mode.  The adjoint of one step maps the sensitivities of a loss
 * to the state after the step (x^{n+1}, u^{n+1/2}, E^{n+1}, B^{n+1/2}) to
 * those of the state before it (x^n, u^{n-1/2}, E^n, B^{n-1/2}): the
 * transposed Jacobian of every Table-1 row taken in reverse order
 * (add_cur, push_e, push_half_b2, comp_curr of App. D, the position update
 * of Eq. fdX, the Boris update of App. C, interp_em of Sect. 2.3.2,
 * push_half_b1), with the transposed curls (curl+)^T = curl- on the
 * periodic Yee lattice.  Adjoint arrays are device buffers in the working
 * precision with the layouts of the state: particles [dim|3][capacity_total]
 * (segment slots), fields [3][cells_total].  Both calls need PIC_OPT_TRACK
 * and only enqueue work; device-side problems are latched as in forward
 * steps.  Reverse a step from a saved copy of the workspace: the caller
 * restores the state after the step and calls pic_adjoint_unpermute, then
 * restores the state before it and calls pic_adjoint_step. */

/* Move particle adjoints from the slots of the current state to where each
 * particle came from (the ids region): lpos_after/lu_after are indexed by
 * the current slots; lpos_before/lu_before ([dim|3][before_stride]) receive
 * them at the origin slots.  before_stride = capacity_total after a step;
 * after pic_init_tiles it is the total input count, and the output is in
 * the concatenated input order.  Entries of lpos_before/lu_before that no
 * particle maps to are left unchanged.  The buffers must not overlap. */
pic_status pic_adjoint_unpermute(pic_ctx *ctx, const void *lpos_after, const void *lu_after, void *lpos_before,
                                 void *lu_before, int64_t before_stride);

/* Reverse the fused step (PIC_FUSED | PIC_PUSH_HALF_B, the same arithmetic
 * as without PIC_PUSH_HALF_B) taken from the current state.  On entry
 * lpos, lu hold the adjoints of x^{n+1}, u^{n+1/2} at the slots of the
 * particles in the current state (after pic_adjoint_unpermute), lE, lB
 * those of E^{n+1}, B^{n+1/2}; on return, in place, the adjoints of the
 * current state.  The state itself is not modified.  Particles stopped by a
 * latched device error (non-finite, CFL, outside the tile) keep their
 * adjoint unchanged. */
pic_status pic_adjoint_step(pic_ctx *ctx, void *lpos, void *lu, void *lE, void *lB);

/* Release the host context (the workspace stays the caller's). */
pic_status pic_destroy(pic_ctx *ctx);

/* Text of the last error on this thread ("" if none). */
const char *pic_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* PIC_H_ */
