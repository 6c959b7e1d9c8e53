/*
 * lbm.h -- C ABI of the MI355X ensemble lattice-Boltzmann + rare-event library.
 *
 * An ensemble of independent trajectories of a 2-D channel flow past a square
 * (paper Section 2) is advanced by a D2Q9 lattice-BGK scheme (paper Appendix
 * A) while the drag on the square is recorded every step (paper Section 2.1).
 * The GKTL algorithm (paper Section 4.2, Appendix C) and trajectory AMS (paper
 * Section 4.1, Appendix B) clone and prune the trajectories; branched copies
 * are perturbed as in paper Appendix D.
 *
 * Conventions shared by every call
 * --------------------------------
 * - Lattice units (dx = dt = 1, c_s^2 = 1/3).  Directions c_0..c_8 are
 *   (0,0), (1,0), (0,1), (-1,0), (0,-1), (1,1), (-1,1), (-1,-1), (1,-1);
 *   weights 4/9, 1/9 (x4), 1/36 (x4).
 * - Geometry: ny fluid rows between halfway bounce-back walls at y = 0 and
 *   y = ny, periodic in x (or fed by an inlet and drained by an outlet,
 *   lbm_set_open_channel).  The square with side s and lower-left cell
 *   (sq_x0, sq_y0) is solid on cells sq_x0..sq_x0+s-1, sq_y0..sq_y0+s-1 and
 *   must keep one fluid cell to every side: 1 <= sq_x0, sq_x0 + s <= nx - 1,
 *   1 <= sq_y0, sq_y0 + s <= ny - 1.  s = 0 means no obstacle.
 * - Populations are stored as FP32 deviations d_i = f_i - w_i from the
 *   rest state, structure-of-arrays: member m occupies a block of 9*nx*ny
 *   floats, laid out [i][y][x] with x fastest, in one of the two buffers.
 *   At lbm_create the block of member m starts at the sum of 9*nx*ny over
 *   members 0..m-1; a GKTL cloning may hand blocks from member to member
 *   (gktl_select_clone), so lbm_member_state and lbm_copy_state_in/out are
 *   the way to a member's current state.  What is stored for step t is the
 *   post-collision state f_i^out(t); streaming happens when step t+1 reads
 *   it.  Solid cells (the square, an open channel's grid bars) are never
 *   written by the lattice steps, and what they hold never enters a result.
 * - Time: lbm_init produces step 0 (equilibrium at rest with the seeded
 *   density, relaxed once) and its drag; each step of lbm_step_batch
 *   produces the next step and its drag.  The drag of step t is written at
 *   column t of the member's row of the drag series.
 * - Collision: BGK, d_i <- d_i + (d_i^eq - d_i)/tau + F_i, with Guo's body
 *   force (u = (sum c_i f_i + F/2)/rho; F_i = (1 - 1/(2 tau)) w_i
 *   [3 (c_i - u) + 9 (c_i.u) c_i].F).  The paper prints the relaxation without
 *   its leading f_i term; this is the standard form its viscosity relation
 *   nu = (tau - 1/2)/3 belongs to.
 * - Drag (x-force on the square) by momentum exchange: the sum over fluid
 *   cells x and directions i with x + c_i in the square of 2 c_ix f_i^out(x).
 * - Random numbers: Philox4x64-10 (Salmon et al., SC'11).  Key = (seed or
 *   key, purpose), purpose tags INIT 0x494E4954, GKTS 0x474B5453,
 *   PRTB 0x50525442, AMSP 0x414D5350; the counter and word used by each
 *   draw are given with the call that makes it.  A word w becomes the
 *   uniform (w >> 11) * 2^-53, or the index floor(w * n / 2^64).
 * - Streams: every call that takes or owns a hipStream_t enqueues its work
 *   on it and returns without waiting, unless its comment says otherwise.
 * - Memory: every large buffer is owned by the caller and passed as a
 *   device pointer; the library never frees caller memory.  The library
 *   allocates its own small device scratch (per-member bookkeeping, drag
 *   partial sums) in lbm_create and frees it in lbm_destroy.
 * - Errors: every call returns LBM_OK (0) or a negative code; the message
 *   of the last failure on the calling thread is lbm_last_error().  Argument
 *   errors are detected before any work is enqueued.
 * - A context is not thread-safe; distinct contexts are independent.
 */
#ifndef MI355X_LBM_H
#define MI355X_LBM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define LBM_OK 0
#define LBM_EINVAL (-1)       /* bad argument (sizes, geometry, tau <= 1/2, null pointer) */
#define LBM_EHIP (-2)         /* a HIP runtime call failed */
#define LBM_ERANGE (-3)       /* drag-series capacity would be exceeded */
#define LBM_EUNSUPPORTED (-4) /* valid request the library does not implement */
#define LBM_ENONFINITE (-5)   /* every trajectory has a non-finite weight */

typedef struct lbm_ctx lbm_ctx;

/* One trajectory: lattice size, obstacle, relaxation time and body force. */
typedef struct {
    int32_t nx, ny;            /* lattice cells; nx >= 4, ny >= 4, 9 nx ny < 2^32 */
    int32_t sq_x0, sq_y0;      /* lower-left solid cell of the square */
    int32_t sq_side;           /* side s in cells, 0 = no obstacle */
    int32_t reserved;          /* must be 0 */
    double tau;                /* BGK relaxation time, > 1/2 (nu = (tau - 1/2)/3) */
    double force_x;            /* body-force density along x (lattice units) */
} lbm_member_desc;

/* Floats one population buffer must hold for this ensemble (sum of 9*nx*ny). */
size_t lbm_state_floats(const lbm_member_desc* members, int32_t n_members);

/*
 * Create a context for n_members independent trajectories of the channel
 * flow (paper Section 2: the flow past the square; Section 4: the rare-event
 * algorithms work on an ensemble of such trajectories, run in parallel).
 *   pop_a, pop_b   caller-owned device buffers of pop_floats floats each
 *                  (>= lbm_state_floats), 16-byte aligned; states ping-pong
 *                  between them.
 *   drag_series    caller-owned device float[n_members][series_capacity];
 *                  drag of step t goes to [m][t].
 *   accum          caller-owned device double[n_members]: running
 *                  sum over steps of (f_d - mu)/sigma * dt (lbm_set_observable),
 *                  the time integral of the observable that GKTL weighs.
 *   hip_stream     hipStream_t every call of this context enqueues on
 *                  (NULL = the null stream).
 * Returns LBM_EINVAL on bad geometry or sizes.  Does not touch the buffers.
 */
int lbm_create(lbm_ctx** out, const lbm_member_desc* members, int32_t n_members,
               float* pop_a, float* pop_b, size_t pop_floats,
               float* drag_series, int32_t series_capacity, double* accum,
               void* hip_stream);

/* Release the context and the library's own scratch (not the caller's buffers). */
int lbm_destroy(lbm_ctx* ctx);

/*
 * Step 0 of every member (paper Section 2: equilibrium start).  Cell (x, y)
 * of member m gets density rho = 1 + noise_amp * (2u - 1), u from Philox
 * key (seed, INIT), counter (y*nx + x, m, 0, 0), word 0; populations are the
 * equilibrium at rest f_i = w_i rho, relaxed once (collision with the body
 * force).  Writes the drag of step 0 at column 0, zeroes accum and the
 * non-finite flags, and activates every member.
 */
int lbm_init(lbm_ctx* ctx, uint64_t seed, double noise_amp);

/* As lbm_init, but the populations start at the equilibrium of density rho and
   the uniform velocity (ux0, 0), |ux0| <= 0.3 (ux0 = 0 is lbm_init).  Used to
   start a channel flow near its developed speed instead of at rest. */
int lbm_init_flow(lbm_ctx* ctx, uint64_t seed, double noise_amp, double ux0);

/* Observable weighed by GKTL: A(t) = (f_d(t) - mu)/sigma, integrated with step dt. */
int lbm_set_observable(lbm_ctx* ctx, double mu, double sigma, double dt);

/*
 * Choose which members lbm_step_batch advances (host int32[n_members], nonzero
 * = active; NULL = all).  An inactive member keeps its state, drag columns
 * and accumulator untouched, and its own step counter stops.
 */
int lbm_set_active(lbm_ctx* ctx, const int32_t* active_host);

/*
 * Advance every active member by n_steps steps (paper Appendix A: stream,
 * then collide).  The collision update is computed in FP64 from the FP32
 * stored deviations and rounded once to FP32 on store (the drag of a step is
 * summed in FP64 and stored in FP32).  Records each step's drag in the
 * member's next column and
 * adding (f_d - mu)/sigma * dt to accum.  A member whose drag becomes
 * non-finite is flagged (lbm_flags).  LBM_ERANGE if an active member would
 * pass series_capacity.  Steps are grouped in chunks of 64 (one drag
 * reduction each); a full chunk is captured once into a HIP graph (on a
 * private stream) and replayed on the context's stream until the launch
 * configuration changes (tile shape, collision, open channel, number of
 * active members, observable), so that the host submits one graph per 64
 * steps instead of 33 to 129 kernel launches.
 */
int lbm_step_batch(lbm_ctx* ctx, int32_t n_steps);

/* Replay captured chunks in lbm_step_batch (on = 1, the default) or launch
   every kernel of every chunk (on = 0).  Both give bit-identical results. */
int lbm_set_graphs(lbm_ctx* ctx, int32_t on);

/* The drag on the square (paper Section 2.1: the x-force the flow exerts on
   the obstacle; here by momentum exchange, see the conventions above) of steps
   t0 .. t1-1 of every member: copies drag columns [t0, t1) into out_dev
   (device float[n][t1-t0], row m = member m), enqueued on the context's
   stream.  LBM_EINVAL unless 0 <= t0 <= t1 <= series_capacity; out_dev may
   be NULL when t0 == t1 (nothing is copied). */
int lbm_drag(const lbm_ctx* ctx, int32_t t0, int32_t t1, float* out_dev);

/* Device pointer to member m's current state ([9][ny][nx] deviations). */
int lbm_member_state(const lbm_ctx* ctx, int32_t m, float** state_dev);

/* Next drag column (= number of steps taken, step 0 included) of member m. */
int lbm_member_time(const lbm_ctx* ctx, int32_t m, int32_t* t);

/* Set every member's next drag column to t (reuse the series buffer). */
int lbm_set_time(lbm_ctx* ctx, int32_t t);

/* Copy the non-finite flags into out_dev (device int32[n_members]): 1 where a
   member's drag has become non-finite since lbm_init. */
int lbm_flags(const lbm_ctx* ctx, int32_t* out_dev);

/* Overwrite the non-finite flags from flags_dev (device int32[n_members],
   non-zero = flagged); used to resume a saved ensemble exactly.  Enqueued on
   the context's stream; flags_dev must stay valid until the copy has run. */
int lbm_set_flags(lbm_ctx* ctx, const int32_t* flags_dev);

/*
 * Pressure, stress and shear on the square's faces, for the populations the
 * next step collides (paper Section 2.1: the drag as the surface integral of
 * the stress of Appendix A, and its forebody-minus-base pressure
 * approximation; Section 3.2.2: the mean shear along the top or bottom face).
 * Each face is represented by the s fluid cells adjacent to it.  Writes
 * out_dev[m * 5 + q] (device FP64) for every member m:
 *   q = 0  p_fb   = sum over the front cells of c_s^2 rho
 *   q = 1  p_base = sum over the base cells of c_s^2 rho
 *   q = 2  drag from the stress: sum of tau_xb n_b over the four faces (n the
 *          square's outward normal), tau_ab = -c_s^2 rho delta_ab
 *          - (1 - 1/(2 tau)) sum_i c_ia c_ib (f_i - f_i^eq)
 *   q = 3  mean shear on top:    (1/s) sum u_x over the top cells / (1/2)
 *   q = 4  mean shear on bottom: (1/s) sum (-u_x) over the bottom cells / (1/2)
 * with u the Guo-shifted velocity and tau the member's (an open channel's
 * sponge is taken not to reach the square); zeros for members without a
 * square.  Enqueued on the context's stream.
 */
int lbm_face_diagnostics(const lbm_ctx* ctx, double* out_dev);

/*
 * Collision operator of every member (paper Appendix A, last paragraph: for
 * its turbulent runs the paper relaxes in central moments instead of BGK).
 * model 0: BGK with Guo forcing (the default; rates ignored).  model 1:
 * central-moment multiple-relaxation-time collision with Guo forcing: the
 * nine central moments of D2Q9 (about the Guo-shifted velocity) relax
 * towards the central moments of the discrete second-order equilibrium and
 * receive the central moments of Guo's source weighted by (1 - s/2); the
 * shear moments k20 - k02 and k11 relax at 1/tau (the viscosity), the trace
 * k20 + k02 at s_bulk, k21 and k12 at s_third, k22 at s_fourth.  Rates in
 * (0, 2); with all three equal to 1/tau the result is BGK's.  With all three
 * equal to 1 (the paper's setting) the library evaluates the same collision
 * in a shorter form (the trace and the third- and fourth-order moments leave
 * it at closed-form values, so their pre-collision values are not formed):
 * equal up to FP64 rounding.  Call before lbm_init (its step 0 collides
 * too); synchronises the context's stream.
 */
int lbm_set_collision(lbm_ctx* ctx, int32_t model, double s_bulk, double s_third, double s_fourth);

/*
 * Open channel (paper Section 2): every member's channel is fed by an inlet
 * and drained by an outlet instead of being periodic in x, with an entrance
 * grid and a sponge zone.  The paper describes these only in words; the
 * reading implemented:
 *   inlet   ghost column x = -1 at the equilibrium of rho = 1 and
 *           u = (u_in(y), 0), u_in(y) = 4 u_c (y + 1/2)(ny - y - 1/2) / ny^2;
 *   grid    solid bars of grid_bar x grid_bar cells in columns grid_x0 ..
 *           grid_x0 + grid_bar - 1, on the rows y >= grid_bar/2 (integer
 *           division) with (y - grid_bar/2) mod (2 grid_bar) < grid_bar;
 *           halfway bounce-back, their force is not part of the drag;
 *           grid_bar = 0: no grid;
 *   sponge  tau(x) = tau + (sponge_tau - tau) r^2, r = (x - sponge_x0) /
 *           (nx - 1 - sponge_x0), for x > sponge_x0 (sponge_x0 >= nx - 1:
 *           none); the central-moment collision takes 1/tau(x) as its
 *           shear rate;
 *   outlet  ghost column x = nx rebuilt before every step from the stored
 *           state (the post-collision populations f of the last step), per
 *           row: u_g = 2 u(nx-1) - u(nx-2) with u = sum c_i f_i / sum f_i,
 *           density rho_g = 1 (outlet_density = 0) or rho_g = 2 rho(nx-1) -
 *           rho(nx-2) (outlet_density = 1, the paper's second-order
 *           extrapolation of the density), strain S from differences (d/dx
 *           the extrapolation slope, d/dy centred, one-sided in the first
 *           and last rows), and g_i = f_i^eq(rho_g, u_g) + w_i / (2 c_s^4)
 *           (c_i c_i - c_s^2 I) : Pi, Pi = -2 rho_g c_s^2 (tau(nx-1) - 1) S.
 *           With the unit-density inlet, an extrapolated outlet density
 *           leaves the channel's pressure level and flow rate to the outlet
 *           (small channels fill until the flow stops, drain to twice the
 *           inlet's flux, or blow up, by tau), hence the default 0.
 * Requirements (every member): grid within columns 1 .. nx - 3 and, with a
 * square, ending at least two columns before it; the square at least two
 * columns from the inlet (sq_x0 >= 2) and three from the outlet
 * (sq_x0 + s <= nx - 3); 0 <= u_c <= 0.3; sponge_tau > 1/2; ny <= 2048
 * (LBM_EUNSUPPORTED beyond: the ghost kernel keeps a column in LDS).  The body
 * force of the members still applies.  A small kernel rebuilds the ghost
 * columns before every launch; the two-step shapes build the outlet column
 * of their second step themselves.  lbm_init then starts every member
 * from the inlet profile (lbm_init_flow requires ux0 = 0).  oc = NULL
 * restores periodic channels.  Call before lbm_init; synchronises the
 * context's stream; allocates 9 * sum(ny) floats of library scratch for the
 * ghost columns (freed by the next call or lbm_destroy).
 */
typedef struct {
    double u_c;            /* inlet centre-line velocity */
    int32_t grid_x0;       /* first column of the grid bars */
    int32_t grid_bar;      /* bar height = width = gap; 0 = no grid */
    int32_t sponge_x0;     /* last column before the sponge ramp */
    int32_t outlet_density; /* 0: held at 1 (default); 1: extrapolated to second order */
    double sponge_tau;     /* relaxation time at the outlet column, > 1/2 */
} lbm_open_channel;

int lbm_set_open_channel(lbm_ctx* ctx, const lbm_open_channel* oc);

/*
 * Launch shape of the lattice step (an index into the library's table of
 * shapes; see lbm_tile_count).  Every shape computes bit-identical states and
 * drag.  Shapes 0-15 make one step per launch (tiles of 256 columns by a few
 * rows).  Shapes 16-19 make two steps per launch: a workgroup sweeps a strip
 * of 256 columns from the bottom row to the top and keeps the intermediate
 * step in on-chip memory, so the populations cross HBM once per two steps.
 * They apply when every member's width is a multiple of 256; otherwise, and
 * for the last step of an odd batch, the library steps with shape 0.  Shapes
 * 21-23 are shape 16 with each strip cut into workgroups of 128, 64 and 32
 * rows (the rows next to a cut are collided by both neighbours).  Shape 20,
 * the default, makes two steps per launch with whole strips when there are
 * at least two per compute unit and with strips cut into the tallest row
 * ranges that give four workgroups per compute unit otherwise (32 rows at
 * the least); it steps with shape 0 while the active members give fewer
 * than 1.5 workgroups per compute unit (the few members an AMS branch
 * re-simulates would leave most compute units idle).
 */
int lbm_set_tile(lbm_ctx* ctx, int32_t tile_id);
int32_t lbm_tile_count(void);
/* Lattice steps per launch that the next lbm_step_batch makes (1 or 2), for
   the shape in use and the members active now. */
int lbm_launch_steps(const lbm_ctx* ctx, int32_t* steps);
/* Time every tile shape on this ensemble (n_steps each, on the context's
   stream, synchronising it) and keep the fastest.  Writes the chosen id.  If
   that shape makes two steps per launch and the ensemble has several runs of
   lattice shapes (an uneven batch), each run's row range (whole strips, 128,
   64 or 32 rows per workgroup) is then tuned on its own, one run at a time,
   keeping a choice only where the whole ensemble's step is at least 1 %
   faster; lbm_get_run_rows reads the result.  Earlier lbm_set_run_rows
   choices are discarded. */
int lbm_autotune(lbm_ctx* ctx, int32_t n_steps, int32_t* best_tile);

/* Runs of consecutive members with one lattice shape: the ensemble's
   segments, each with its own row range in two-step launches. */
int lbm_run_count(const lbm_ctx* ctx, int32_t* n_runs);
/* Rows per workgroup of each run in two-step launches: rows[r] = -1 as the
   tile shape says (its own policy), 0 whole strips of 256 columns, else row
   ranges of rows[r] rows (a range of ny or more is a whole strip).  n_runs
   must be lbm_run_count's, or 0 (rows may then be NULL) to drop every
   choice.  Results are bit-identical whatever the ranges (each range
   collides the rows beside it that its second step pulls).  Kept across
   lbm_set_tile; LBM_EINVAL on a wrong count or a value below -1 (nothing
   changes). */
int lbm_set_run_rows(lbm_ctx* ctx, const int32_t* rows, int32_t n_runs);
/* The rows per workgroup each run uses now (0: whole strips; -1 for every
   run if the shape in use makes one step per launch): writes n_runs and, if
   rows is not NULL, max_runs >= n_runs entries. */
int lbm_get_run_rows(const lbm_ctx* ctx, int32_t* rows, int32_t max_runs, int32_t* n_runs);
/* lbm_autotune with a persisted table: path is a text file of lines
   "<key>\t<tile id>[ <rows of run 0>,<rows of run 1>,...]", the key naming
   the runs of lattice shapes, the collision and whether the channels are
   open.  A line with this context's key sets its shape (and row ranges)
   without timing anything; otherwise the context is tuned and a line
   appended (the file is created if missing).  LBM_EINVAL if the line cannot
   be written (the tuned shape is set all the same). */
int lbm_autotune_cached(lbm_ctx* ctx, int32_t n_steps, const char* path, int32_t* best_tile);

/*
 * GKTL cloning at the end of a period (paper Appendix C.1, weight equation;
 * Appendix D, perturbation).  All members must share one lattice shape.
 *   s_n = k * accum[n]; ln R = ln((1/N) sum_n exp(s_n)) in FP64 with the
 *   largest s_n factored out; ln R goes to ln_r_dev[0] (device double).
 *   Multinomial resampling: new slot m takes ancestor a_m, the first n
 *   whose running sum C_n = sum_{l<=n} exp(s_l - s_max) (index order)
 *   exceeds u_m * C_{N-1}, u_m from key (key, GKTS), counter (m, period, 0, 0),
 *   word 0.  Non-finite s_n has weight 0.  ancestors_dev (device int32[N])
 *   receives a_m.  Every member's state becomes its ancestor's.  The lowest
 *   slot taking each ancestor is an exact copy; every other copy is
 *   perturbed: f <- f + eps * sum_n alpha_n f^(n) with alpha_n from key
 *   (key, PRTB), counter (m, period, n / 4, 0), word n % 4, then scaled by
 *   one factor that restores its mass before perturbation.
 *   How the copies are made (lbm_set_cloning): by default the exact copy of
 *   ancestor n takes over n's block, so it moves no data, and each further
 *   copy is written (copied or perturbed) into the block of a state that
 *   left no descendant (the k-th further copy in slot order into the k-th
 *   such block in slot order), so that only further copies cost memory
 *   traffic; or every copy is gathered into the other buffer.  The states,
 *   drag and results of every later call are the same bit for bit.
 *   snapshots: device, n_snap <= 16 states in this library's deviation
 *   layout ([n_snap][9][ny][nx]), 16-byte aligned; may be NULL when
 *   eps == 0 or n_snap == 0.
 *   accum is reset to 0; flags are copied from the ancestor.
 * LBM_ENONFINITE if every s_n is non-finite (nothing is changed).  Waits once
 * on the context's stream (after the selection, to read its status).
 * Members <= 4096.
 */
int gktl_select_clone(lbm_ctx* ctx, double k, uint64_t key, int32_t period,
                      double eps, const float* snapshots, int32_t n_snap,
                      int32_t* ancestors_dev, double* ln_r_dev);

/* How gktl_select_clone makes its copies: relabel = 1 (the default) moves
   only the copies beyond the first of each ancestor, relabel = 0 gathers
   every copy into the other buffer (each member keeps its block).  Same
   results either way. */
int lbm_set_cloning(lbm_ctx* ctx, int32_t relabel);

/*
 * Perturb selected members in place (paper Appendix D) without cloning:
 * member m with mask_host[m] != 0 gets f <- f + eps * sum_n alpha_n f^(n),
 * alphas from key (key, PRTB), counter (m, period, n / 4, 0), word n % 4,
 * then the scale that restores its mass.  Used at AMS branching points.
 */
int lbm_perturb(lbm_ctx* ctx, const int32_t* mask_host, uint64_t key, int32_t period,
                double eps, const float* snapshots, int32_t n_snap);

/*
 * Copy states between members of this context and external device buffers
 * (checkpoints).  lbm_copy_state_out writes member m's current state into
 * dst_dev ([9][ny][nx] floats); lbm_copy_state_in makes src_dev the current
 * state of member m and sets its next drag column to t.
 */
int lbm_copy_state_out(const lbm_ctx* ctx, int32_t m, float* dst_dev);
int lbm_copy_state_in(lbm_ctx* ctx, int32_t m, const float* src_dev, int32_t t);

/*
 * Trajectory-AMS selection (paper Section 4.1; Appendix B.1).  Independent of
 * any context: works on N score series of length t_len (device float[N][t_len],
 * row-major).  The maximum of each row goes to maxima_dev (device float[N]);
 * a row holding NaN or +inf (a blown-up trajectory) counts as -inf, while -inf
 * entries are ordinary lowest scores (e.g. before a time average is defined).  The level is the n_kill-th
 * lowest maximum; every member at or below it is killed (ties together), in
 * increasing slot order, into killed_dev[0..K-1].  Kill j picks its parent
 * uniformly among the survivors (increasing slot order) with index
 * floor(w * n_surv / 2^64), w from key (key, AMSP), counter (j, iteration, 0, 0),
 * word 0, into parent_dev[j]; branch_t_dev[j] is the first column where the
 * parent's score is strictly above the level.  n_killed_dev (device int32)
 * receives K, level_dev (device float) the level.  If every member is at the
 * level (extinction) K = N and parents/branch times are -1.  N <= 2048.
 */
int ams_score_kill_branch(const float* series_dev, int32_t n, int32_t t_len, int32_t n_kill,
                          uint64_t key, int32_t iteration,
                          int32_t* killed_dev, int32_t* parent_dev, int32_t* branch_t_dev,
                          int32_t* n_killed_dev, float* level_dev, float* maxima_dev,
                          void* hip_stream);

/*
 * Window mean of each member's drag series (paper Section 3.2, time-averaged
 * drag): out_dev[m][t] = (1/T) sum_{t' = t-T+1}^{t} f_d(t') for t >= T-1 within
 * [0, t_len) of the device series (float[n][ld]), and -inf for t < T-1.
 * Sums in FP64 (each thread sums its first window in order and slides over
 * its next 15 outputs).  Used as the plain AMS score.
 */
int lbm_window_mean(const float* series_dev, int32_t n, int32_t ld, int32_t t_len, int32_t window,
                    float* out_dev, void* hip_stream);

/*
 * GKTL estimators (paper Appendix C.1-C.2), FP64 on the device.
 *
 * gktl_rebuild: the final trajectory j of a run with n_periods cloning
 * periods of tau steps is traced back through ancestors_dev ([n_periods][n],
 * as written by gktl_select_clone: slot m after period i continued slot a_m of
 * period i).  traj_dev[j] (device float[n][n_periods*tau]) receives its drag
 * series, rebuilt from series_dev (device float[n][ld]; period i occupies
 * columns col0 + i*tau .. col0 + (i+1)*tau - 1 of the slot that carried it);
 * traj_integral_dev[j] the integral of the observable along the lineage (sum
 * over periods of integrals_dev[i][slot], device double[n_periods][n], in
 * period order); log_weight_dev[j] = sum_i ln R_i - k * traj_integral[j], the
 * log of the weight that turns the biased ensemble back into the unbiased law
 * (the paper prints this weight with the exponent's sign flipped).
 */
int gktl_rebuild(const int32_t* ancestors_dev, const double* integrals_dev, const double* ln_r_dev,
                 const float* series_dev, int32_t ld, int32_t col0, int32_t n, int32_t n_periods, int32_t tau,
                 double k, float* traj_dev, double* log_weight_dev, double* traj_integral_dev, void* hip_stream);

/*
 * Largest window mean of each row: fmax_dev[r] = max_t (1/window) sum of
 * series[r][t-window+1 .. t] over the windows inside the row (paper Section
 * 3.2, time-averaged drag).  FP64 running sums; prefix_scratch_dev is device
 * double[rows][len+1].
 */
int window_mean_max(const float* series_dev, int32_t rows, int32_t len, int32_t window,
                    double* prefix_scratch_dev, double* fmax_dev, void* hip_stream);

/*
 * prob_dev[q] = (1/n) sum_j exp(log_weight_dev[j]) [fmax_dev[j] >= levels_dev[q]],
 * summed in index order in FP64 (all log-weights 0 gives the direct-sampling
 * estimate).  The return time follows as r = -(T_a - T) / ln(1 - p).
 */
int tail_probability(const double* fmax_dev, const double* log_weight_dev, int32_t n,
                     const double* levels_dev, int32_t n_levels, double* prob_dev, void* hip_stream);

/*
 * SCGF estimate of a GKTL run (paper Appendix C.1): out_dev[0] =
 * (1/t_a) sum_i ln_r_dev[i], the sum in period order in FP64; t_a the
 * simulated time (T_a, in the units the caller wants lambda in).  ln_r_dev:
 * device double[n_periods] as written by gktl_select_clone; out_dev: device
 * double[1].  LBM_EINVAL for n_periods < 1 or t_a not finite and > 0.
 */
int gktl_scgf(const double* ln_r_dev, int32_t n_periods, double t_a, double* out_dev, void* hip_stream);

/*
 * Return times from probabilities (paper Appendix C.2): for a block of length
 * t_a and windows of length `window` (the time-averaged observable; 0 for a
 * plain observable), r_dev[q] = -(t_a - window) / ln(1 - prob_dev[q]) in FP64
 * (log1p); +inf where the probability is 0, 0 where it is 1.  Device
 * double[n] each (NULL allowed for n = 0).  LBM_EINVAL unless 0 <= window <
 * t_a, both finite.
 */
int return_times(const double* prob_dev, int32_t n, double t_a, double window, double* r_dev, void* hip_stream);

/*
 * Unbiased AMS estimate of P(max >= a) (paper Appendix B: the estimator of
 * trajectory AMS): prob_dev[q] = prod_j (1 - k_history_dev[j] / n) (in
 * iteration order) times (1/n) #{m : final_max_dev[m] >= levels_dev[q]}, in
 * FP64.  k_history_dev: device int32[n_iter], the trajectories discarded at
 * each iteration (NULL if n_iter = 0); final_max_dev: device double[n], the
 * maxima of the final ensemble; levels_dev, prob_dev: device double[n_levels]
 * (NULL allowed for n_levels = 0).  Valid for levels at or above the one every
 * trajectory reached when the run stopped.  LBM_EINVAL for n < 1 or negative
 * sizes.
 */
int ams_probability(const int32_t* k_history_dev, int32_t n_iter, int32_t n, const double* final_max_dev,
                    const double* levels_dev, int32_t n_levels, double* prob_dev, void* hip_stream);

/*
 * AMS score built from a learned prediction ghat for the target event
 * {max_t F_T(t) >= level} (F_T: time-averaged drag; paper Section 4.1: the
 * score may be any function of the state that reaches the level exactly when
 * the event happens).  out = level where ft >= level; elsewhere the
 * prediction mapped strictly increasingly into (-inf, level):
 *   out = level - width * ln(1 + exp((level - ghat) / width)),
 * computed in FP64, rounded to FP32 and held at or below the float just under
 * the level; -inf for a non-finite ghat.  The map follows ghat far below the
 * level (within width * exp(-(level - ghat)/width)) and approaches the level
 * from below as ghat grows past it, so predictions above the level keep
 * their order (FP32 resolves them until ghat exceeds the level by about
 * width * ln(width / ulp(level))) instead of tying, and max_t out >= level
 * exactly when the event happened.  All arrays device float[count]; level
 * finite, width finite and > 0.
 */
int ams_learned_score(const float* ghat_dev, const float* ft_dev, int64_t count, float level, float width,
                      float* out_dev, void* hip_stream);

/*
 * Learned AMS score (the paper's conclusion proposes learning the score
 * function).  A small network maps a 3 x 16 x 16 picture of the near wake to
 * one number: three zero-padded 3x3 convolutions with 32 output channels and
 * ReLU, a global average over the 16 x 16 positions and a linear read-out.
 * Parameters are one FP32 vector (score_net_params() floats) in the order
 * w1[32][3][3][3], b1[32], w2[32][32][3][3], b2[32], w3[32][32][3][3], b3[32],
 * w4[32], b4; convolution weights [out][in][dy][dx] act as cross-correlation.
 * The convolutions run on BF16 matrix cores: weights and layer inputs are
 * rounded to BF16 (nearest even), sums are FP32.
 */
int32_t score_net_params(void);

/*
 * Device workspace (256-byte aligned) score_net_forward / score_net_grad need
 * for a batch; it serves every smaller batch too (the size never decreases
 * with the batch).
 */
size_t score_net_workspace_bytes(int32_t batch);

/*
 * Input pictures of the learned AMS score (the score function of Section 4.1
 * learned from the flow state, as the Conclusion proposes).
 * Features of members m0 .. m0+n-1 from their current states: u_x * u_scale,
 * u_y * u_scale and (rho - 1) * rho_scale averaged over pool x pool blocks of
 * the patch x patch cells whose lower-left cell is (px0, py0); rho and u are
 * those of the step the state belongs to (u = (sum c_i f_i - F/2) / rho from
 * the post-collision populations); obstacle cells count as rho = 1, u = 0.
 * out_dev: device float[n][3][patch/pool][patch/pool], patch/pool <= 16.
 */
int score_features(const lbm_ctx* ctx, int32_t m0, int32_t n, int32_t px0, int32_t py0, int32_t patch,
                   int32_t pool, double u_scale, double rho_scale, float* out_dev);

/*
 * score_features for the members the ensemble currently steps (AMS scores the
 * trajectories it re-simulates after a branching, Appendix B.1; the mask of
 * lbm_set_active; every member before any mask is set, after lbm_init and
 * after a NULL mask): row r of out_dev is the r-th active member in
 * ascending member order, with the same arithmetic as score_features.  The
 * number of rows (the active count) goes to *n_rows (host, may be NULL),
 * also when the output is too small.  out_dev: device float[max_rows][3][patch/pool]
 * [patch/pool] (may be NULL when no member is active).  LBM_EINVAL, with
 * nothing written, when more than max_rows members are active or the patch
 * does not lie inside every active member.
 * Async on the ensemble's stream; reads the mask the last lbm_set_active
 * queued on it.
 */
int score_features_active(const lbm_ctx* ctx, int32_t px0, int32_t py0, int32_t patch, int32_t pool,
                          double u_scale, double rho_scale, float* out_dev, int32_t max_rows, int32_t* n_rows);

/* y_dev[b] = network(x_dev[b]) for a batch of device float[batch][3][16][16]. */
int score_net_forward(const float* params_dev, const float* x_dev, int32_t batch, float* y_dev,
                      void* workspace, size_t workspace_bytes, void* hip_stream);

/*
 * Gradient of the mean squared error (1/B) sum_b (y_b - label_b)^2 with
 * respect to every parameter (device float[score_net_params()]), and the loss
 * into loss_dev (device float, may be NULL).  Deterministic for a given batch
 * size: the images are taken k at a time (k = batch / 2048 clamped to 1..8),
 * each group's contributions added in image order into one row; the rows are
 * added in order within chunks of c rows, c the smallest power of two from 8
 * to 256 with c * c >= the number of rows (16 at a batch of 256), then the
 * chunk sums in chunk order; the loss by a fixed-order tree.
 */
int score_net_grad(const float* params_dev, const float* x_dev, const float* labels_dev, int32_t batch,
                   float* grads_dev, float* loss_dev, void* workspace, size_t workspace_bytes, void* hip_stream);

/*
 * score_net_grad for callers that cannot allocate device memory: code under
 * HIP graph capture, tight training or serving loops, harnesses that forbid
 * hipMalloc.  Same kernels, arguments and results as score_net_grad (bit for
 * bit), but the workspace is a static array of the library (31 MiB, the
 * workspace of a batch of 256 images) that every GPU the library runs on
 * holds until the process ends; no call allocates or frees anything.
 * batch in [1, 256], else LBM_EINVAL.  The first call on each device looks
 * up that device's copy of the array (hipGetSymbolAddress; make it outside
 * any graph capture); later calls only enqueue kernels on hip_stream, which
 * must belong to the current device.  All calls on one device share its
 * array: calls that overlap in time on one device race (serialise them, for
 * instance on one stream).  Nothing in the array needs clearing: each call
 * writes every part of it that it reads.
 */
int score_net_grad_noalloc(const float* params_dev, const float* x_dev, const float* labels_dev, int32_t batch,
                           float* grads_dev, float* loss_dev, void* hip_stream);

/* One Adam step (Kingma & Ba, bias-corrected, step >= 1) on FP32 parameters with moments m, v. */
int score_net_adam(float* params_dev, float* m_dev, float* v_dev, const float* grads_dev, int32_t step,
                   double lr, double beta1, double beta2, double eps, void* hip_stream);

/* Message of the last failed call on this thread ("" if none). */
const char* lbm_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* MI355X_LBM_H */
