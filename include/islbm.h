/*
 * islbm.h -- C-ABI of the MI355X (gfx950) interpolation-supplemented lattice
 * Boltzmann solver for buoyancy-driven convection in a side-heated cavity.
 *
 * Method: Xu, Zhao, Xu & Jiang, "Interpolation-supplemented lattice
 * Boltzmann simulation of thermal convection on non-uniform meshes"
 * (IJHMT 2025).  One call of islbm_step advances the double-distribution
 * MRT model (Sec. 2.1) by whole time steps: pull-streaming onto a stretched
 * tensor-product mesh by quadratic interpolation at the departure points
 * x - e_i dt (Sec. 2.2), the half-way wall rules (Sec. 2.3), then the MRT
 * collision of the flow (D2Q9 / D3Q19, Guo forcing) and temperature
 * (D2Q5 / D3Q7) populations.  Each time step is one fused kernel launch.
 *
 * Conventions shared by every entry point
 *  - Axes: x (index i, fastest), y (j), z (k).  Gravity acts along -y, so the
 *    buoyancy force is F = rho g beta (T - T0) along +y.  The isothermal walls
 *    are x = min (T_hot) and x = max (T_cold); all other walls are adiabatic;
 *    every wall is no-slip (Sec. 3 and Sec. 4 problem statements).
 *  - Mesh: per axis a, n[a] fluid nodes with coordinates x_1..x_N plus the
 *    ghost mirrors x_0 and x_{N+1}; the walls sit half-way between x_0,x_1 and
 *    x_N,x_{N+1} (Sec. 2.3, Fig. 2, Eq. (erf)).  spacing[a] holds n[a]+1
 *    entries, spacing[a][m] = x_{m+1} - x_m.  The first and last entries are
 *    the lattice unit Delta and must be equal on every axis (one time step is
 *    shared); no entry may be smaller than Delta (relative 1e-12).
 *    The characteristic length is H = (wall-to-wall height along y)/Delta
 *    (Table 1).
 *  - Populations on the host are double arrays [q][n_z][n_y][n_x], x fastest,
 *    in these velocity orderings:
 *      D2Q9 : 0 (0,0); 1 (1,0); 2 (0,1); 3 (-1,0); 4 (0,-1); 5 (1,1);
 *             6 (-1,1); 7 (-1,-1); 8 (1,-1)
 *      D2Q5 : 0 (0,0); 1 (1,0); 2 (0,1); 3 (-1,0); 4 (0,-1)
 *      D3Q19: 0; 1 +x; 2 -x; 3 +y; 4 -y; 5 +z; 6 -z; 7 (1,1,0); 8 (-1,-1,0);
 *             9 (1,-1,0); 10 (-1,1,0); 11 (1,0,1); 12 (-1,0,-1); 13 (1,0,-1);
 *             14 (-1,0,1); 15 (0,1,1); 16 (0,-1,-1); 17 (0,1,-1); 18 (0,-1,1)
 *      D3Q7 : 0; 1 +x; 2 -x; 3 +y; 4 -y; 5 +z; 6 -z
 *  - The state kept between calls is the post-collision population set
 *    f+(x,t), g+(x,t) (Sec. 2.1, collision step), held on the device as
 *    deviations f - w_i (flow) and g (thermal), in x-rows: for every (z, y)
 *    row of the mesh the rows of all populations of a set lie one after
 *    another ([z][y][pop][x], padded row pitch).
 *  - Every call returns 0 on success or a negative islbm_status.  Out
 *    parameters are untouched on error.  Calls on one context are not
 *    thread-safe; distinct contexts are independent.  Work is enqueued on the
 *    context's HIP stream; calls that return host data synchronise it.
 */
#ifndef ISLBM_H
#define ISLBM_H

#include <stddef.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct islbm_ctx islbm_ctx;

typedef enum {
  ISLBM_OK = 0,
  ISLBM_EINVAL = -1,     /* NULL pointer, n < 3, Ra or Pr <= 0, unknown enum */
  ISLBM_EMESH = -2,      /* spacing violates the mesh convention above       */
  ISLBM_EPARAM = -3,     /* parameters outside the stable range (a_T > 1)    */
  ISLBM_ENOMEM = -4,     /* device or host allocation failed                 */
  ISLBM_EDEVICE = -5,    /* HIP runtime error, or no usable gfx950 device     */
  ISLBM_ENONFINITE = -6  /* the last reduction met a non-finite node         */
} islbm_status;

typedef enum { ISLBM_D2Q9_D2Q5 = 2, ISLBM_D3Q19_D3Q7 = 3 } islbm_lattice;

/* Storage type of the populations in HBM.  Arithmetic is FP32 for FP32,
 * FP16DEV and BF16DEV (deviations f - w_i and g stored in half / bfloat16;
 * FP16 scaled by 2^12, so it holds deviations up to 16 in magnitude), and
 * FP64 for FP64 and FP32SR (FP32 storage, FP64 arithmetic).  The time step
 * writes FP16DEV / BF16DEV / FP32SR with stochastic rounding (expected stored
 * value = the unrounded result), its random bits a hash of node, population
 * and a device-side step counter; all other conversions round to nearest. */
typedef enum {
  ISLBM_FP32 = 0,
  ISLBM_FP64 = 1,
  ISLBM_FP16DEV = 2,
  ISLBM_BF16DEV = 3,
  ISLBM_FP32SR = 4
} islbm_storage;

typedef struct {
  double u_f;            /* free-fall velocity in lattice units per step; 0 => Ma = 0.1,
                            u_f = 0.1/sqrt(3) (Sec. 3, reference velocity)          */
  double T_hot, T_cold;  /* wall temperatures, used as given (islbm_default_options and a
                            NULL options pointer give +0.5 / -0.5).  The buoyancy
                            reference is T0 = (T_hot + T_cold)/2, Delta_T = T_hot - T_cold
                            (1 when the two are equal)                               */
  double s_e, s_eps, s_q, s_pi, s_m;  /* flow rates; 0 => s_e = s_eps = s_pi = s_nu,
                            s_q = s_m = 8(2 - s_nu)/(8 - s_nu)                      */
  double q_j, q_e, q_nu; /* thermal rates; 0 => q_j = 3 - sqrt(3), q_e = q_nu = 4 sqrt(3) - 6 */
  int storage;           /* islbm_storage; default ISLBM_FP32                        */
  void* stream;          /* hipStream_t to enqueue on; NULL => the library's own      */
  void* buffers[4];      /* optional caller-owned device buffers fA, fB, gA, gB, each at
                            least the sizes from islbm_query_bytes; all four or none */
  int allow_unstable;    /* 0 => ISLBM_EPARAM when a_T > 1 (negative rest weight of the
                            thermal equilibrium); 1 => accept                         */
  int stream_only;       /* 1 => collision is the identity (diagnostic of the streaming
                            and wall rules alone)                                    */
  int no_graph;          /* 1 => never replay step batches through a HIP graph       */
  int force_interp;      /* 1 => use the interpolating kernel even when every weight is
                            one-hot (uniform mesh); 0 => the plain-shift kernel there  */
} islbm_options;

/* Result of the reductions (Sec. 3 and Sec. 4 definitions; Eqs. (16)-(18)):
 * nu_vol = sqrt(Ra Pr) <u* T*>_V + 1; nu_hot / nu_cold = -<d(T*)/d(x*)> on the
 * isothermal walls (Eq. (17) one-sided derivative, q = second/first spacing);
 * nu_mid = <sqrt(Ra Pr) u* T* - d(T*)/d(x*)> on the mid-plane x* = 1/2 (quadratic
 * through the nearest three nodes, average of the two candidates when they
 * tie); re_vol = sqrt(Ra/Pr) <|u*|>_V over all velocity components, re_uv the
 * same with (u*, v*) only; mass = sum rho V / Delta^d (midpoint volumes,
 * Eq. (18)); rho_sum = plain sum of rho; umax/vmax/wmax = max |u*|, |v*|,
 * |w*|; nonfinite = number of nodes with a non-finite rho, u or T;
 * re_rms = sqrt(Ra/Pr) sqrt(<|u*|^2>_V) (Reynolds number of the root-mean-
 * square velocity).  Averages use midpoint weights normalised by the
 * wall-to-wall extent (Sec. 2.3). */
typedef struct {
  double nu_vol, nu_hot, nu_cold, nu_mid, re_vol, re_uv, mass, rho_sum;
  double umax, vmax, wmax;
  long long nonfinite;
  long long step;        /* time level t of the state the statistics describe */
  double re_rms;
} islbm_stats;

/* Default options (all fields as described above). */
void islbm_default_options(islbm_options* opt);

/* Bytes of one flow buffer and one thermal buffer for a lattice, mesh size
 * and storage type (caller-provided buffers must be at least this large). */
int islbm_query_bytes(int lattice, const int n[3], int storage, size_t* f_bytes,
                      size_t* g_bytes);

/* Node coordinates helper (Sec. 2.3): writes n+1 spacings of a mesh of n
 * fluid nodes on [0,1]: kind 0 uniform (Eq. (14) with ghost mirrors),
 * 1 error-function stretching with coefficient a (Eq. (erf)), 2 cosine
 * x_j = (1 - cos(pi j/(n+1)))/2, 3 tanh x_j = (tanh(a(j/(n+1) - 1/2))/tanh(a/2) + 1)/2. */
int islbm_mesh_spacing(int kind, int n, double a, double* spacing);

/* Creates a context on the current HIP device: validates the mesh, derives
 * nu = u_f H sqrt(Pr/Ra), alpha = u_f H / sqrt(Ra Pr), g beta = u_f^2 / (H dT),
 * s_nu = 1/(3 nu + 1/2), a_T (20 sqrt3 alpha - 4 or 42 sqrt3 alpha - 6) and
 * the anti-bounce-back weight ((4 + a_T)/10 or (6 + a_T)/21), builds the
 * per-axis interpolation tables, and initialises the state at rest with T = 0
 * inside (f_i = w_i, g_i = 0).  n[2] is ignored for the 2-D lattice.
 * On failure *out = NULL and islbm_last_error(NULL) describes the cause. */
int islbm_create(islbm_ctx** out, int lattice, const int n[3],
                 const double* const spacing[3], double Ra, double Pr,
                 const islbm_options* opt);

/* Enqueues nsteps fused time steps (nsteps >= 0; 0 changes nothing).  The
 * last one also writes the FP64 reduction partials used by islbm_nu_re.
 * Runs of at least 128 plain steps are replayed in batches of 64 through a
 * HIP graph that the context captures on first use (one per buffer parity).
 * The plain launches left after the batches (at least 4 of them) are
 * replayed from a graph of their own once the same count recurs from the same
 * buffer parity, or after islbm_plan_steps asked for it; the context keeps
 * four such graphs (a fifth count replaces the oldest, after waiting for the
 * stream).  Options.no_graph = 1 launches every step directly.  Results are
 * bitwise the same either way.  Asynchronous. */
int islbm_step(islbm_ctx* ctx, long long nsteps);

/* Captures, without running a step, the HIP graphs that a following
 * islbm_step(ctx, nsteps) from the current state would replay (the 64-step
 * batch graph and the graph of the remaining plain launches), so that call
 * issues only graph launches and the final, reducing launch.  The first call
 * on a context also launches an empty graph and waits for it, so that the
 * runtime's one-time graph-launch set-up does not fall into the next step
 * call.  Advances no time level.  nsteps >= 0; ISLBM_EINVAL on a null
 * context or negative count, ISLBM_EDEVICE when a capture or the empty
 * launch fails.  A no-op when options.no_graph is set. */
int islbm_plan_steps(islbm_ctx* ctx, long long nsteps);

/* Macroscopic fields at the current time level (pre-collision moments:
 * rho = sum f, u = (sum e f + F/2)/rho, T = sum g) into host arrays of
 * n_x n_y n_z doubles (x fastest).  Any pointer may be NULL (uz ignored in
 * 2-D).  Synchronises the stream. */
int islbm_fields(islbm_ctx* ctx, double* rho, double* ux, double* uy, double* uz, double* T);

/* Same as islbm_fields, into device arrays; asynchronous. */
int islbm_fields_device(islbm_ctx* ctx, double* rho, double* ux, double* uy, double* uz,
                        double* T);

/* Statistics of the current time level (see islbm_stats).  Uses the partials
 * of the last fused step when they describe the current state, else runs a
 * reduction over the stored state.  Synchronises the stream.  Returns
 * ISLBM_ENONFINITE (with *out filled) when a node is non-finite. */
int islbm_nu_re(islbm_ctx* ctx, islbm_stats* out);

/* Steady-state measure of Sec. 3 (the convergence criterion there, with the
 * caller choosing the interval, 2000 steps in the paper): with u, T the
 * current fields (as islbm_fields) and u', T' those of the previous call,
 *   *du = sum_nodes |u - u'|_2 / sum_nodes |u'|_2,
 *   *dT = sum_nodes |T - T'|   / sum_nodes |T'|,
 * summed in FP64 in a fixed order; a zero denominator gives 0 (no change) or
 * +inf.  The current fields then become the snapshot (4 n_x n_y n_z doubles
 * of device memory, allocated on the first call and kept by the context).
 * The first call, and the first after islbm_set_populations,
 * islbm_load_state or islbm_init_fields[_device], only takes the snapshot
 * and returns +inf for both.  *steps (may be NULL) receives the time steps
 * between the two field sets.  Synchronises the stream. */
int islbm_steady_change(islbm_ctx* ctx, double* du, double* dT, long long* steps);

/* Copies the post-collision state to host arrays f [q_f][nodes] and
 * g [q_g][nodes] (either may be NULL).  Synchronises the stream. */
int islbm_get_populations(islbm_ctx* ctx, double* f, double* g);

/* Sets the state from host arrays.  post_collision = 1: the arrays are
 * post-collision populations and are stored as given (checkpoint restore);
 * 0: they are pre-collision populations f(x,t), g(x,t) and are collided
 * first.  The time level is left unchanged. */
int islbm_set_populations(islbm_ctx* ctx, const double* f, const double* g, int post_collision);

/* Size in bytes of the raw state (both population sets in the storage type,
 * then the 4-byte step counter of the stochastic rounding; the checkpoint
 * format of islbm_save_state / islbm_load_state). */
int islbm_state_bytes(const islbm_ctx* ctx, size_t* bytes);

/* Copies the raw post-collision state (storage type, device layout) into a
 * host buffer of at least islbm_state_bytes bytes.  Exact: a state restored
 * with islbm_load_state continues bitwise as the original.  Synchronises. */
int islbm_save_state(islbm_ctx* ctx, void* host, size_t bytes);

/* Restores a state written by islbm_save_state of a context with the same
 * lattice, mesh size and storage type.  The time level is not changed. */
int islbm_load_state(islbm_ctx* ctx, const void* host, size_t bytes);

/* Equilibrium initialisation from host fields (warm start): rho = 1,
 * velocity (ux, uy[, uz]) and temperature T per node; the pre-collision
 * equilibria are collided once and stored.  uz is ignored in 2-D. */
int islbm_init_fields(islbm_ctx* ctx, const double* ux, const double* uy, const double* uz,
                      const double* T);

/* Same as islbm_init_fields, from device arrays; asynchronous. */
int islbm_init_fields_device(islbm_ctx* ctx, const double* ux, const double* uy,
                             const double* uz, const double* T);

/* Derived parameters: lattice unit (input coordinate units), H in lattice
 * units, nu, alpha, a_T, g beta (lattice units).  Any pointer may be NULL. */
int islbm_info(const islbm_ctx* ctx, double* delta, double* H_lu, double* nu, double* alpha,
               double* a_T, double* gbeta);

/* Current time level t (number of steps applied since create). */
long long islbm_time(const islbm_ctx* ctx);

/* Sets the time level (checkpoint restore). */
int islbm_set_time(islbm_ctx* ctx, long long t);

/* Waits for all work enqueued by this context. */
int islbm_sync(islbm_ctx* ctx);

/* Releases the context and library-owned device memory; NULL is a no-op. */
void islbm_destroy(islbm_ctx* ctx);

/* Static description of a status code. */
const char* islbm_strerror(int code);

/* Last error text of a context; NULL => the calling thread's last failed
 * islbm_create. */
const char* islbm_last_error(const islbm_ctx* ctx);

/* Device-side timing of the fused step kernel: enqueues nsteps steps as
 * islbm_step does, bracketed by HIP events on the context's stream, waits,
 * and returns the elapsed milliseconds in *ms. */
int islbm_time_steps(islbm_ctx* ctx, long long nsteps, double* ms);

/* The same with the timed region split at the final launch (the one that also
 * writes the reduction partials): *ms_total for all nsteps launches,
 * *ms_plain for the nsteps - 1 plain launches before it, *ms_reduce for the
 * reducing launch (ms_total - ms_plain).  nsteps >= 1.  Synchronises. */
int islbm_time_steps_split(islbm_ctx* ctx, long long nsteps, double* ms_total, double* ms_plain,
                           double* ms_reduce);

/* Measurement helper, not part of the time step: copies `bytes` bytes from
 * device buffer src to device buffer dst with 16-byte vector loads and stores
 * (a streaming kernel's bandwidth ceiling on this device).  Both pointers
 * 16-byte aligned, bytes a positive multiple of 16, buffers not overlapping;
 * else ISLBM_EINVAL.  Asynchronous on `stream` (a hipStream_t, NULL = default). */
int islbm_copy_bytes(void* dst, const void* src, size_t bytes, void* stream);

#ifdef __cplusplus
}
#endif

#endif /* ISLBM_H */
