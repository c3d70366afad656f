/*
 * exx.h -- C ABI of the MI355X exact-exchange library (libexx.so).
 *
 * The library evaluates, for one spin channel of real (or, with
 * EXX_PLAN_COMPLEX, complex) orbitals psi_i on a uniform cubic grid with
 * occupations f_i,
 *
 *   rho_ij(r) = conj(psi_j(r)) psi_i(r)          (co-density, Eq. 2; Eq. 8 for real psi)
 *   V_ij      = solution of lap V = -4 pi rho_ij         (pair potential, Eq. 4)
 *   E_x       = -1/2 sum_{i,j} f_i f_j h^3 sum_r Re(conj(rho_ij) V_ij)     (Eq. 5)
 *   (K psi)_i = sum_j f_j V_ij psi_j         (minus the Fock action D_X, Eq. 3)
 *
 * (V_ji = conj(V_ij), so the sum over unordered pairs covers every term.)
 * A spin-polarized system is two calls (or a batch of two systems), one per
 * spin channel with its own orbitals and occupations f_i,sigma (Eq. 2).
 *
 * following Ratcliff et al., arXiv:1712.07973, Section 2 (the pair-sum
 * scheme with one Poisson solve per unordered pair, N(N+1)/2 solves) and
 * Section 2.1.2 (Poisson solve by FFT convolution with a Green's kernel,
 * zero padding for isolated systems).
 *
 * Conventions shared by every entry point
 *   - grid point (ix,iy,iz), 0 <= i < n, sits at r = (hx ix, hy iy, hz iz);
 *   - psi and K psi are FP64, C-contiguous [n_orb][n][n][n] with x fastest,
 *     in DEVICE memory, 16-byte aligned;  occ is FP64 [n_orb] in device memory;
 *     with EXX_PLAN_COMPLEX every psi and K psi value is an interleaved (re, im)
 *     pair of FP64, [n_orb][n][n][n][2] (C99 double complex / complex128);
 *   - periodic boundary: FFT grid n^3, kernel 4 pi / |G|^2 with G = 0 dropped;
 *   - free boundary: FFT grid (2n)^3 with the data in the first octant, kernel
 *     4 pi (1 - cos |G| R) / |G|^2 (value 2 pi R^2 at G = 0), potential cropped
 *     back to n^3; R <= 0 selects R = min(n hx, n hy, n hz), the largest radius
 *     free of periodic images on the doubled grid;
 *   - G = 2 pi k / (m h) per axis with k folded to (-m/2, m/2].
 *
 * Ownership: the caller owns psi, occ, every output and the workspace; the
 * library owns only plans and batches (host objects plus small device tables)
 * and never allocates inside exx_compute / exx_batch_compute, except the
 * per-orbital-count schedule that exx_plan_prepare builds (see there).
 *
 * Errors: every entry point returns EXX_OK (0) or a negative EXX_ERR_* code;
 * arguments are validated before any HIP call; nothing aborts or throws across
 * the ABI.  exx_last_error() gives a thread-local message for the last failure.
 *
 * Streams: every compute call is stream-ordered on the given hipStream_t
 * (passed as void*, NULL = the default stream), never synchronises the host
 * and can be captured into a HIP graph once its schedule is prepared.
 */
#ifndef EXX_H
#define EXX_H

#include <stddef.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- enumerations ------------------------------------------------------ */
/* Boundary conditions (Section 2.1.2 lists free, surface and periodic ones).
 *   PERIODIC: periodic in x, y, z; kernel 4 pi / G^2, G = 0 dropped;
 *   FREE    : isolated; zero padding to 2n per axis, Coulomb cut at |r| = R;
 *   SURFACE : periodic in x and y, isolated along z; zero padding to 2n along
 *             z only, Coulomb cut at |z| = R:
 *               4 pi / G^2 [1 + e^{-Gp R} (Gz / Gp sin(Gz R) - cos(Gz R))], Gp > 0,
 *               4 pi / Gz^2 [1 - cos(Gz R) - Gz R sin(Gz R)],  Gp = 0 (the in-plane
 *               G = 0 part is the transform of -2 pi |z|), -2 pi R^2 at G = 0,
 *             with Gp the in-plane and Gz the normal wave vector;
 *   WIRE    : isolated in x and y, periodic along z; zero padding to 2n in x and y,
 *             Coulomb cut at in-plane distance rho = R:
 *               4 pi / G^2 [1 + R (Gp J1(Gp R) K0(|Gz| R) - |Gz| J0(Gp R) K1(|Gz| R))], Gz != 0,
 *               4 pi / Gp^2 [1 - J0(Gp R) - Gp R J1(Gp R) ln R],  Gz = 0 (the transform of
 *               the 2-D potential -2 ln rho, rho in bohr), pi R^2 (1 - 2 ln R) at G = 0. */
enum exx_bc { EXX_BC_PERIODIC = 0, EXX_BC_FREE = 1, EXX_BC_SURFACE = 2, EXX_BC_WIRE = 3 };

/* Kernel of the pair Poisson problem.  COULOMB is 1/r (Eq. 4; truncated at R
 * for free boundaries).  SCREENED is erfc(omega r)/r, the short-range kernel of
 * screened hybrids: the paper notes only kernel 2's filter changes for them
 * (Section 3.2.3); periodic boundary only.  ISF is the Green's function of the
 * interpolating-scaling-function Poisson solver of Section 2.1.2 (free boundary
 * only; R unused): the density is read as its order-16 Deslauriers-Dubuc
 * interpolant and V is that density's exact Coulomb potential at the grid
 * points, K(d) = hx hy hz int phi(u1) phi(u2) phi(u3) / |H (d - u)| du, applied on
 * the doubled grid (exact: no displacement wraps).  The table is built on the
 * host in FP64 from a 1/r Gaussian expansion (about 0.5 s at n = 128). */
enum exx_kernel { EXX_KERNEL_COULOMB = 0, EXX_KERNEL_SCREENED = 1, EXX_KERNEL_ISF = 2 };

/* Arithmetic path.
 *   FP32      : FP32 FFTs, two real pairs packed per complex transform,
 *               FP64 pair-energy and K psi accumulation (the fast path);
 *   FP64_PLAIN: FP64 throughout, one pair per complex transform, one launch per
 *               FFT axis, no packing and no pruning (the reference GPU path);
 *   FP64_FUSED: the FP32 path's fused kernels instantiated in FP64 (ablation;
 *               n <= 96). */
enum exx_precision { EXX_PREC_FP32 = 0, EXX_PREC_FP64_PLAIN = 1, EXX_PREC_FP64_FUSED = 2 };

/* What to compute.  ENERGY alone uses Parseval's identity (one forward
 * transform per pair) unless pair energies are requested; that route folds
 * sqrt(f_i f_j) into the co-densities and so needs f_i >= 0 (a negative f_i
 * counts as 0 there): for signed occupations request pair_e, which takes the
 * route through the potentials (the Python binding does so by itself). */
enum exx_mode { EXX_MODE_ENERGY = 1, EXX_MODE_KPSI = 2, EXX_MODE_ENERGY_KPSI = 3 };

/* Flags of exx_compute / exx_batch_compute. */
#define EXX_FLAG_ACCUMULATE 1u /* add into kpsi instead of overwriting it */

/* Flags of exx_plan_create.  COMPLEX: complex orbitals (Eq. 2 with the
 * conjugate): psi and K psi hold interleaved (re, im) FP64 pairs; every pair
 * i <= j is one complex transform (the fused paths cannot pack two pairs per
 * transform, so a complex evaluation costs twice the transforms of a real one);
 * pair energies stay real. */
#define EXX_PLAN_COMPLEX 1u

/* Error codes. */
enum exx_status {
  EXX_OK = 0,
  EXX_ERR_INVALID_ARG = -1,      /* null pointer, non-positive size or spacing, bad enum */
  EXX_ERR_UNSUPPORTED_SIZE = -2, /* n not in {16,32,48,64,80,96,112,128} or n > path limit */
  EXX_ERR_CAPACITY = -3,         /* n_orb above the plan's n_orb_max */
  EXX_ERR_WORKSPACE = -4,        /* workspace missing or smaller than required */
  EXX_ERR_ALIGNMENT = -5,        /* psi / kpsi / workspace not 16-byte aligned */
  EXX_ERR_HIP = -6,              /* a HIP runtime call failed (message has the hipError_t) */
  EXX_ERR_NOT_PREPARED = -7,     /* schedule missing for this n_orb while capturing */
  EXX_ERR_INTERNAL = -8
};

/* ---- plans --------------------------------------------------------------- */
typedef struct exx_grid {
  int nx, ny, nz;    /* grid points per axis; must be equal (cubic grid) */
  double hx, hy, hz; /* spacings in bohr, > 0 */
  int bc;            /* enum exx_bc */
  int kernel;        /* enum exx_kernel */
  double R;          /* truncation radius (FREE: |r|, SURFACE: |z|, WIRE: in-plane
                        distance); <= 0 selects the box length n h */
  double omega;      /* screening parameter for EXX_KERNEL_SCREENED (> 0) */
} exx_grid;

typedef struct exx_plan exx_plan;

/* Creates a plan for one grid and precision on the current HIP device: FFT
 * twiddles (computed in FP64 on the host, rounded once), the Green's kernel
 * table (FP64 on the host), and the default pair-tile schedule.  n_orb_max
 * bounds every later n_orb.  flags: 0 (real orbitals) or EXX_PLAN_COMPLEX;
 * other bits give EXX_ERR_INVALID_ARG.  Allocates device memory; synchronous. */
int exx_plan_create(exx_plan** out, const exx_grid* grid, int precision, int n_orb_max,
                    unsigned flags);
void exx_plan_destroy(exx_plan* plan);

/* Builds (once per n_orb) the device-side pair schedule used by exx_compute.
 * exx_compute calls it implicitly; call it yourself before capturing a graph.
 * Allocates device memory; synchronous. */
int exx_plan_prepare(exx_plan* plan, int n_orb);

/* Bytes of device workspace exx_compute needs for n_orb orbitals. */
int exx_workspace_bytes(const exx_plan* plan, int n_orb, size_t* bytes);

/* Evaluates the exchange for n_orb orbitals.
 *   psi    [n_orb][n][n][n] FP64 (complex plan: (re, im) pairs), device;
 *          occ [n_orb] FP64, device (f_i >= 0);
 *   mode   enum exx_mode;  flags EXX_FLAG_*;
 *   ex_out device FP64 scalar receiving E_x (Hartree); required if mode has ENERGY;
 *   kpsi   device FP64 like psi receiving (K psi)_i; required if mode has KPSI;
 *   pair_e device FP64 [n_orb][n_orb] receiving e_ij = h^3 sum_r Re(conj(rho_ij) V_ij)
 *          (real and symmetric, both triangles written), or NULL;
 *   ws     device workspace of ws_bytes >= exx_workspace_bytes(), 256-byte aligned;
 *   stream hipStream_t or NULL.
 * Outputs are complete when the stream reaches the end of the call. */
int exx_compute(exx_plan* plan, const double* psi, const double* occ, int n_orb, int mode,
                unsigned flags, double* ex_out, double* kpsi, double* pair_e, void* ws,
                size_t ws_bytes, void* stream);

/* Gradient of E_x for reverse-mode differentiation (Eq. 3 and Eq. 5: E_x is a
 * quartic in the orbitals and a quadratic in the occupations).
 *   gbar     device FP64 scalar: the derivative of the caller's loss with
 *            respect to E_x (read on the device, so no host sync is needed);
 *   grad_psi device FP64 like psi, overwritten with
 *            gbar dE_x/dpsi_k(r) = -2 gbar f_k h^3 (K psi)_k(r); for a complex
 *            plan, the derivative with respect to Re psi plus i times the one
 *            with respect to Im psi;
 *   grad_occ device FP64 [n_orb] or NULL: gbar dE_x/df_k = -gbar sum_j f_j e_kj;
 *   pair_e   device FP64 [n_orb][n_orb], required with grad_occ (it receives the
 *            pair energies e_kj), ignored without;
 * psi, occ, n_orb, ws, ws_bytes and stream as exx_compute (the evaluation is
 * exx_compute in KPSI mode, recomputing every pair potential; signed
 * occupations are allowed).  Errors as exx_compute, plus EXX_ERR_INVALID_ARG
 * for a missing gbar or grad_psi, or grad_occ without pair_e. */
int exx_gradient(exx_plan* plan, const double* psi, const double* occ, int n_orb,
                 const double* gbar, double* grad_psi, double* grad_occ, double* pair_e, void* ws,
                 size_t ws_bytes, void* stream);

/* exx_compute without any allocation, for callers that cannot allocate (code
 * under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc).  Same arguments, results and stream ordering as exx_compute, but
 * the workspace is the library's own static device array of
 * EXX_NOALLOC_SCRATCH_BYTES per GPU (held from the library's first use of that
 * GPU to the end of the process), and nothing is allocated: the plan's
 * schedule for n_orb must already exist (exx_plan_prepare, or an earlier
 * exx_compute), else EXX_ERR_NOT_PREPARED; profiling events are not recorded.
 * The current device must be the plan's.  A problem whose workspace
 * (exx_workspace_bytes) exceeds the maximum gives EXX_ERR_WORKSPACE with the
 * sizes in exx_last_error(); lower the plan's batch_slots (exx_plan_set_tuning,
 * then exx_plan_prepare) to fit.  Every call on a GPU uses the same array:
 * calls that overlap on one GPU (other streams, other threads) race, and the
 * array keeps the last call's contents (no part of it needs clearing). */
#define EXX_NOALLOC_SCRATCH_BYTES (64u << 20)
int exx_compute_noalloc(exx_plan* plan, const double* psi, const double* occ, int n_orb,
                        int mode, unsigned flags, double* ex_out, double* kpsi, double* pair_e,
                        void* stream);

/* Tuning knobs of a plan (pair-tile edge, slots per launch, slab workgroup
 * size, pass streams).  Returned by exx_autotune and settable explicitly;
 * a field left 0 keeps the plan's value.  Every setting gives the same
 * results bit for bit except `tile`, which changes the summation order. */
typedef struct exx_tuning {
  int tile;         /* orbitals per pair-tile edge (2..16) */
  int batch_slots;  /* packed pair slots per pass launch (>= 1) */
  int slab_threads; /* threads per slab workgroup of the y/z pass (256 or 512 at n = 64) */
  int streams;      /* 1: every pass on the caller's stream, one launch per pass and chunk;
                       3: per round of pair tiles, the pair-build pass, the y/z pass and the
                       reduction pass run on three streams, so that the memory-bound passes
                       of one round overlap the y/z pass of another (fused paths only) */
  int slab_form;    /* enum exx_slab_form: how the y/z pass works through a slab */
} exx_tuning;

/* Forms of the y/z pass (exx_tuning.slab_form).
 *   SHARED: the workgroup shares every line exchange through LDS behind
 *           workgroup barriers (two slab buffers where they fit, else three
 *           launches through a scratch of y-transformed slabs);
 *   WAVE  : one slab buffer; a wavefront owns whole lines in each phase, so line
 *           exchanges synchronise one wavefront only and two workgroup barriers
 *           per y class remain (FP32: every n; FP64_FUSED: n <= 80). */
enum exx_slab_form { EXX_SLAB_SHARED = 1, EXX_SLAB_WAVE = 2 };

int exx_plan_get_tuning(const exx_plan* plan, exx_tuning* out);
int exx_plan_set_tuning(exx_plan* plan, const exx_tuning* t);

/* Times candidate tunings for n_orb orbitals with hipEvents on `stream` using
 * the caller's psi/occ/kpsi/ws buffers, keeps the fastest, and if cache_path is
 * non-NULL reads/writes a small text cache keyed by GPU arch, grid, boundary,
 * precision and n_orb.  budget_ms bounds the search's wall time: no new
 * candidate starts once it is spent (<= 0: 20 s).  Synchronises the stream. */
int exx_autotune(exx_plan* plan, const double* psi, const double* occ, int n_orb, double* kpsi,
                 void* ws, size_t ws_bytes, void* stream, int budget_ms, const char* cache_path);

/* ---- batches of independent systems ------------------------------------- */
typedef struct exx_system {
  const double* psi; /* [n_orb][n][n][n] FP64, device */
  const double* occ; /* [n_orb] FP64, device */
  double* ex_out;    /* device FP64 scalar or NULL */
  double* kpsi;      /* device FP64 like psi, or NULL */
  double* pair_e;    /* device FP64 [n_orb][n_orb] or NULL */
} exx_system;

typedef struct exx_batch exx_batch;

/* Flags of exx_batch_create. */
#define EXX_BATCH_GRAPH 1u   /* capture the evaluation into a HIP graph and replay it */
#define EXX_BATCH_COMPLEX 2u /* every system has complex orbitals (as EXX_PLAN_COMPLEX) */
#define EXX_BATCH_MERGE 4u   /* shared launches per grid class (below) */

/* A batch of n_systems independent systems (any mix of supported grids and
 * orbital counts, one precision, all real or all complex orbitals; e.g. the
 * two spin channels of a spin-polarized system, Eq. 2's sum over sigma).  Each
 * system keeps its own plan (kernels are specialised per grid size); the
 * systems are issued on a few side streams forked from `stream` (largest
 * first) so that they overlap, and joined back.  With EXX_BATCH_GRAPH the
 * whole evaluation is captured into one HIP graph on the first
 * exx_batch_compute and replayed afterwards, one graph launch per call (the
 * system pointers, mode, flags, workspace and stream must then stay the same;
 * a change recaptures).  Unknown flag bits give EXX_ERR_INVALID_ARG.
 *
 * EXX_BATCH_MERGE (FP32 only): systems on the same grid (size, spacing,
 * boundary, kernel, radius) form a class of up to 32 systems that share
 * launches: their pair schedules are merged (the round-robin rounds of tile
 * pairs of every member, round by round, Sec. 2.1), so one pass-A and one
 * pass-B launch cover a chunk of all members' slots and one pass-C launch a
 * round of all members' tile pairs; the classes run on the side streams.
 * Results equal the unmerged batch's bit for bit.  A merged batch evaluates
 * EXX_MODE_KPSI and EXX_MODE_ENERGY_KPSI without pair energies (pair_e NULL);
 * other calls, and exx_batch_autotune, give EXX_ERR_INVALID_ARG.  It sizes its
 * workspace per class rather than per system. */
int exx_batch_create(exx_batch** out, const exx_grid* grids, const int* n_orb, int n_systems,
                     int precision, unsigned flags);
void exx_batch_destroy(exx_batch* batch);
int exx_batch_workspace_bytes(const exx_batch* batch, size_t* bytes);
int exx_batch_compute(exx_batch* batch, const exx_system* systems, int mode, unsigned flags,
                      void* ws, size_t ws_bytes, void* stream);

/* Autotunes a batch: its systems are grouped by grid (same kernels and kernel
 * table); exx_autotune runs on each group's member with the most orbitals, on
 * that system's psi, occ and (as scratch) K psi buffers and its share of ws,
 * with budget_ms split over the groups, and the winning tuning is applied to
 * every member of the group whose share of the workspace holds it.  The
 * workspace size does not change.  Synchronises the stream; a graph captured
 * earlier is captured again on the next exx_batch_compute. */
int exx_batch_autotune(exx_batch* batch, const exx_system* systems, void* ws, size_t ws_bytes,
                       void* stream, int budget_ms, const char* cache_path);
/* The tuning of system `system`'s plan (0 <= system < n_systems). */
int exx_batch_get_tuning(const exx_batch* batch, int system, exx_tuning* out);

/* ---- profiling ----------------------------------------------------------- */
/* Per-pass device time measured with hipEvents recorded on the compute stream
 * around every kernel launch of exx_compute (not while a graph is captured).
 * Pass kinds index ms[] / launches[]: */
enum exx_pass_kind {
  EXX_PASS_CONVERT = 0, /* FP64 -> FP32 orbital copy */
  EXX_PASS_ZERO = 1,    /* clearing accumulators */
  EXX_PASS_A = 2,       /* co-densities + forward x-transform */
  EXX_PASS_B = 3,       /* y/z transforms, kernel multiply, inverse y/z */
  EXX_PASS_C = 4,       /* inverse x-transform, pair energies, K psi */
  EXX_PASS_FINALIZE = 5,
  EXX_PASS_PLAIN_FFT = 6,   /* plain path: one axis transform */
  EXX_PASS_PLAIN_OTHER = 7, /* plain path: build, kernel multiply, reduce */
  EXX_PASS_KINDS = 8
};
typedef struct exx_pass_times {
  double ms[EXX_PASS_KINDS];
  long long launches[EXX_PASS_KINDS];
} exx_pass_times;

/* Enables (1) or disables (0) event recording for later exx_compute calls. */
int exx_plan_enable_profiling(exx_plan* plan, int enable);
/* Waits for the recorded events, returns the accumulated times since the last
 * read and resets them. */
int exx_plan_read_profile(exx_plan* plan, exx_pass_times* out);

/* ---- diagnostics --------------------------------------------------------- */
const char* exx_error_string(int code);
const char* exx_last_error(void);
/* Pair count N(N+1)/2 and packed-slot count of the plan's schedule for n_orb. */
int exx_plan_schedule_info(exx_plan* plan, int n_orb, long long* n_pairs, long long* n_slots);
/* Library version, e.g. "exx 0.1 gfx950". */
const char* exx_version(void);

#ifdef __cplusplus
}
#endif
#endif /* EXX_H */
