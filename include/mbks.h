/*
 * mbks.h - C ABI of the mixed-basis Kohn-Sham operator library for MI355X (gfx950).
 *
 * Basis (paper Sec. II.B.1): phi_{G,i}(r) = A_c^{-1/2} exp(i(k+G).rho) B_i(z), with
 * G an in-plane reciprocal lattice vector and B_i a B-spline of order kappa on a
 * clamped knot sequence (Sec. II.A, eqs. 1-3).  The first and last spline are
 * dropped (hard walls), so with N_int knot intervals there are
 * N_b = N_int + kappa - 3 basis splines.  The discrete problem is the generalized
 * Hermitian eigenproblem H c = eps S c (Sec. II.B.2 form) with
 *   S = I_G (x) S_z                           (overlap elements, Sec. II.B.1)
 *       + sum_p q_p |beta_p><beta_p|          (ultrasoft form, Sec. II.B.2; only when a
 *                                              species carries augmentation charges)
 *   T = 1/2 (D_z + |k+G|^2 S_z) per G         (kinetic elements, Sec. II.B.1; Hartree)
 *   V_loc: Gaussian local potential applied through the in-plane grid
 *          (matrix elements of Sec. II.B.1 with the transform taken on the grid)
 *   V_NL = sum_p E_p |beta_p><beta_p|        (Kleinman-Bylander form, eq. KBeq)
 * Integrals of non-polynomial integrands use a per-interval Gauss-Legendre rule.
 *
 * Units: Hartree atomic units (energies Ha, lengths bohr).
 *
 * Vector layout (all entry points): a block of nbands vectors is one array
 *   x[band][i][G] (G fastest), row stride ld >= N_G complex elements,
 * interleaved complex: complex128 (re, im doubles) for MB_FP64, complex64
 * (re, im floats) for MB_FP32 and MB_BF16X3.  G runs over the library's
 * G-set order of the k-point (see mb_problem_gvectors).  Entries [N_G, ld) of
 * each row are padding: inputs ignore them, outputs set them to zero.
 *
 * Memory and streams: vector pointers are device pointers owned by the caller;
 * the library never frees them.  `stream` is a hipStream_t (NULL = default
 * stream); apply/solve calls are enqueued on it and return without
 * synchronising.  lanczos_lowest synchronises `stream` (it returns host
 * eigenvalues).  A problem handle owns its device tables and one set of work
 * buffers per k-point.  Calls on different k-points of one handle may run
 * concurrently (from different host threads, on different streams); calls on
 * the same k-point must not overlap (issue them on one stream from one thread).
 * On the grids with a plane kernel, H applications with projectors also use a
 * stream of the k-point's own (created with the handle, default priority): it is
 * forked from `stream` and joined back to it by events inside the call, so the
 * call's work is complete, and capturable into a graph, on `stream` alone.
 *
 * Errors: every entry point returns an mb_status; arguments are validated
 * before anything is enqueued.  mb_last_error() returns a thread-local message
 * for the last failure.
 */
#ifndef MBKS_H
#define MBKS_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    MB_OK = 0,
    MB_ERR_INVALID_ARG = -1,  /* a size, pointer or option is outside what the call accepts */
    MB_ERR_NOT_SPD = -2,      /* the overlap S_z (or a preconditioner block) is not positive definite */
    MB_ERR_NOT_CONVERGED = -3,/* lanczos_lowest hit max_iter; outputs hold the last iterate */
    MB_ERR_NONFINITE = -4,    /* a NaN or Inf appeared in the eigensolver's small matrices or residuals */
    MB_ERR_OOM = -5,          /* a device allocation failed */
    MB_ERR_HIP = -6,          /* a HIP runtime call failed */
    MB_ERR_NO_DEVICE = -7     /* the call needs a GPU and the handle was created host-only */
} mb_status;

typedef enum {
    MB_FP64 = 0,   /* complex128 vectors; every step in FP64 */
    MB_FP32 = 1,   /* complex64 vectors; FFT, potential multiply and projector contractions in FP32 */
    MB_BF16X3 = 2  /* complex64 vectors; as MB_FP32 but projector contractions as three BF16 products */
} mb_precision;

#define MB_MAX_GAUSS 4

/* One species: local part sum_t gauss_A[t] exp(-r^2 / gauss_w[t]^2) (the Gaussian
 * terms of the local pseudopotential, Sec. II.B.1) and, if nonlocal != 0, one s and
 * three real Cartesian p Kleinman-Bylander projectors (eq. KBeq; Gaussian radial
 * parts exp(-alpha r^2), normalised to one) with energies E_s, E_p.
 * q_s, q_p: augmentation charges of the s and p projectors in the ultrasoft overlap
 * S = I_G (x) S_z + sum_p q_p |beta_p><beta_p| (Sec. II.B.2, with the charge matrix
 * q_nm of an atom taken diagonal, one charge per projector channel).  Both zero: the
 * norm-conserving problem.  Must be finite and >= 0 (S then stays positive definite);
 * ignored when nonlocal == 0. */
typedef struct {
    int32_t ngauss;
    double gauss_A[MB_MAX_GAUSS];
    double gauss_w[MB_MAX_GAUSS];
    int32_t nonlocal;
    double alpha_s, alpha_p;
    double E_s, E_p;
    double q_s, q_p;
} mb_species;

typedef struct {
    int32_t species;
    double pos[3];   /* Cartesian, bohr */
} mb_atom;

#define MB_GSET_BOX 0
#define MB_GSET_SPHERE 1

/* Problem description.  Pointers are read during mb_problem_create only. */
typedef struct {
    double a1[2], a2[2];          /* in-plane lattice vectors */
    int32_t order;                /* spline order kappa, 2..6 (4 = cubic) */
    int32_t nbreak;               /* number of breakpoints = N_int + 1 >= 2 */
    const double* breakpoints;    /* strictly increasing z_0 < ... < z_Nint */
    int32_t nq;                   /* Gauss points per interval, 1..8 */
    int32_t grid[2];              /* in-plane FFT grid N1 x N2, each 2^a 3^b 5^c, 4..256 */
    int32_t gset_kind;            /* MB_GSET_BOX: |m_i| <= mmax[i]; MB_GSET_SPHERE: 1/2|k+G|^2 <= ecut */
    int32_t mmax[2];
    double ecut;
    int32_t nk;
    const double* kfrac;          /* nk x 2 fractional k-point coordinates */
    int32_t nspecies;
    const mb_species* species;
    int32_t natoms;
    const mb_atom* atoms;
} mb_desc;

typedef struct mb_problem mb_problem;

/* Initialise the HIP runtime this library links and report the number of GPUs it
 * sees (0 on a machine without one; not an error).  Optional: GPU entry points
 * initialise on first use.  A process that also loads another HIP runtime (for
 * example a framework's bundled copy) should call it right after loading the
 * library, before the other runtime initialises. */
mb_status mb_init(int* ndevices);

/* Build every table of the problem on the host (knots, Gauss rule, B-spline
 * values, banded S_z / D_z and the Cholesky factor of S_z, G sets, grid maps,
 * projector factors) and upload them to `device`, where the local potential is
 * sampled on the grid.  With device < 0 the handle is host-only: queries work,
 * GPU calls return MB_ERR_NO_DEVICE.  Returns MB_ERR_INVALID_ARG for an
 * inconsistent description (a G that does not map to a distinct grid point,
 * non-increasing breakpoints, ...), MB_ERR_NOT_SPD if S_z is singular. */
mb_status mb_problem_create(const mb_desc* desc, int device, mb_problem** out);
mb_status mb_problem_destroy(mb_problem* p);

/* ---- the 1D-periodic form --------------------------------------------------
 * Two B-spline directions and plane waves along the periodic one (the extension named
 * at the end of Sec. II.B.2, for wires and ribbons without a vacuum supercell):
 *   chi_{G,i,j}(x, y, z) = L^{-1/2} e^{i(k+G) y} B_i(x) B_j(z),  G = 2 pi m / L,
 *   1/2 (k+G)^2 <= ecut,  k = kfrac 2 pi / L,
 * with hard-wall spline sets along x and z (same order and Gauss points per interval).
 *   S = I_G (x) S_x (x) S_z
 *   T = 1/2 [D_x (x) S_z + S_x (x) D_z + (k+G)^2 S_x (x) S_z]   per G
 *   V_loc: the Gaussian wells of the species (summed over the images along y) sampled at
 *          (x_q, y_n, z_p), y_n = n L / ny, and applied through ny-point transforms along y
 *   V_NL = sum_p E_p |beta_p><beta_p| with the s, p_x, p_y, p_z projectors of mb_species,
 *          <G,i,j|beta_p> = F_p(G) X_p(i) Z_p(j)  (three one-dimensional integrals)
 * Vectors: x[band][i][j][G], rows i * N_bz + j, row stride ld >= N_G (the slab layout with
 * N_b = N_bx N_bz rows).  Handles from mb_wire_create work with mb_problem_destroy,
 * mb_problem_dims (N_b = N_bx N_bz, nzq = z Gauss points), mb_problem_gvectors (m as
 * (m, 0) pairs, |k+G|^2), hpsi_apply, spsi_apply, s_solve and lanczos_lowest (FP64;
 * MB_FP32 and MB_BF16X3 run the local and nonlocal parts in FP32, the projections on the
 * vector units).  Every other call returns MB_ERR_INVALID_ARG for them.  Augmentation
 * charges are not supported in this form (MB_ERR_INVALID_ARG). */
typedef struct {
    double period;                /* L along y, bohr (> 0) */
    int32_t order;                /* spline order (4: the GPU kernels are cubic) */
    int32_t nbreak_x;             /* breakpoints along x, strictly increasing (>= 2) */
    const double* breakpoints_x;
    int32_t nbreak_z;             /* breakpoints along z */
    const double* breakpoints_z;
    int32_t nq;                   /* Gauss points per interval in both directions, 1..8 */
    int32_t ny;                   /* transform length along y: 8, 12, 16, 24, 32, 48, 64 or 128;
                                     2 m_max + 1 <= ny */
    double ecut;                  /* plane waves with 1/2 (k+G)^2 <= ecut (Ha) */
    int32_t nk;
    const double* kfrac;          /* nk fractions of 2 pi / L */
    int32_t nspecies;
    const mb_species* species;
    int32_t natoms;
    const mb_atom* atoms;         /* positions (x, y, z), bohr */
} mb_wire_desc;

/* Build the tables of a 1D-periodic problem (as mb_problem_create: host tables, then
 * upload to `device`, device < 0 host-only).  MB_ERR_INVALID_ARG for an inconsistent
 * description, MB_ERR_NOT_SPD if S_x or S_z is singular. */
mb_status mb_wire_create(const mb_wire_desc* desc, int device, mb_problem** out);
/* Sizes of a 1D-periodic problem: splines along x and z, Gauss points along x and z,
 * transform length along y.  MB_ERR_INVALID_ARG for a slab problem. */
mb_status mb_wire_dims(const mb_problem* p, int64_t* nbx, int64_t* nbz, int64_t* nxq, int64_t* nzq, int64_t* ny);

/* Sizes for k-point ik: N_G, N_b, recommended ld, number of projectors, number
 * of Gauss points N_q = nq * N_int. Any output pointer may be NULL. */
mb_status mb_problem_dims(const mb_problem* p, int ik, int64_t* ng, int64_t* nb, int64_t* ld,
                          int64_t* nproj, int64_t* nzq);

/* Host copies of set-up tables (for checks against an independent code):
 * mb_problem_gvectors: m (N_G x 2 int32, library order) and |k+G|^2 (N_G doubles);
 * mb_problem_zrule: z_q and w_q (N_q doubles each);
 * mb_problem_zbands: S_z and D_z as N_b x kappa arrays, band[i][d] = M[i][i+d]
 *   (zero past the end);
 * mb_problem_projectors: F (N_p x N_G complex128 = 2*N_p*N_G doubles), Z (N_p x N_b),
 *   E (N_p) with <G,i|beta_p> = F[p][G] Z[p][i]. */
mb_status mb_problem_gvectors(const mb_problem* p, int ik, int32_t* m, double* kg2);
mb_status mb_problem_zrule(const mb_problem* p, double* zq, double* wq);
mb_status mb_problem_zbands(const mb_problem* p, double* sband, double* dband);
mb_status mb_problem_projectors(const mb_problem* p, int ik, double* F, double* Z, double* E);
/* Augmentation charge q_p of every projector (N_p doubles, projector order of
 * mb_problem_projectors); all zero for a norm-conserving description. */
mb_status mb_problem_augmentation(const mb_problem* p, double* q);

/* Replace the local potential by a caller-given real grid V[q][j1][j2]
 * (N_q x N1 x N2 doubles, host memory, V at rho = j1/N1 a1 + j2/N2 a2, z = z_q).
 * Synchronous. */
mb_status mb_problem_set_potential(mb_problem* p, const double* v_host);

/* y = H c for nbands vectors of k-point ik (all terms of H above).  The local
 * part is one pass of: B-spline evaluate at the Gauss planes, G-sphere scatter,
 * inverse 2D FFT, multiply by V(rho, z_q), forward 2D FFT, gather, B-spline
 * project (matrix elements of the local potential, Sec. II.B.1).
 * c and y must not overlap. */
mb_status hpsi_apply(mb_problem* p, int ik, const void* c, void* y, int64_t nbands, int64_t ld,
                     mb_precision prec, void* stream);

/* y = H c for real wavefunctions at the Gamma point (k = 0): every band must satisfy
 * c(-G) = conj c(G), i.e. psi(rho, z) real, the form the eigenvectors take there when
 * the potential and projectors are real (the plane-wave half of the basis of Sec. II.A
 * at k = 0).  The local part can then transform two bands per complex FFT
 * (psi_a + i psi_b; the two results separate by the G -> -G symmetry), halving the
 * transform work of hpsi_apply.  It does so where that is faster (the 128 x 64 grid with
 * FP32 local arithmetic); elsewhere the bands are transformed one by one.  Vectors
 * keep the full-sphere layout of hpsi_apply; for bands that are not real in space the
 * result is not H c.  MB_ERR_INVALID_ARG if k-point ik is not Gamma or its G set is
 * not closed under G -> -G.  Arguments, layout and errors otherwise as hpsi_apply. */
mb_status hpsi_apply_gamma(mb_problem* p, int ik, const void* c, void* y, int64_t nbands, int64_t ld,
                           mb_precision prec, void* stream);

/* hpsi_apply for callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same operator
 * and kernels as hpsi_apply, with every work buffer (local partial rows, projections,
 * matrix-core partial projections) in a fixed 256 MiB array that the library holds on
 * each GPU it runs on until the process ends.  No hipMalloc, hipFree or allocating
 * library call is made.  Bands are processed in groups whose work space fits the
 * array (a group holds e.g. 5 bands of a 128x64-grid, 192-spline slab in FP64, or all
 * 32 of a 36x36-grid, 80-spline slab); MB_ERR_INVALID_ARG if a single band needs
 * more than 256 MiB.  The array keeps the last call's contents and no kernel reads
 * it before writing it.  Every call on one GPU shares that GPU's array: calls that
 * overlap on one GPU (different streams or threads, any problem) race and give
 * wrong results; serialise them.  Arguments and layout as for hpsi_apply. */
mb_status hpsi_apply_noalloc(mb_problem* p, int ik, const void* c, void* y, int64_t nbands, int64_t ld,
                             mb_precision prec, void* stream);

/* y = S c (banded overlap, Sec. II.B.1).  With augmentation charges (ultrasoft form,
 * Sec. II.B.2) y = S_z c + sum_p q_p |beta_p> <beta_p|c>: the projections <beta_p|c>
 * run through the same projection kernels as hpsi_apply and the expansion is fused
 * into the banded pass; the projections use the k-point's projection work buffers
 * (allocated on first use like hpsi_apply's, or reserved by mb_problem_reserve).
 * c and y must not overlap. */
mb_status spsi_apply(mb_problem* p, int ik, const void* c, void* y, int64_t nbands, int64_t ld,
                     mb_precision prec, void* stream);

/* Electron density of nbands vectors of k-point ik at the Gauss planes (the charge
 * density of Sec. II.B.1, rho_e = sum of |phi|^2 over occupied states):
 *   rho[q][j1][j2] += sum_b w[b] |phi_b(rho_j, z_q)|^2,
 *   phi_b(rho, z) = A^{-1/2} sum_{G,i} c_b(G, i) e^{i(k+G).rho} B_i(z),
 *   rho_j = (j1/N1) a1 + (j2/N2) a2.
 * rho: device, N_q x N1 x N2 doubles, accumulated into (zero it first; sum k-points and
 * band blocks over several calls on one stream).  w: device, nbands doubles (occupation
 * times k-point weight).  c: as hpsi_apply (complex128 for MB_FP64, complex64 otherwise);
 * the transforms and sums run in FP64 in every precision.  One workgroup per Gauss plane
 * sums the bands in a fixed order (deterministic, no atomics); the plane must fit in LDS
 * (N1 (N2 + 1) complex doubles <= ~158 KB) and N1 N2 <= 16 x the plane kernel's threads.
 * rho must not overlap c. */
mb_status density_accumulate(mb_problem* p, int ik, const void* c, int64_t nbands, int64_t ld, const double* w,
                             double* rho, mb_precision prec, void* stream);

/* Hartree (Coulomb) potential of a charge density given on the grid at every Gauss plane,
 * in the (z, g) form of Sec. II.B.1 (eq. Coul, from the 2D transform of 1/r):
 *   rho(z_q, g) = 1/(N1 N2) sum_j rho[q][j] e^{i g.rho_j},
 *   V(z_q, g)   = sum_q' w_q' rho(z_q', g) (2 pi/|g|) e^{-|g| |z_q - z_q'|}   (g != 0),
 *   V(z_q, 0)   = -2 pi sum_q' w_q' rho(z_q', 0) |z_q - z_q'|   (the finite part; the
 *                 divergent constant multiplies the cell's net charge, zero if neutral),
 *   vh[q][j]    = sum_g V(z_q, g) e^{-i g.rho_j}   (real).
 * The z integral is the Gauss rule of the knot intervals; each grid frequency is taken at
 * its shortest alias |(m1 + n1 N1) b1 + (m2 + n2 N2) b2|, n in {-1,0,1}^2, which keeps
 * the potential real.  The z sums run as recursions over the ordered Gauss points, O(N_q)
 * per frequency.  rho, vh: device, N_q x N1 x N2 doubles (vh may equal rho).  vzg: NULL or
 * device N_q x N1 x N2 complex128 receiving V(z_q, g) by grid frequency (j1, j2).  Work
 * planes (N_q x N1 x N2 complex128, twice without vzg) are allocated on first use and kept
 * by the problem; the call then enqueues kernels only.  FP64. */
mb_status hartree_potential(mb_problem* p, const double* rho, double* vh, void* vzg, void* stream);

/* Reserve the H work buffers of k-point ik (local partial rows, projections, matrix-core
 * partial projections; with augmentation charges also s_solve's in-place copy of r) for
 * calls of up to max_bands vectors with row stride ld (0: the
 * recommended ld), in any precision.  With lock != 0 they are also locked: later
 * hpsi_apply / spsi_apply / s_solve / lanczos_lowest calls on this k-point that would need larger buffers
 * return MB_ERR_INVALID_ARG instead of reallocating them, and solves do not release
 * them, so their device addresses stay fixed until mb_problem_reserve is called again
 * (lock = 0 unlocks) or the problem is destroyed.  A HIP graph that captured
 * hpsi_apply / spsi_apply / s_solve on this k-point holds these addresses: reserve and
 * lock before capturing, and keep the lock while the graph may be replayed.  Without a
 * lock a later call on the k-point with more bands, or a solve of hundreds of bands,
 * may free and reallocate the buffers, and a replay would write to freed memory.
 * Synchronises the device when it grows a buffer; no call on this k-point may be in
 * flight.  max_bands = 0 only sets the lock. */
mb_status mb_problem_reserve(mb_problem* p, int ik, int64_t max_bands, int64_t ld, int lock);

/* Autotuner of the operator's kernel choices for one k-point, block size and
 * precision: times the local-potential kernels that support the grid, each with the
 * combine pass that projects its output (the line-per-thread kernel at LDS budgets of
 * 22-160 KB per workgroup, i.e. 1 to all Gauss planes of an interval per workgroup;
 * the two-step line kernel; the generic kernel; the plane kernel in its two lane
 * splits) and, in FP32, the two projector paths (vector kernel, matrix cores), on
 * nbands scratch vectors, and makes the fastest the choice of later hpsi_apply and
 * eigensolver calls on that k-point (MB_FP32 / MB_BF16X3 also set it for the
 * eigensolver's FP32 arithmetic on complex128 vectors).  A measurement call: it
 * allocates and frees scratch memory and synchronises `stream`; it must not overlap
 * other calls on the same k-point.  info may be NULL. */
typedef struct {
    int32_t local_kernel;     /* 0 line-per-thread, 1 two-step line, 2 generic, 3 plane; -1 untuned rule */
    int32_t lds_budget_kb;    /* line-per-thread kernel: LDS budget per workgroup (22..160) */
    int32_t plane_variant;    /* plane kernel: 0 8 points per lane, 1 16 points per lane */
    int32_t nl_matrix_cores;  /* FP32 projectors: 1 matrix cores, 0 vector kernel, -1 not tuned */
    int32_t combine_bands;    /* partial-row combine pass: bands per thread 1 or 4, 0 = by projector count */
    int32_t candidates;       /* configurations timed */
    double local_ms;          /* chosen local kernel + combine pass, per call of nbands vectors */
    double local_default_ms;  /* the untuned choice (local kernel + combine pass), per call */
    double nl_ms;             /* chosen projector path, per call (0 if not tuned) */
} mb_tune_info;
mb_status mb_autotune(mb_problem* p, int ik, int64_t nbands, mb_precision prec, void* stream,
                      mb_tune_info* info);

/* Kernel choices of k-point ik for one precision class (MB_FP64; MB_FP32 and MB_BF16X3
 * share one class), as mb_autotune left them or as set here; timing fields are zero.
 * mb_tune_set applies choices without timing (MB_ERR_INVALID_ARG for a value outside the
 * ranges above, or the plane kernel on a grid it does not support); local_kernel = -1
 * restores the untuned rules.  Host-side; no GPU needed. */
mb_status mb_tune_get(const mb_problem* p, int ik, mb_precision prec, mb_tune_info* info);
mb_status mb_tune_set(mb_problem* p, int ik, mb_precision prec, const mb_tune_info* info);

/* Persisted autotuner cache.  mb_tune_save merges the tuned choices of every k-point and
 * precision class of the problem into the JSON file at `path` (created if missing; entries
 * of other problems in it are kept).  Each entry is keyed by what the choice depends on:
 * grid N1 x N2, spline order, N_b, knot intervals, Gauss points per interval, N_G,
 * projector count, recommended ld and the GPU architecture ("host" for host-only
 * handles).  mb_tune_load applies every entry whose key matches a k-point and class of
 * the problem and reports how many it applied (applied may be NULL); a missing file
 * applies nothing and is not an error; MB_ERR_INVALID_ARG for a malformed file.  Host
 * file I/O only. */
mb_status mb_tune_save(const mb_problem* p, const char* path);
mb_status mb_tune_load(mb_problem* p, const char* path, int* applied);

/* x = S^{-1} r by forward and back substitution with the banded Cholesky factor
 * of S_z, shared by every G and band.  With augmentation charges (ultrasoft overlap
 * S = S_0 + B Q B^H, S_0 = I_G (x) S_z, B = [beta_1 .. beta_Np], Q = diag(q_p)) the
 * Woodbury identity gives S^{-1} = S_0^{-1} - S_0^{-1} B W B^H S_0^{-1} with
 * W = Q (I + (B^H S_0^{-1} B) Q)^{-1}, an N_p x N_p matrix built per k-point on the
 * host in FP64 at creation (B^H S_0^{-1} B factors into in-plane and z sums).  The
 * call then runs: x = S_0^{-1} r, P = B^H x, P' = -W P (FP64), t = r + B P',
 * x = S_0^{-1} t; work buffers as for spsi_apply, plus one vector block when x == r
 * (a copy of r).  x may equal r (in place). */
mb_status s_solve(mb_problem* p, int ik, const void* r, void* x, int64_t nbands, int64_t ld,
                  mb_precision prec, void* stream);

typedef struct {
    int32_t block;        /* vectors per block of the block cycle (>= 1) */
    int32_t krylov;       /* Krylov vectors per block per block cycle (>= 1) */
    int32_t krylov_global;/* Krylov vectors of the global cycle (>= 0) */
    int32_t max_iter;     /* grand cycles (>= 1) */
    double tol;           /* converged when every ||H x - eps S x||_2 <= tol (x^H S x = 1) */
    double sigma;         /* shift of the kinetic preconditioner (T + sigma S_0)^{-1}, Ha (default 0.05);
                             <= 0: S_0^{-1} (S_0 = I_G (x) S_z; augmentation charges are left out of the
                             preconditioner, not out of H, S or the Rayleigh-Ritz step) */
    double switch_tol;    /* MB_FP32/MB_BF16X3: residual at which the solve continues in FP64 */
    uint64_t seed;        /* seed of the random start when x0 is NULL */
    int32_t extra;        /* buffer vectors iterated above the nev wanted ones (not required to
                             converge); < 0: min(16, max(4, nev / 4)) */
    int32_t dense_low;    /* MB_FP32/MB_BF16X3: 1 (default) = during the reduced-precision cycles the
                             vector combinations of 128 or more vectors (rotations, Gram-Schmidt
                             updates) use FP32 matrix-core arithmetic on the FP64 vectors, and the
                             Krylov vectors are orthogonalised against the trial vectors in one
                             classical Gram-Schmidt pass instead of two; 0 = FP64 and two passes
                             throughout.  Gram products stay FP64 (the projected problems need their
                             overlap matrices to FP64 accuracy); the FP64 cycles that finish the
                             solve are unaffected. */
} mb_lanczos_opts;

typedef struct {
    int32_t iters;        /* grand cycles done */
    int32_t iters_low;    /* of which in reduced precision */
    int64_t h_applies;    /* band-vectors of H applied */
    int64_t h_applies_low;/* of which in reduced precision */
    double max_resid;     /* largest final residual norm */
    double time_ms;       /* wall time of the call */
} mb_lanczos_info;

/* Fill opts with the defaults. */
void mb_lanczos_default_opts(mb_lanczos_opts* opts);

/* Lowest nev eigenpairs of H c = eps S c for k-point ik by the generalized
 * Lanczos-Krylov method (Sec. II.C): alternating (a) a global Rayleigh-Ritz over
 * the trial vectors together with a Krylov subspace grown from one trial vector
 * and (b) a block cycle in which each small block of trial vectors is
 * diagonalised together with a Krylov subspace grown from one of its vectors,
 * roots selected by maximum overlap with the block's inputs.  Gram-Schmidt in the
 * S inner product throughout, Jacobi diagonalisation of every projected matrix.
 * Krylov vectors are grown with a preconditioned shifted operator
 * K (H - theta S), K = (T + sigma S)^{-1}.
 * prec = MB_FP64: all in FP64.  MB_FP32 / MB_BF16X3: H is applied in reduced
 * precision until every residual is below opts->switch_tol, then the solve
 * continues in FP64 (Gram products, Krylov coefficients and every projected
 * eigenproblem are FP64 throughout; opts->dense_low sets the vector combinations
 * and Gram-Schmidt passes of the reduced-precision cycles).
 * Soft locking: a block whose residuals are all <= opts->tol sits out the block
 * cycle (its vectors stay in every global Rayleigh-Ritz step) until a residual
 * rises above opts->tol again.
 * x0: device complex128 [nev][N_b][ld] start vectors, or NULL for a seeded random
 * start.  eig: host, nev doubles (ascending).  x: device complex128
 * [nev][N_b][ld] output, S-orthonormal.  info and opts may be NULL (defaults).
 * Limits: nev + buffer + krylov_global <= 512, block + krylov <= 64.
 * Device memory: the k-point keeps its solver workspace between calls, except that a
 * solve whose vectors exceed 8 GiB (hundreds of bands on large slabs) frees them and
 * the k-point's H work buffers when it returns.  MB_ERR_OOM if they do not fit.
 * Returns MB_ERR_NOT_CONVERGED (outputs filled) after opts->max_iter cycles. */
mb_status lanczos_lowest(mb_problem* p, int ik, int nev, mb_precision prec,
                         const mb_lanczos_opts* opts, const void* x0, double* eig, void* x,
                         mb_lanczos_info* info, void* stream);

/* ---- many independent problems at once -------------------------------------
 * A batch is a fixed list of (problem, k-point) items, of different cells, grids,
 * B-spline counts, G sets and band counts.  Items of one problem share its
 * tables; the batch owns its own workspaces.  Destroying a problem before a batch
 * that names it is an error of the caller. */
typedef struct mb_batch mb_batch;

/* items t = 0..nitems-1 are (probs[t], iks[t]); every problem must be on the same
 * device.  Host arrays, copied.  Returns MB_ERR_INVALID_ARG for a NULL or host-only
 * problem, a k index out of range, nitems < 1 or > 65536. */
mb_status mb_batch_create(mb_problem* const* probs, const int* iks, int nitems, mb_batch** out);
mb_status mb_batch_destroy(mb_batch* b);

/* y_t = H_t c_t for every item t: the operator of hpsi_apply (Sec. II.B), with the
 * in-plane FFT work of all items sharing one launch per grid size, one launch for
 * the banded combine over all items and per-item projector contractions.
 * c, y: host arrays of nitems device pointers, vectors [nbands[t]][N_b][ld[t]]
 * (complex128 for MB_FP64, complex64 for MB_FP32 / MB_BF16X3); ld may be NULL
 * (then each item's recommended ld).  nbands[t] = 0 skips the item.  c_t and y_t
 * must not overlap, and no y_t may overlap another item's c or y.
 * Stream-ordered: the small descriptor tables of the launches are staged through
 * pinned host memory owned by the batch, so successive calls on one batch must
 * be issued on one stream (or be synchronised in between).  Not capturable into
 * a graph (it copies from host memory that later calls reuse): mb_batch_bind +
 * hpsi_apply_batched_bound are the capturable form. */
mb_status hpsi_apply_batched(mb_batch* b, const void* const* c, void* const* y, const int64_t* nbands,
                             const int64_t* ld, mb_precision prec, void* stream);

/* Bind vector blocks to the batch for repeated, capturable applications: the arguments
 * of hpsi_apply_batched (validated here), work buffers of their own sized for exactly
 * these blocks, and a staging slot of their own.  Allocates and synchronises the device;
 * a later bind replaces the earlier one (a graph that captured the earlier bound call
 * must not be replayed after it).  The bound device blocks must stay allocated while
 * bound calls may run. */
mb_status mb_batch_bind(mb_batch* b, const void* const* c, void* const* y, const int64_t* nbands,
                        const int64_t* ld, mb_precision prec);

/* y_t = H_t c_t for the bound blocks, as hpsi_apply_batched.  Enqueues kernels and copies
 * of launch descriptors from the bound staging slot only: no allocation, no host
 * synchronisation, and the slot's contents are the same on every call, so the call can
 * be captured into a HIP graph and replayed (the replays read the current contents of the
 * bound c blocks).  Bound calls on one batch must not overlap each other. */
mb_status hpsi_apply_batched_bound(mb_batch* b, void* stream);

/* lanczos_lowest for every item t (nev[t] eigenpairs, eig[t] host nev[t] doubles,
 * x[t] device complex128 [nev[t]][N_b][ld_t] with the item's recommended ld_t,
 * info[t] filled; info may be NULL).  Items are solved concurrently on streams of
 * their own (up to 16 at a time, and no more than the free device memory holds at
 * the call's start, estimated from the largest item's workspace); items naming the
 * same (problem, k-point) one after another;
 * `stream` waits for all of them.  opts as for lanczos_lowest (NULL: defaults),
 * x0 = NULL start for every item.  Returns the first error, or
 * MB_ERR_NOT_CONVERGED when some item did not converge (all outputs filled). */
mb_status lanczos_lowest_batched(mb_batch* b, const int* nev, mb_precision prec, const mb_lanczos_opts* opts,
                                 double* const* eig, void* const* x, mb_lanczos_info* info, void* stream);

/* The projected-eigenproblem step of lanczos_lowest on its own (Rayleigh-Ritz with
 * the Jacobi method, Sec. II.C): nz independent generalized Hermitian problems
 * H y = theta S y of size N (1..512), H and S row-major N x N complex128 each
 * (2*N*N doubles, interleaved re/im), S positive definite.  S = L L^H is reduced
 * by a Cholesky factor, A = L^{-1} H L^{-H} is diagonalised by cyclic Jacobi
 * sweeps with the round-robin parallel ordering, Y = L^{-H} V.  Outputs: evals
 * (nz x N, ascending per problem), Y (nz x N x N complex128, column j = vector of
 * evals[j], Y^H S Y = I), sweeps (nz ints, may be NULL).  Host buffers; allocates
 * device memory internally and synchronises `stream`.  Directions of S that are
 * numerically dependent are deflated to theta = 1e30. */
mb_status mb_small_geneig(const double* H, const double* S, int N, int nz, double* evals, double* Y,
                          int* sweeps, void* stream);

/* Stage timer for measurement runs: while enabled, every kernel launch of the
 * library is bracketed by HIP events recorded on the stream it is launched on.
 * mb_timer_enable(1) clears earlier records; mb_timer_read synchronises the
 * recorded events of one stage and returns the summed kernel time (ms) and the
 * number of launches.  Stages: MB_STAGE_LOCAL (fused evaluate / FFT / V / FFT /
 * project, FP64 arithmetic), MB_STAGE_NL_PROJECT, MB_STAGE_COMBINE, MB_STAGE_SPSI, MB_STAGE_SSOLVE,
 * MB_STAGE_PRECOND, MB_STAGE_GRAM, MB_STAGE_COMBO, MB_STAGE_SMALLEIG, MB_STAGE_OTHER,
 * MB_STAGE_LOCAL32, MB_STAGE_DENSITY, MB_STAGE_HARTREE.
 * Not thread safe; enable only in single-threaded measurement code. */
#define MB_STAGE_LOCAL 0
#define MB_STAGE_NL_PROJECT 1
#define MB_STAGE_COMBINE 2
#define MB_STAGE_SPSI 3
#define MB_STAGE_SSOLVE 4
#define MB_STAGE_PRECOND 5
#define MB_STAGE_GRAM 6
#define MB_STAGE_COMBO 7
#define MB_STAGE_SMALLEIG 8
#define MB_STAGE_OTHER 9
#define MB_STAGE_LOCAL32 10  /* the local-potential kernel with FP32 arithmetic */
#define MB_STAGE_DENSITY 11
#define MB_STAGE_HARTREE 12
#define MB_NSTAGE 13
mb_status mb_timer_enable(int on);
/* total_ms: summed kernel time; count: launches; units (may be NULL): summed band
 * count of the launches (vectors processed) */
mb_status mb_timer_read(int stage, double* total_ms, int64_t* count, int64_t* units);

/* Message of the last failed call on this thread ("" if none). */
const char* mb_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* MBKS_H */
