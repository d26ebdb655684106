// Internal declarations of the mixed-basis operator library (host + device).
#pragma once

#include <hip/hip_runtime.h>

#include <complex>
#include <cstdint>
#include <string>
#include <vector>

#include "../../include/mbks.h"

namespace mb {

using zd = std::complex<double>;

// Radix plan of one FFT axis: n = prod rad[0..nr).
struct FftPlan {
    int n;
    int nr;
    int rad[12];
};

struct Workspace {
    void* ptr = nullptr;
    size_t bytes = 0;
};

// Tables of one B-spline direction (hard-wall set of order kappa on clamped knots):
// Gauss points and weights, kept-spline values bval[q][t] = B_{s-1+t}(z_q) on the
// interval s of point q (zero for dropped splines), w_q bval, derivatives, and the
// banded overlap, derivative overlap and Cholesky factor, band[i][d].
struct SplineDir {
    int nint = 0, nb = 0, nq = 0, nzq = 0;
    std::vector<double> bp, zq, wq, bval, wbval, dval, sband, dband, lband;
};

// The 1D-periodic form: B-splines along x and z, plane waves along the period L in y.
// Vector rows are (i, j) = i * nbz + j (x spline i, z spline j), G fastest.
struct WireTables {
    double period = 0.0;
    int ny = 0;              // FFT length along y
    SplineDir x, z;
    std::vector<double> Xp, Zp;             // np x nbx, np x nbz projector factors
    std::vector<int32_t> xwin, zwin;        // np x 2: first, last non-negligible row
    std::vector<int32_t> ploff, plist;      // per x row i: projectors whose x window holds i
    std::vector<double> Uz, lamz;           // D_z u = lambda S_z u, Uz[j][j'] S_z-orthonormal columns
    // device copies (T: double and float)
    double *d_bx = nullptr, *d_wbx = nullptr, *d_bz = nullptr, *d_wbz = nullptr;
    float *d_bxf = nullptr, *d_wbxf = nullptr, *d_bzf = nullptr, *d_wbzf = nullptr;
    double *d_sx = nullptr, *d_dx = nullptr, *d_lx = nullptr;
    double *d_sz = nullptr, *d_dz = nullptr, *d_lz = nullptr;
    double *d_X = nullptr, *d_Z = nullptr;
    float *d_Xf = nullptr, *d_Zf = nullptr;
    int32_t *d_xwin = nullptr, *d_zwin = nullptr, *d_ploff = nullptr, *d_plist = nullptr;
    double *d_Uz = nullptr, *d_lamz = nullptr;
    double* d_V = nullptr;   // [p][q][n] = V(x_q, y_n, z_p) / ny
    float* d_Vf = nullptr;
    void *d_tw = nullptr, *d_twf = nullptr;  // exp(+2 pi i k / ny)
};

// Per-k-point tables and the device workspaces of calls on this k-point (calls on
// different k-points of one problem may run concurrently on different streams).
struct KPoint {
    int ng = 0;
    int ld = 0;
    std::vector<int32_t> m;       // ng x 2
    std::vector<double> kg;       // ng x 2, Cartesian k+G
    std::vector<double> kg2;      // ng
    std::vector<int32_t> gmap;    // ng: grid index j1 * N2 + j2 of G
    std::vector<int32_t> rows;    // grid rows j1 that hold sphere points
    std::vector<zd> F;            // np x ld, in-plane projector factors (padding zero)
    std::vector<int32_t> gtab;    // rows.size() x N2: G index at (sphere row, column j2), -1 outside
    // device copies
    double* d_kg2 = nullptr;
    float* d_kg2f = nullptr;
    int32_t* d_gmap = nullptr;
    int32_t* d_rows = nullptr;
    int32_t* d_gtab = nullptr;
    void* d_F64 = nullptr;        // np x ld complex128
    void* d_F32 = nullptr;        // np x ld complex64
    // ultrasoft overlap: W = Q (I + (B^H S_0^{-1} B) Q)^{-1}, np x np complex128 row-major
    // (empty without augmentation charges)
    std::vector<zd> W;
    void* d_W = nullptr;
    // preconditioner factors (T + sigma S_0) per G, [i][d][ld] doubles, built on demand
    double* d_pfac = nullptr;
    double pfac_sigma = -1.0;
    int gamma_sym = -1;  // Gamma point with a G set closed under G -> -G: 1, else 0; -1 unknown
    // H work buffers (ws_part, ws_proj, ws_nlpart) sized once by mb_problem_reserve and
    // locked: calls that need more fail instead of reallocating, and solves do not free them
    bool locked = false;
    Workspace ws_part;    // local-potential partial projections
    Workspace ws_proj;    // projections <beta|c>
    Workspace ws_nlpart;  // per-row partial projections of the matrix-core kernels
    Workspace ws_aux;     // s_solve with augmentation charges in place: copy of r
    Workspace ws_lz;      // eigensolver vectors
    Workspace ws_small;   // eigensolver small matrices
    // H applications on the plane-kernel grids run the projections on this stream,
    // forked from and joined to the caller's stream by the two events, so that they
    // overlap the plane kernel (created with the problem; null elsewhere)
    hipStream_t aux = nullptr;
    hipEvent_t ev_fork = nullptr, ev_join = nullptr;
    // kernel choices measured by mb_autotune, per arithmetic class of the local part
    // (0: FP64, 1: FP32 with complex64 vectors, 2: FP32 with complex128 vectors)
    struct Tune {
        int set = 0;
        int kind = -1;        // local kernel: 0 line-per-thread, 1 two-step, 2 generic, 3 plane
        int budget_kb = 110;  // LDS budget of the line-per-thread kernel (planes per group)
        int nl_mfma = -1;     // FP32 projector path: 1 matrix cores, 0 vector kernel, -1 default
        int plane_var = 0;    // plane kernel lane split: 0 8 points per lane, 1 16 points per lane
        int combine_bb = 0;   // partial-row combine pass: bands per thread (1, 4), 0 = by projector count
    } tune[3];
};

struct Problem {
    // description
    double a1[2], a2[2];
    double area = 0.0;
    double b1[2], b2[2];
    int order = 4;
    int nint = 0;        // knot intervals
    int nb = 0;          // kept splines
    int nq = 0;          // Gauss points per interval
    int nzq = 0;         // nq * nint
    int N1 = 0, N2 = 0;
    int np = 0;          // projectors
    std::vector<double> bp;      // breakpoints
    std::vector<double> kfrac;   // nk x 2
    std::vector<mb_species> species;
    std::vector<mb_atom> atoms;

    // z tables
    std::vector<double> zq, wq;  // nzq
    std::vector<double> bval;    // nzq x order: kept spline (s - 1 + t) at point q of interval s
    std::vector<double> wbval;   // w_q * bval
    std::vector<double> sband, dband;  // nb x order: M[i][i + d]
    std::vector<double> lband;   // nb x order: Cholesky L[i][i - d]

    // projectors
    std::vector<double> Zp;      // np x nb
    std::vector<double> Ep;      // np
    std::vector<double> Qp;      // np: augmentation charges of the ultrasoft overlap
    bool uspp = false;           // some q_p != 0
    std::vector<int32_t> zwin;   // np x 2: first, last row with a non-negligible Z
    std::vector<KPoint> kp;

    FftPlan plan1{}, plan2{};

    // device
    int device = -1;
    double* d_bval = nullptr;  float* d_bvalf = nullptr;
    double* d_wbval = nullptr; float* d_wbvalf = nullptr;
    double* d_sband = nullptr; float* d_sbandf = nullptr;
    double* d_dband = nullptr; float* d_dbandf = nullptr;
    double* d_lband = nullptr; float* d_lbandf = nullptr;
    double* d_Z = nullptr;     float* d_Zf = nullptr;
    double* d_E = nullptr;     float* d_Ef = nullptr;
    double* d_Q = nullptr;     float* d_Qf = nullptr;   // augmentation charges
    double* d_one = nullptr;   float* d_onef = nullptr; // np ones (unscaled projections)
    double* d_iband = nullptr;  // identity band (nb x kappa): the combine pass as y = c + expansion
    int32_t* d_zwin = nullptr;
    int32_t* d_gwin = nullptr;  // union z-window of each group of 16 projectors
    // per spline row i: the groups of 16 projectors whose union z-window holds it
    // (d_rgoff[i] .. d_rgoff[i+1] into d_rglist); rg_max = the largest count
    int32_t* d_rgoff = nullptr;
    int32_t* d_rglist = nullptr;
    int rg_max = 0;
    double* d_V = nullptr;     float* d_Vf = nullptr;   // nzq x N1 x N2
    double* d_Vt = nullptr;    float* d_Vtf = nullptr;  // nzq x N2 x N1 (plane kernel grids only)
    void* d_tw1 = nullptr; void* d_tw1f = nullptr;      // N1 twiddles exp(+2 pi i k / N1)
    void* d_tw2 = nullptr; void* d_tw2f = nullptr;
    // Hartree step: z_q, w_q, shortest-alias |g| per grid frequency (first use), and its
    // work planes rho(z_q, g) (+ V(z_q, g) when the caller does not take them)
    double* d_zq = nullptr; double* d_wq = nullptr; double* d_gnorm = nullptr;
    Workspace ws_hartree;

    // the 1D-periodic form (null for the slab): then nb = nbx * nbz rows, N1 = ny, and
    // nzq, nq refer to the z direction
    WireTables* wire = nullptr;
};

// stage timer: brackets one kernel launch with events when enabled
struct StageScope {
    int stage;
    hipStream_t s;
    int64_t units;
    void* ev0 = nullptr;
    StageScope(int stage, hipStream_t s, int64_t units = 0);
    ~StageScope();
};

// status helpers
mb_status set_error(mb_status s, const std::string& msg);
#define MB_HIP_TRY(call)                                                               \
    do {                                                                               \
        hipError_t e_ = (call);                                                        \
        if (e_ != hipSuccess)                                                          \
            return ::mb::set_error(MB_ERR_HIP, std::string(#call) + ": " + hipGetErrorString(e_)); \
    } while (0)

#define MB_TRY(call)                \
    do {                            \
        mb_status s_ = (call);      \
        if (s_ != MB_OK) return s_; \
    } while (0)

// host set-up (setup.cpp)
mb_status build_tables(const mb_desc* d, Problem* p);
// one B-spline direction: knots, Gauss rule, spline tables, banded overlap / derivative
// overlap and the Cholesky factor of the overlap (name: for the error message)
mb_status build_spline_dir(const std::vector<double>& bp, int order, int nq, SplineDir* out, const char* name);
bool fft_plan(int n, FftPlan* plan);
int recommended_ld(int ng);

// the 1D-periodic form (wire.cpp: host tables; k_wire.hip: upload and kernels)
mb_status build_wire(const mb_wire_desc* d, Problem* p);
mb_status upload_wire(Problem* p);
void free_wire(Problem* p);  // device tables (when on a device) and the host tables
// y = H c (sy = S c if non-null); lp 0 FP64, 1 FP32 complex64, 2 FP32 arithmetic on complex128
mb_status wire_apply_h(Problem* p, int ik, const void* c, void* y, void* sy, int nbands, int ld, int lp,
                       hipStream_t s);
mb_status wire_spsi(Problem* p, int ik, const void* c, void* y, int nbands, int ld, int prec, hipStream_t s);
mb_status wire_ssolve(Problem* p, int ik, const void* r, void* x, int nbands, int ld, int prec, hipStream_t s);
mb_status wire_prec_factor(Problem* p, int ik, double sigma, hipStream_t s);
mb_status wire_prec_apply(Problem* p, int ik, const void* h, const void* sv, const double* theta, const int32_t* sel,
                          void* x, int nvec, int ld, hipStream_t s);
// MB_ERR_INVALID_ARG with a message when h is a 1D-periodic problem (calls of the slab only)
mb_status refuse_wire(const mb_problem* h, const char* what);

// device upload (capi.hip)
bool ranges_overlap(const void* a, size_t na, const void* b, size_t nb);
// validation shared by the vector entry points; sets the error message
mb_status check_vec_args(const mb_problem* h, int ik, const void* in, const void* out, int64_t nbands, int64_t ld,
                         const char* what);
Problem* problem_of(mb_problem* h);
mb_status upload(Problem* p);
mb_status ensure_ws(Workspace& w, size_t bytes);
// ensure_ws for the H work buffers of a k-point; a locked k-point never reallocates them
mb_status ensure_hws(KPoint& kp, Workspace& w, size_t bytes);

// Caller-provided H work buffers (no allocation in apply_h): local partial rows, projections
// and matrix-core partial projections, each large enough for the call's bands.
struct HWork {
    void* part = nullptr;
    void* proj = nullptr;
    void* nlpart = nullptr;
};
// bytes of each H work buffer for nbands vectors; prec as for apply_h
size_t hwork_part_bytes(const Problem* p, int ik, int nbands, int ld, int prec, bool gamma = false);
size_t hwork_proj_bytes(const Problem* p, int nbands, int prec);
size_t hwork_nlpart_bytes(const Problem* p, int nbands, int prec);
mb_status upload_group_windows(Problem* p);

// kernel launchers (k_*.hip); prec 0 = fp64, 1 = fp32
mb_status launch_vgrid(Problem* p, hipStream_t s);
mb_status launch_local(Problem* p, int ik, const void* c, void* part, int nbands, int ld,
                       int prec, hipStream_t s);
// line-per-thread variant for small grids; MB_ERR_INVALID_ARG = no variant for this grid
mb_status launch_local_split(Problem* p, int ik, const void* c, void* part, int nbands, int ld, int prec,
                             hipStream_t s);
mb_status launch_local_lines(Problem* p, int ik, const void* c, void* part, int nbands, int ld,
                             int prec, hipStream_t s, int budget_kb = 110);
// scaling of the projections <beta_p|c> written by the projection kernels
enum ProjScale { PROJ_E = 0, PROJ_Q = 1, PROJ_ONE = 2 };
// proj[b][p] = scale_p <beta_p|c_b>; projq (optional) [b][p] = q_p <beta_p|c_b>
mb_status launch_nl_project(Problem* p, int ik, const void* c, void* proj, int nbands, int ld,
                            int prec, hipStream_t s, int scale = PROJ_E, void* projq = nullptr);
// plane kernel (one output row per Gauss plane); MB_ERR_INVALID_ARG = no variant for this grid
bool plane_kernel_grid(const Problem* p);
// gamma: bands are real wavefunctions at the Gamma point, transformed two at a time
mb_status launch_local_plane(Problem* p, int ik, const void* c, void* u, int nbands, int ld, int prec,
                             hipStream_t s, bool gamma = false);
// transposed potential copies for the plane kernel (after the potential changes)
mb_status refresh_vt(Problem* p, hipStream_t s);
// the local kernel apply_h runs for (k-point, local precision) writes one row per Gauss
// plane (true) or kappa partial rows per knot interval (false)
bool local_uses_planes(const Problem* p, int ik, int lp);
// matrix-core projections: mode 1 FP32 MFMA, mode 2 BF16x3 MFMA; vin64 = complex128 vectors
mb_status launch_nl_project_mfma(Problem* p, int ik, const void* c, void* proj, int nbands, int ld, int mode,
                                 bool vin64, hipStream_t s, void* nlpart = nullptr, int scale = PROJ_E,
                                 void* projq = nullptr);
// the projection path of apply_h (vector kernel or matrix cores, by projector count,
// tuning and precision); prec as apply_h; nlpart: caller's matrix-core partials or null
mb_status project(Problem* p, int ik, const void* c, void* proj, int nbands, int ld, int prec, hipStream_t s,
                  void* nlpart, int scale = PROJ_E, void* projq = nullptr);
// bytes of the matrix-core partial projections; mode 0 FP64, else FP32 partials
size_t nl_mfma_part_bytes(const Problem* p, int nbands, int mode);
// y = T c + local partials + nonlocal; sy = S c if sy != nullptr; part/proj may be null;
// planes: part holds one row per Gauss plane (plane kernel) instead of kappa rows per interval;
// projq: q-scaled projections, sy gains sum_p |beta_p> projq_p (ultrasoft overlap);
// sband: band of the sy product (null: S_z)
mb_status launch_combine(Problem* p, int ik, const void* c, const void* part, const void* proj,
                         void* y, void* sy, int nbands, int ld, int prec, hipStream_t s, bool planes = false,
                         const void* projq = nullptr, const double* sband = nullptr);
// the combine pass of the plane layout with the z contractions on the matrix cores
mb_status launch_zcombine(Problem* p, int ik, const void* c, const void* u, const void* proj, void* y, void* sy,
                          int nbands, int ld, int prec, hipStream_t s, const void* projq = nullptr);
// y = S c and x = S^{-1} r, with the ultrasoft terms when the problem has augmentation charges
mb_status launch_spsi(Problem* p, int ik, const void* c, void* y, int nbands, int ld, int prec,
                      hipStream_t s);
mb_status launch_ssolve(Problem* p, int ik, const void* r, void* x, int nbands, int ld, int prec,
                        hipStream_t s);
// the banded parts alone: y = S_0 c, x = S_0^{-1} r (S_0 = I_G (x) S_z)
mb_status launch_spsi_banded(Problem* p, int ik, const void* c, void* y, int nbands, int ld, int prec,
                             hipStream_t s);
mb_status launch_ssolve_banded(Problem* p, int ik, const void* r, void* x, int nbands, int ld, int prec,
                               hipStream_t s);
// electron density at the Gauss planes (accumulated into rho) and the Hartree potential
// of a density in the (z, g) form; prec 0 complex128 vectors, else complex64
mb_status launch_density(Problem* p, int ik, const void* c, int nbands, int ld, const double* w, double* rho,
                         int prec, hipStream_t s);
// the density with the plane kernel's lane-split transforms; MB_ERR_INVALID_ARG = no variant
mb_status launch_density_plane(Problem* p, int ik, const void* c, int nbands, int ld, const double* w, double* rho,
                               int prec, hipStream_t s);
size_t hartree_work_bytes(const Problem* p, bool with_vzg);
mb_status launch_hartree(Problem* p, const double* rho, double* vh, void* vzg, void* work, hipStream_t s);
// kernel choices of (k-point, class 0 FP64 / 1 FP32): validated and applied (class 1 also
// sets class 2, complex128 vectors with FP32 arithmetic); kind -1 restores the defaults
mb_status apply_tune(Problem* p, int ik, int cls, int kind, int budget_kb, int plane_var, int nl_mfma,
                     int combine_bb);
// persisted choices (JSON file, merged on save, matched by size key on load)
mb_status tune_save(const Problem* p, const char* path);
mb_status tune_load(Problem* p, const char* path, int* applied);
// host: per k-point Woodbury matrices of the ultrasoft overlap (after the projector tables)
mb_status build_augmentation(Problem* p);
// bytes of s_solve's in-place copy of r (0 without augmentation charges)
size_t aux_bytes(const Problem* p, int ik, int nbands, int ld, int prec);
mb_status launch_prec_factor(Problem* p, int ik, double sigma, hipStream_t s);
// x[j] = K (h[j] - theta[j] s[j]), K = (T + sigma S)^{-1}; theta on device (nvec doubles),
// sel: optional device index list mapping output j to input vector sel[j]
mb_status launch_prec_apply(Problem* p, int ik, const void* h, const void* sv, const double* theta,
                            const int32_t* sel, void* x, int nvec, int ld, hipStream_t s);

// ---- batched application over many (problem, k-point) items ------------------
struct BatchItem {
    Problem* p;
    int ik;
    const void* c;
    void* y;
    void* part;        // local partial rows of this item
    void* proj;        // projections of this item
    int nbands;
    int ld;
    void* nlpart = nullptr;  // matrix-core partial projections (null: the k-point's own buffer)
};

// Copies small descriptor tables to the device in stream order through a pinned
// host buffer; callers wait on `done` before refilling the host buffer.
struct TableUploader {
    char* host = nullptr;
    char* dev = nullptr;
    size_t cap = 0;
    size_t used = 0;
    // reserve bytes (256-aligned); returns host and device addresses
    bool reserve(size_t bytes, void** h, void** d) {
        size_t off = (used + 255) / 256 * 256;
        if (off + bytes > cap) return false;
        *h = host + off;
        *d = dev + off;
        used = off + bytes;
        return true;
    }
};

// each returns MB_ERR_INVALID_ARG (without a message) when it cannot take the items
mb_status launch_local_lines_batch(const std::vector<BatchItem>& items, int prec, TableUploader& up,
                                   hipStream_t s);
mb_status launch_local_split_batch(const std::vector<BatchItem>& items, int prec, TableUploader& up,
                                   hipStream_t s);
mb_status launch_local_batch(const std::vector<BatchItem>& items, int prec, TableUploader& up, hipStream_t s);
mb_status launch_combine_batch(const std::vector<BatchItem>& items, int prec, TableUploader& up, hipStream_t s);

// eigensolver (lanczos.hip): arguments already validated
size_t lanczos_vector_bytes(const Problem* p, int ik, int nev, const mb_lanczos_opts& o);
size_t lanczos_device_bytes(const Problem* p, int ik, int nev, const mb_lanczos_opts& o);
mb_status lanczos_impl(Problem* p, int ik, int nev, mb_precision prec, const mb_lanczos_opts& o, const void* x0,
                       double* eig, void* x, mb_lanczos_info* info, hipStream_t s);
bool timer_enabled();

// composite operator (capi.hip): y = H c (and sy = S c if non-null).
// prec: 0 FP64; 1 FP32 (complex64 vectors); 2 complex128 vectors with FP32 local and
// nonlocal arithmetic; 3 = 1 and 4 = 2 with BF16x3 projector contractions.
// ext: caller-provided work buffers (nothing allocated), else the k-point's own.
// gamma: the bands are real wavefunctions at the Gamma point (c(-G) = conj c(G)); where
// gamma_pairs() holds, their local part is transformed two bands at a time.
mb_status apply_h(Problem* p, int ik, const void* c, void* y, void* sy, int nbands, int ld, int prec,
                  hipStream_t s, const HWork* ext = nullptr, bool gamma = false);
// 1 if k-point ik is Gamma and its G set is closed under G -> -G, else 0 (cached)
bool gamma_point(Problem* p, int ik);
// real-wavefunction pairing is used for this grid and local precision
bool gamma_pairs(const Problem* p, int lp);

}  // namespace mb
