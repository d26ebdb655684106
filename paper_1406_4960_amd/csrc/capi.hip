// C ABI entry points: argument validation, device upload of the set-up tables and
// composition of the operator kernels on the caller's stream.
#include <algorithm>
#include <cmath>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <string>

#include "cplx.h"
#include "mbks_internal.h"

struct mb_problem {
    mb::Problem p;
};

namespace mb {

namespace {
thread_local std::string g_last_error;

template <typename T>
mb_status upload_vec(T** dst, const std::vector<T>& src) {
    if (src.empty()) {
        *dst = nullptr;
        return MB_OK;
    }
    if (hipMalloc(dst, src.size() * sizeof(T)) != hipSuccess) return set_error(MB_ERR_OOM, "hipMalloc failed");
    MB_HIP_TRY(hipMemcpy(*dst, src.data(), src.size() * sizeof(T), hipMemcpyHostToDevice));
    return MB_OK;
}

template <typename T>
mb_status upload_f32(float** dst, const std::vector<T>& src) {
    std::vector<float> f(src.begin(), src.end());
    return upload_vec(dst, f);
}

mb_status upload_twiddles(int n, void** d64, void** d32) {
    std::vector<cx<double>> t(n);
    std::vector<cx<float>> tf(n);
    for (int k = 0; k < n; ++k) {
        double a = 2.0 * 3.14159265358979323846 * k / n;
        t[k] = mk<double>(std::cos(a), std::sin(a));
        tf[k] = mk<float>((float)t[k].x, (float)t[k].y);
    }
    MB_TRY(upload_vec((cx<double>**)d64, t));
    MB_TRY(upload_vec((cx<float>**)d32, tf));
    return MB_OK;
}

void free_all(Problem* p) {
    if (p->device < 0) return;
    void* ptrs[] = {p->d_bval, p->d_bvalf, p->d_wbval, p->d_wbvalf, p->d_sband, p->d_sbandf, p->d_dband,
                    p->d_dbandf, p->d_lband, p->d_lbandf, p->d_Z, p->d_Zf, p->d_E, p->d_Ef, p->d_zwin,
                    p->d_V, p->d_Vf, p->d_Vt, p->d_Vtf, p->d_tw1, p->d_tw1f, p->d_tw2, p->d_tw2f, p->d_gwin, p->d_rgoff, p->d_rglist,
                    p->d_Q, p->d_Qf, p->d_one, p->d_onef, p->d_iband, p->d_zq, p->d_wq, p->d_gnorm,
                    p->ws_hartree.ptr};
    for (void* q : ptrs)
        if (q) (void)hipFree(q);
    for (auto& kp : p->kp) {
        void* kq[] = {kp.d_kg2, kp.d_kg2f, kp.d_gmap, kp.d_rows, kp.d_gtab, kp.d_F64, kp.d_F32, kp.d_pfac,
                      kp.d_W, kp.ws_part.ptr, kp.ws_proj.ptr, kp.ws_nlpart.ptr, kp.ws_aux.ptr, kp.ws_lz.ptr,
                      kp.ws_small.ptr};
        for (void* q : kq)
            if (q) (void)hipFree(q);
        if (kp.aux) (void)hipStreamSynchronize(kp.aux);
        if (kp.ev_fork) (void)hipEventDestroy(kp.ev_fork);
        if (kp.ev_join) (void)hipEventDestroy(kp.ev_join);
        if (kp.aux) (void)hipStreamDestroy(kp.aux);
    }
}

struct TimerState {
    bool on = false;
    std::vector<std::pair<hipEvent_t, hipEvent_t>> ev[MB_NSTAGE];
    double done_ms[MB_NSTAGE] = {0};
    int64_t done_n[MB_NSTAGE] = {0};
    int64_t units[MB_NSTAGE] = {0};
};
TimerState g_timer;

void timer_clear() {
    for (int k = 0; k < MB_NSTAGE; ++k) {
        for (auto& pr : g_timer.ev[k]) {
            (void)hipEventDestroy(pr.first);
            (void)hipEventDestroy(pr.second);
        }
        g_timer.ev[k].clear();
        g_timer.done_ms[k] = 0;
        g_timer.done_n[k] = 0;
        g_timer.units[k] = 0;
    }
}

}  // namespace

bool timer_enabled() { return g_timer.on; }

// set while a no-allocation call runs on this thread: the stage timer creates no events
thread_local bool t_no_events = false;

StageScope::StageScope(int st, hipStream_t str, int64_t u) : stage(st), s(str), units(u) {
    if (!g_timer.on || t_no_events) return;
    hipEvent_t e;
    if (hipEventCreate(&e) != hipSuccess) return;
    (void)hipEventRecord(e, s);
    ev0 = (void*)e;
}

StageScope::~StageScope() {
    if (!ev0) return;
    hipEvent_t e1;
    if (hipEventCreate(&e1) != hipSuccess) return;
    (void)hipEventRecord(e1, s);
    g_timer.ev[stage].emplace_back((hipEvent_t)ev0, e1);
    g_timer.units[stage] += units;
}

mb_status set_error(mb_status s, const std::string& msg) {
    g_last_error = msg;
    return s;
}

bool ranges_overlap(const void* a, size_t na, const void* b, size_t nb) {
    const char* x = (const char*)a;
    const char* y = (const char*)b;
    return x < y + nb && y < x + na;
}

mb_status check_vec_args(const mb_problem* h, int ik, const void* in, const void* out, int64_t nbands, int64_t ld,
                         const char* what) {
    if (!h) return set_error(MB_ERR_INVALID_ARG, std::string(what) + ": problem is NULL");
    const Problem& p = h->p;
    if (p.device < 0) return set_error(MB_ERR_NO_DEVICE, std::string(what) + ": host-only problem");
    if (ik < 0 || ik >= (int)p.kp.size()) return set_error(MB_ERR_INVALID_ARG, std::string(what) + ": ik out of range");
    if (nbands < 0 || nbands > (1 << 20)) return set_error(MB_ERR_INVALID_ARG, std::string(what) + ": nbands");
    if (ld < p.kp[ik].ng || ld > (1 << 24)) return set_error(MB_ERR_INVALID_ARG, std::string(what) + ": ld < N_G");
    if (nbands > 0 && (!in || !out)) return set_error(MB_ERR_INVALID_ARG, std::string(what) + ": NULL vector");
    if (p.order != 4) return set_error(MB_ERR_INVALID_ARG, std::string(what) + ": GPU kernels support order 4 only");
    return MB_OK;
}

mb_status refuse_wire(const mb_problem* h, const char* what) {
    if (h && h->p.wire)
        return set_error(MB_ERR_INVALID_ARG, std::string(what) + ": not available for the 1D-periodic form");
    return MB_OK;
}

mb_status ensure_ws(Workspace& w, size_t bytes) {
    if (w.bytes >= bytes) return MB_OK;
    if (w.ptr) {
        MB_HIP_TRY(hipDeviceSynchronize());
        MB_HIP_TRY(hipFree(w.ptr));
        w.ptr = nullptr;
        w.bytes = 0;
    }
    size_t want = bytes + bytes / 8;
    if (hipMalloc(&w.ptr, want) != hipSuccess) {
        (void)hipGetLastError();
        return set_error(MB_ERR_OOM, "device workspace allocation failed");
    }
    w.bytes = want;
    return MB_OK;
}

mb_status ensure_hws(KPoint& kp, Workspace& w, size_t bytes) {
    if (kp.locked && w.bytes < bytes)
        return set_error(MB_ERR_INVALID_ARG,
                         "the k-point's H work buffers are locked by mb_problem_reserve and are smaller than "
                         "this call needs (reserve more bands)");
    return ensure_ws(w, bytes);
}

// Real-wavefunction pairing (two bands per transform, in the plane kernel) where it was
// measured faster: the 128 x 64 grid with FP32 local arithmetic (surface slab, 320 bands
// at Gamma: H 17.5 against 20.8 ms).  In FP64 that plane kernel holds one workgroup per
// CU, and the gather pass with its two barriers costs more than the halved transforms
// save (H 47.2 against 37.7 ms); on the 36 x 36 grid nothing is gained (0.121 against
// 0.118 ms FP32, 0.220 against 0.196 ms FP64).  MBKS_GAMMA_PAIR=1 pairs on every
// plane-kernel grid, =0 never.
bool gamma_pairs(const Problem* p, int lp) {
    if (!plane_kernel_grid(p)) return false;
    const char* e = getenv("MBKS_GAMMA_PAIR");
    if (e && e[0] == '1') return true;
    if (e && e[0] == '0') return false;
    return p->N1 == 128 && p->N2 == 64 && lp != 0;
}

size_t hwork_part_bytes(const Problem* p, int ik, int nbands, int ld, int prec, bool gamma) {
    const int lp = prec == 3 ? 1 : prec == 4 ? 2 : prec;
    // the plane kernel writes a row per Gauss plane, the others kappa rows per interval;
    // real-wavefunction pairing takes the plane kernel
    const bool planes = (gamma && gamma_pairs(p, lp)) || local_uses_planes(p, ik, lp);
    const size_t rows = planes ? (size_t)p->nzq : (size_t)p->nint * 4;
    return (size_t)nbands * rows * ld * (lp == 0 ? sizeof(cx<double>) : sizeof(cx<float>));
}

// projections [b][p]; with augmentation charges a second block of q-scaled ones follows
size_t hwork_proj_bytes(const Problem* p, int nbands, int prec) {
    const int lp = prec == 3 ? 1 : prec == 4 ? 2 : prec;
    return (p->uspp ? 2 : 1) * (size_t)nbands * p->np * (lp == 0 ? sizeof(cx<double>) : sizeof(cx<float>));
}

size_t aux_bytes(const Problem* p, int ik, int nbands, int ld, int prec) {
    if (!p->uspp) return 0;
    (void)ik;
    return (size_t)nbands * p->nb * ld * (prec == 1 ? sizeof(cx<float>) : sizeof(cx<double>));
}

size_t hwork_nlpart_bytes(const Problem* p, int nbands, int prec) {
    if (p->np == 0) return 0;
    const int lp = prec == 3 ? 1 : prec == 4 ? 2 : prec;
    return nl_mfma_part_bytes(p, nbands, prec >= 3 ? 2 : lp == 0 ? 0 : 1);
}

mb_status upload(Problem* p) {
    MB_TRY(upload_vec(&p->d_bval, p->bval));
    MB_TRY(upload_f32(&p->d_bvalf, p->bval));
    MB_TRY(upload_vec(&p->d_wbval, p->wbval));
    MB_TRY(upload_f32(&p->d_wbvalf, p->wbval));
    MB_TRY(upload_vec(&p->d_sband, p->sband));
    MB_TRY(upload_f32(&p->d_sbandf, p->sband));
    MB_TRY(upload_vec(&p->d_dband, p->dband));
    MB_TRY(upload_f32(&p->d_dbandf, p->dband));
    MB_TRY(upload_vec(&p->d_lband, p->lband));
    MB_TRY(upload_f32(&p->d_lbandf, p->lband));
    {
        std::vector<double> ib((size_t)p->nb * p->order, 0.0);
        for (int i = 0; i < p->nb; ++i) ib[(size_t)i * p->order] = 1.0;
        MB_TRY(upload_vec(&p->d_iband, ib));
    }
    if (p->np > 0) {
        MB_TRY(upload_vec(&p->d_Z, p->Zp));
        MB_TRY(upload_f32(&p->d_Zf, p->Zp));
        MB_TRY(upload_vec(&p->d_E, p->Ep));
        MB_TRY(upload_f32(&p->d_Ef, p->Ep));
        MB_TRY(upload_vec(&p->d_Q, p->Qp));
        MB_TRY(upload_f32(&p->d_Qf, p->Qp));
        const std::vector<double> ones(p->np, 1.0);
        MB_TRY(upload_vec(&p->d_one, ones));
        MB_TRY(upload_f32(&p->d_onef, ones));
        MB_TRY(upload_vec(&p->d_zwin, p->zwin));
        MB_TRY(upload_group_windows(p));
    }
    size_t nv = (size_t)p->nzq * p->N1 * p->N2;
    if (hipMalloc(&p->d_V, nv * sizeof(double)) != hipSuccess) return set_error(MB_ERR_OOM, "potential grid");
    if (hipMalloc(&p->d_Vf, nv * sizeof(float)) != hipSuccess) return set_error(MB_ERR_OOM, "potential grid");
    MB_TRY(upload_twiddles(p->N1, &p->d_tw1, &p->d_tw1f));
    MB_TRY(upload_twiddles(p->N2, &p->d_tw2, &p->d_tw2f));
    for (auto& kp : p->kp) {
        MB_TRY(upload_vec(&kp.d_kg2, kp.kg2));
        MB_TRY(upload_f32(&kp.d_kg2f, kp.kg2));
        MB_TRY(upload_vec(&kp.d_gmap, kp.gmap));
        MB_TRY(upload_vec(&kp.d_rows, kp.rows));
        if (plane_kernel_grid(p)) {
            // G index of every (sphere row, column) of the grid, -1 off the sphere
            std::vector<int32_t> rowpos(p->N1, -1);
            for (size_t r = 0; r < kp.rows.size(); ++r) rowpos[kp.rows[r]] = (int32_t)r;
            kp.gtab.assign(kp.rows.size() * (size_t)p->N2, -1);
            for (int g = 0; g < kp.ng; ++g) {
                const int j1 = kp.gmap[g] / p->N2, j2 = kp.gmap[g] % p->N2;
                kp.gtab[(size_t)rowpos[j1] * p->N2 + j2] = g;
            }
            MB_TRY(upload_vec(&kp.d_gtab, kp.gtab));
        }
        if (p->np > 0) {
            std::vector<cx<double>> F(kp.F.size());
            std::vector<cx<float>> Ff(kp.F.size());
            for (size_t e = 0; e < kp.F.size(); ++e) {
                F[e] = mk<double>(kp.F[e].real(), kp.F[e].imag());
                Ff[e] = mk<float>((float)kp.F[e].real(), (float)kp.F[e].imag());
            }
            MB_TRY(upload_vec((cx<double>**)&kp.d_F64, F));
            MB_TRY(upload_vec((cx<float>**)&kp.d_F32, Ff));
        }
        if (!kp.W.empty()) {
            std::vector<cx<double>> W(kp.W.size());
            for (size_t e = 0; e < kp.W.size(); ++e) W[e] = mk<double>(kp.W[e].real(), kp.W[e].imag());
            MB_TRY(upload_vec((cx<double>**)&kp.d_W, W));
        }
    }
    MB_TRY(launch_vgrid(p, 0));
    MB_TRY(refresh_vt(p, 0));
    // the projections' stream and events of each k-point (default priority)
    if (plane_kernel_grid(p) && p->np > 0) {
        for (auto& kp : p->kp) {
            if (!kp.aux) MB_HIP_TRY(hipStreamCreateWithFlags(&kp.aux, hipStreamNonBlocking));
            if (!kp.ev_fork) MB_HIP_TRY(hipEventCreateWithFlags(&kp.ev_fork, hipEventDisableTiming));
            if (!kp.ev_join) MB_HIP_TRY(hipEventCreateWithFlags(&kp.ev_join, hipEventDisableTiming));
        }
    }
    return MB_OK;
}

// MBKS_NL_OVERLAP=0 keeps the projections on the caller's stream (read per call)
static bool overlap_enabled() {
    const char* e = getenv("MBKS_NL_OVERLAP");
    return !(e && e[0] == '0');
}

// y = H c (sy = S c if non-null).  prec: 0 FP64, 1 FP32 (c64), 2 c128 vectors with FP32 local/nonlocal.
bool gamma_point(Problem* p, int ik) {
    KPoint& kp = p->kp[ik];
    if (kp.gamma_sym < 0) {
        bool ok = p->kfrac[2 * ik] == 0.0 && p->kfrac[2 * ik + 1] == 0.0;
        if (ok) {
            std::vector<std::pair<int, int>> ms;
            for (int g = 0; g < kp.ng; ++g) ms.emplace_back(kp.m[2 * g], kp.m[2 * g + 1]);
            std::sort(ms.begin(), ms.end());
            for (int g = 0; g < kp.ng && ok; ++g)
                ok = std::binary_search(ms.begin(), ms.end(), std::make_pair(-kp.m[2 * g], -kp.m[2 * g + 1]));
        }
        kp.gamma_sym = ok ? 1 : 0;
    }
    return kp.gamma_sym == 1;
}

mb_status apply_h(Problem* p, int ik, const void* c, void* y, void* sy, int nbands, int ld, int prec, hipStream_t s,
                  const HWork* ext, bool gamma) {
    if (nbands == 0) return MB_OK;
    const int lp = prec == 3 ? 1 : prec == 4 ? 2 : prec;  // local / combine precision
    if (p->wire) {
        if (ext) return set_error(MB_ERR_INVALID_ARG, "apply_h: caller work buffers are not used by the 1D-periodic form");
        return wire_apply_h(p, ik, c, y, sy, nbands, ld, lp, s);
    }
    KPoint& kp = p->kp[ik];
    void* part = ext ? ext->part : nullptr;
    if (!ext) {
        MB_TRY(ensure_hws(kp, kp.ws_part, hwork_part_bytes(p, ik, nbands, ld, prec, gamma)));
        part = kp.ws_part.ptr;
    }
    void* proj = nullptr;
    void* projq = nullptr;  // q-scaled projections for sy (ultrasoft overlap)
    if (p->np > 0) {
        if (ext && (!ext->proj || !ext->nlpart))
            return set_error(MB_ERR_INVALID_ARG, "apply_h: caller work buffers lack the projection buffers");
        if (ext) {
            proj = ext->proj;
        } else {
            MB_TRY(ensure_hws(kp, kp.ws_proj, hwork_proj_bytes(p, nbands, prec)));
            proj = kp.ws_proj.ptr;
        }
        if (sy && p->uspp)
            projq = (char*)proj + (size_t)nbands * p->np * (lp == 0 ? sizeof(cx<double>) : sizeof(cx<float>));
    }
    // real-wavefunction pairing lives in the plane kernel (the partial-row buffer above
    // is sized by the same choice); elsewhere the bands go one by one
    const bool pair = gamma && gamma_pairs(p, lp);
    const bool planes = pair || local_uses_planes(p, ik, lp);
    if (planes) {
        // the projections (matrix cores, memory) run beside the plane kernel (bound by
        // vector instruction issue) on the k-point's own stream: forked after everything
        // the caller's stream has queued (c is ready, the previous call's combine pass has
        // read the projection buffers), joined before the combine pass reads them
        const bool overlap = p->np > 0 && kp.aux && overlap_enabled();
        if (p->np > 0) {
            hipStream_t sp = s;
            if (overlap) {
                MB_HIP_TRY(hipEventRecord(kp.ev_fork, s));
                MB_HIP_TRY(hipStreamWaitEvent(kp.aux, kp.ev_fork, 0));
                sp = kp.aux;
            }
            MB_TRY(project(p, ik, c, proj, nbands, ld, prec, sp, ext ? ext->nlpart : nullptr, PROJ_E, projq));
            if (overlap) MB_HIP_TRY(hipEventRecord(kp.ev_join, kp.aux));
        }
        MB_TRY(launch_local_plane(p, ik, c, part, nbands, ld, lp, s, pair));
        if (overlap) MB_HIP_TRY(hipStreamWaitEvent(s, kp.ev_join, 0));
        MB_TRY(launch_zcombine(p, ik, c, part, proj, y, sy, nbands, ld, lp, s, projq));
    } else {
        if (p->np > 0)
            MB_TRY(project(p, ik, c, proj, nbands, ld, prec, s, ext ? ext->nlpart : nullptr, PROJ_E, projq));
        MB_TRY(launch_local(p, ik, c, part, nbands, ld, lp, s));
        MB_TRY(launch_combine(p, ik, c, part, proj, y, sy, nbands, ld, lp, s, false, projq));
    }
    return MB_OK;
}

mb_status project(Problem* p, int ik, const void* c, void* proj, int nbands, int ld, int prec, hipStream_t s,
                  void* nlpart, int scale, void* projq) {
    if (p->np == 0 || nbands == 0) return MB_OK;
    const int lp = prec == 3 ? 1 : prec == 4 ? 2 : prec;
    // FP32 and FP64 projections go to the matrix cores once there are enough
    // projectors to fill their 16-wide tiles (measured: with 8 or 32 projectors the
    // vector kernel is faster, with 256 the matrix cores are 2.7x faster in FP32);
    // BF16x3 always uses them.  MBKS_NL_KERNEL=vector / =mfma forces one path (used
    // to cross-check them).
    const char* sel = getenv("MBKS_NL_KERNEL");
    bool vector_path = p->np < 64;
    const KPoint::Tune& tn = p->kp[ik].tune[lp];
    if (tn.set && tn.nl_mfma >= 0 && lp != 0) vector_path = tn.nl_mfma == 0;
    if (sel && std::string(sel) == "vector") vector_path = true;
    if (sel && std::string(sel) == "mfma") vector_path = false;
    if (prec >= 3) vector_path = false;
    if (vector_path) return launch_nl_project(p, ik, c, proj, nbands, ld, lp, s, scale, projq);
    return launch_nl_project_mfma(p, ik, c, proj, nbands, ld, prec >= 3 ? 2 : lp == 0 ? 0 : 1, lp == 2, s, nlpart,
                                  scale, projq);
}

}  // namespace mb

using mb::set_error;

namespace mb {
namespace {
// Work buffers of hpsi_apply_noalloc: one array per GPU, held for the life of the process.
constexpr size_t NOALLOC_SCRATCH_BYTES = (size_t)256 << 20;
static __device__ __align__(256) unsigned char scratch[NOALLOC_SCRATCH_BYTES];
constexpr int MAX_DEVICES = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[MAX_DEVICES] = {};

// Device address of `scratch` on `device`, looked up once per device with that device
// current (each GPU holds its own copy of the array).
mb_status scratch_address(int device, void** out) {
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (device < 0 || device >= MAX_DEVICES) return set_error(MB_ERR_INVALID_ARG, "scratch: device index");
    if (!g_scratch_ptr[device]) {
        int prev = -1;
        MB_HIP_TRY(hipGetDevice(&prev));
        if (prev != device) MB_HIP_TRY(hipSetDevice(device));
        void* ptr = nullptr;
        const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (prev != device) (void)hipSetDevice(prev);
        if (e != hipSuccess || !ptr)
            return set_error(MB_ERR_HIP, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
        g_scratch_ptr[device] = ptr;
    }
    *out = g_scratch_ptr[device];
    return MB_OK;
}

size_t align256(size_t b) { return (b + 255) / 256 * 256; }

// scratch bytes of one apply_h call on n bands (part, proj, matrix-core partials)
size_t noalloc_bytes(const Problem* p, int ik, int n, int ld, int prec) {
    return align256(hwork_part_bytes(p, ik, n, ld, prec)) + align256(hwork_proj_bytes(p, n, prec)) +
           align256(hwork_nlpart_bytes(p, n, prec));
}
}  // namespace
}  // namespace mb

extern "C" {

const char* mb_last_error(void) { return mb::g_last_error.c_str(); }

mb_status mb_init(int* ndevices) {
    int n = 0;
    if (hipGetDeviceCount(&n) != hipSuccess) {
        (void)hipGetLastError();
        n = 0;
    }
    if (ndevices) *ndevices = n;
    return MB_OK;
}

mb_status mb_timer_enable(int on) {
    mb::timer_clear();
    mb::g_timer.on = on != 0;
    return MB_OK;
}

mb_status mb_timer_read(int stage, double* total_ms, int64_t* count, int64_t* units) {
    if (stage < 0 || stage >= MB_NSTAGE) return set_error(MB_ERR_INVALID_ARG, "mb_timer_read: stage");
    auto& v = mb::g_timer.ev[stage];
    for (auto& pr : v) {
        MB_HIP_TRY(hipEventSynchronize(pr.second));
        float ms = 0.f;
        MB_HIP_TRY(hipEventElapsedTime(&ms, pr.first, pr.second));
        mb::g_timer.done_ms[stage] += ms;
        mb::g_timer.done_n[stage] += 1;
        (void)hipEventDestroy(pr.first);
        (void)hipEventDestroy(pr.second);
    }
    v.clear();
    if (total_ms) *total_ms = mb::g_timer.done_ms[stage];
    if (count) *count = mb::g_timer.done_n[stage];
    if (units) *units = mb::g_timer.units[stage];
    return MB_OK;
}

mb_status mb_problem_create(const mb_desc* desc, int device, mb_problem** out) {
    if (!out) return set_error(MB_ERR_INVALID_ARG, "out is NULL");
    *out = nullptr;
    auto* h = new mb_problem;
    mb_status st = mb::build_tables(desc, &h->p);
    if (st != MB_OK) {
        delete h;
        return st;
    }
    if (device >= 0) {
        int ndev = 0;
        if (hipGetDeviceCount(&ndev) != hipSuccess || device >= ndev) {
            delete h;
            return set_error(MB_ERR_NO_DEVICE, "no such GPU");
        }
        if (hipSetDevice(device) != hipSuccess) {
            delete h;
            return set_error(MB_ERR_HIP, "hipSetDevice failed");
        }
        h->p.device = device;
        st = mb::upload(&h->p);
        if (st != MB_OK) {
            mb::free_all(&h->p);
            delete h;
            return st;
        }
    }
    *out = h;
    return MB_OK;
}

mb_status mb_wire_create(const mb_wire_desc* desc, int device, mb_problem** out) {
    if (!out) return set_error(MB_ERR_INVALID_ARG, "out is NULL");
    *out = nullptr;
    auto* h = new mb_problem;
    mb_status st = mb::build_wire(desc, &h->p);
    if (st != MB_OK) {
        mb::free_wire(&h->p);
        delete h;
        return st;
    }
    if (device >= 0) {
        int ndev = 0;
        if (hipGetDeviceCount(&ndev) != hipSuccess || device >= ndev) {
            mb::free_wire(&h->p);
            delete h;
            return set_error(MB_ERR_NO_DEVICE, "no such GPU");
        }
        if (hipSetDevice(device) != hipSuccess) {
            mb::free_wire(&h->p);
            delete h;
            return set_error(MB_ERR_HIP, "hipSetDevice failed");
        }
        h->p.device = device;
        st = mb::upload_wire(&h->p);
        if (st != MB_OK) {
            mb::free_all(&h->p);
            mb::free_wire(&h->p);
            delete h;
            return st;
        }
    }
    *out = h;
    return MB_OK;
}

mb_status mb_wire_dims(const mb_problem* h, int64_t* nbx, int64_t* nbz, int64_t* nxq, int64_t* nzq, int64_t* ny) {
    if (!h) return set_error(MB_ERR_INVALID_ARG, "problem is NULL");
    const mb::WireTables* w = h->p.wire;
    if (!w) return set_error(MB_ERR_INVALID_ARG, "mb_wire_dims: not a 1D-periodic problem");
    if (nbx) *nbx = w->x.nb;
    if (nbz) *nbz = w->z.nb;
    if (nxq) *nxq = w->x.nzq;
    if (nzq) *nzq = w->z.nzq;
    if (ny) *ny = w->ny;
    return MB_OK;
}

mb_status mb_problem_destroy(mb_problem* h) {
    if (!h) return MB_OK;
    if (h->p.device >= 0) {
        (void)hipDeviceSynchronize();
        mb::free_all(&h->p);
    }
    mb::free_wire(&h->p);
    delete h;
    return MB_OK;
}

mb_status mb_problem_dims(const mb_problem* h, int ik, int64_t* ng, int64_t* nb, int64_t* ld, int64_t* nproj,
                          int64_t* nzq) {
    if (!h) return set_error(MB_ERR_INVALID_ARG, "problem is NULL");
    if (ik < 0 || ik >= (int)h->p.kp.size()) return set_error(MB_ERR_INVALID_ARG, "ik out of range");
    if (ng) *ng = h->p.kp[ik].ng;
    if (nb) *nb = h->p.nb;
    if (ld) *ld = h->p.kp[ik].ld;
    if (nproj) *nproj = h->p.np;
    if (nzq) *nzq = h->p.nzq;
    return MB_OK;
}

mb_status mb_problem_gvectors(const mb_problem* h, int ik, int32_t* m, double* kg2) {
    if (!h) return set_error(MB_ERR_INVALID_ARG, "problem is NULL");
    if (ik < 0 || ik >= (int)h->p.kp.size()) return set_error(MB_ERR_INVALID_ARG, "ik out of range");
    const auto& kp = h->p.kp[ik];
    if (m) std::memcpy(m, kp.m.data(), kp.m.size() * sizeof(int32_t));
    if (kg2) std::memcpy(kg2, kp.kg2.data(), kp.kg2.size() * sizeof(double));
    return MB_OK;
}

mb_status mb_problem_zrule(const mb_problem* h, double* zq, double* wq) {
    if (mb::refuse_wire(h, "mb_problem_zrule") != MB_OK) return MB_ERR_INVALID_ARG;
    if (!h) return set_error(MB_ERR_INVALID_ARG, "problem is NULL");
    if (zq) std::memcpy(zq, h->p.zq.data(), h->p.zq.size() * sizeof(double));
    if (wq) std::memcpy(wq, h->p.wq.data(), h->p.wq.size() * sizeof(double));
    return MB_OK;
}

mb_status mb_problem_zbands(const mb_problem* h, double* sband, double* dband) {
    if (mb::refuse_wire(h, "mb_problem_zbands") != MB_OK) return MB_ERR_INVALID_ARG;
    if (!h) return set_error(MB_ERR_INVALID_ARG, "problem is NULL");
    if (sband) std::memcpy(sband, h->p.sband.data(), h->p.sband.size() * sizeof(double));
    if (dband) std::memcpy(dband, h->p.dband.data(), h->p.dband.size() * sizeof(double));
    return MB_OK;
}

mb_status mb_problem_projectors(const mb_problem* h, int ik, double* F, double* Z, double* E) {
    if (mb::refuse_wire(h, "mb_problem_projectors") != MB_OK) return MB_ERR_INVALID_ARG;
    if (!h) return set_error(MB_ERR_INVALID_ARG, "problem is NULL");
    if (ik < 0 || ik >= (int)h->p.kp.size()) return set_error(MB_ERR_INVALID_ARG, "ik out of range");
    const auto& p = h->p;
    const auto& kp = p.kp[ik];
    if (F)
        for (int q = 0; q < p.np; ++q)
            for (int g = 0; g < kp.ng; ++g) {
                F[2 * ((size_t)q * kp.ng + g)] = kp.F[(size_t)q * kp.ld + g].real();
                F[2 * ((size_t)q * kp.ng + g) + 1] = kp.F[(size_t)q * kp.ld + g].imag();
            }
    if (Z) std::memcpy(Z, p.Zp.data(), p.Zp.size() * sizeof(double));
    if (E) std::memcpy(E, p.Ep.data(), p.Ep.size() * sizeof(double));
    return MB_OK;
}

mb_status mb_problem_augmentation(const mb_problem* h, double* q) {
    if (mb::refuse_wire(h, "mb_problem_augmentation") != MB_OK) return MB_ERR_INVALID_ARG;
    if (!h || !q) return set_error(MB_ERR_INVALID_ARG, "NULL argument");
    std::memcpy(q, h->p.Qp.data(), h->p.Qp.size() * sizeof(double));
    return MB_OK;
}

mb_status mb_problem_set_potential(mb_problem* h, const double* v) {
    if (mb::refuse_wire(h, "mb_problem_set_potential") != MB_OK) return MB_ERR_INVALID_ARG;
    if (!h || !v) return set_error(MB_ERR_INVALID_ARG, "NULL argument");
    auto& p = h->p;
    if (p.device < 0) return set_error(MB_ERR_NO_DEVICE, "host-only problem");
    size_t n = (size_t)p.nzq * p.N1 * p.N2;
    for (size_t e = 0; e < n; ++e)
        if (!std::isfinite(v[e])) return set_error(MB_ERR_NONFINITE, "potential holds a NaN or Inf");
    std::vector<float> vf(v, v + n);
    MB_HIP_TRY(hipMemcpy(p.d_V, v, n * sizeof(double), hipMemcpyHostToDevice));
    MB_HIP_TRY(hipMemcpy(p.d_Vf, vf.data(), n * sizeof(float), hipMemcpyHostToDevice));
    return mb::refresh_vt(&p, 0);
}

mb_status hpsi_apply(mb_problem* h, int ik, const void* c, void* y, int64_t nbands, int64_t ld, mb_precision prec,
                     void* stream) {
    mb_status st = mb::check_vec_args(h, ik, c, y, nbands, ld, "hpsi_apply");
    if (st != MB_OK) return st;
    if (prec != MB_FP64 && prec != MB_FP32 && prec != MB_BF16X3)
        return set_error(MB_ERR_INVALID_ARG, "hpsi_apply: unknown precision");
    size_t bytes = (size_t)nbands * h->p.nb * ld * (prec == MB_FP64 ? 16 : 8);
    if (nbands > 0 && mb::ranges_overlap(c, bytes, y, bytes))
        return set_error(MB_ERR_INVALID_ARG, "hpsi_apply: c and y overlap");
    return mb::apply_h(&h->p, ik, c, y, nullptr, (int)nbands, (int)ld,
                       prec == MB_FP64 ? 0 : prec == MB_FP32 ? 1 : 3, (hipStream_t)stream);
}


mb_status hpsi_apply_gamma(mb_problem* h, int ik, const void* c, void* y, int64_t nbands, int64_t ld,
                           mb_precision prec, void* stream) {
    mb_status st = mb::check_vec_args(h, ik, c, y, nbands, ld, "hpsi_apply_gamma");
    if (st != MB_OK) return st;
    if (mb::refuse_wire(h, "hpsi_apply_gamma") != MB_OK) return MB_ERR_INVALID_ARG;
    if (prec != MB_FP64 && prec != MB_FP32 && prec != MB_BF16X3)
        return set_error(MB_ERR_INVALID_ARG, "hpsi_apply_gamma: unknown precision");
    if (!mb::gamma_point(&h->p, ik))
        return set_error(MB_ERR_INVALID_ARG,
                         "hpsi_apply_gamma: k-point is not Gamma or its G set is not closed under G -> -G");
    size_t bytes = (size_t)nbands * h->p.nb * ld * (prec == MB_FP64 ? 16 : 8);
    if (nbands > 0 && mb::ranges_overlap(c, bytes, y, bytes))
        return set_error(MB_ERR_INVALID_ARG, "hpsi_apply_gamma: c and y overlap");
    return mb::apply_h(&h->p, ik, c, y, nullptr, (int)nbands, (int)ld,
                       prec == MB_FP64 ? 0 : prec == MB_FP32 ? 1 : 3, (hipStream_t)stream, nullptr, true);
}

mb_status hpsi_apply_noalloc(mb_problem* h, int ik, const void* c, void* y, int64_t nbands, int64_t ld,
                             mb_precision prec, void* stream) {
    mb_status st = mb::check_vec_args(h, ik, c, y, nbands, ld, "hpsi_apply_noalloc");
    if (st != MB_OK) return st;
    if (mb::refuse_wire(h, "hpsi_apply_noalloc") != MB_OK) return MB_ERR_INVALID_ARG;
    if (prec != MB_FP64 && prec != MB_FP32 && prec != MB_BF16X3)
        return set_error(MB_ERR_INVALID_ARG, "hpsi_apply_noalloc: unknown precision");
    mb::Problem* p = &h->p;
    const size_t vsz = prec == MB_FP64 ? 16 : 8;
    const size_t bytes = (size_t)nbands * p->nb * ld * vsz;
    if (nbands > 0 && mb::ranges_overlap(c, bytes, y, bytes))
        return set_error(MB_ERR_INVALID_ARG, "hpsi_apply_noalloc: c and y overlap");
    if (nbands == 0) return MB_OK;
    const int iprec = prec == MB_FP64 ? 0 : prec == MB_FP32 ? 1 : 3;
    const size_t one = mb::noalloc_bytes(p, ik, 1, (int)ld, iprec);
    if (one > mb::NOALLOC_SCRATCH_BYTES)
        return set_error(MB_ERR_INVALID_ARG,
                         "hpsi_apply_noalloc: one band needs " + std::to_string(one >> 20) +
                             " MiB of work space, more than the " + std::to_string(mb::NOALLOC_SCRATCH_BYTES >> 20) +
                             " MiB this entry point holds per GPU (use hpsi_apply)");
    void* base = nullptr;
    st = mb::scratch_address(p->device, &base);
    if (st != MB_OK) return st;
    // bands per group: the largest count whose work space fits the scratch array
    int lo = 1, hi = (int)nbands;
    while (lo < hi) {
        const int mid = lo + (hi - lo + 1) / 2;
        if (mb::noalloc_bytes(p, ik, mid, (int)ld, iprec) <= mb::NOALLOC_SCRATCH_BYTES) lo = mid; else hi = mid - 1;
    }
    const int group = lo;
    mb::t_no_events = true;
    for (int b0 = 0; b0 < (int)nbands && st == MB_OK; b0 += group) {
        const int n = std::min(group, (int)nbands - b0);
        mb::HWork w;
        char* q = (char*)base;
        w.part = q;
        q += mb::align256(mb::hwork_part_bytes(p, ik, n, (int)ld, iprec));
        w.proj = q;
        q += mb::align256(mb::hwork_proj_bytes(p, n, iprec));
        w.nlpart = q;
        const size_t off = (size_t)b0 * p->nb * ld * vsz;
        st = mb::apply_h(p, ik, (const char*)c + off, (char*)y + off, nullptr, n, (int)ld, iprec,
                         (hipStream_t)stream, &w);
    }
    mb::t_no_events = false;
    return st;
}

mb_status mb_problem_reserve(mb_problem* h, int ik, int64_t max_bands, int64_t ld, int lock) {
    if (mb::refuse_wire(h, "mb_problem_reserve") != MB_OK) return MB_ERR_INVALID_ARG;
    mb::Problem* p = mb::problem_of(h);
    if (!p) return set_error(MB_ERR_INVALID_ARG, "mb_problem_reserve: problem is NULL");
    if (p->device < 0) return set_error(MB_ERR_NO_DEVICE, "mb_problem_reserve: host-only problem");
    if (ik < 0 || ik >= (int)p->kp.size()) return set_error(MB_ERR_INVALID_ARG, "mb_problem_reserve: ik out of range");
    mb::KPoint& kp = p->kp[ik];
    if (ld == 0) ld = kp.ld;
    if (max_bands < 0 || max_bands > (1 << 20) || ld < kp.ng || ld > (1 << 24))
        return set_error(MB_ERR_INVALID_ARG, "mb_problem_reserve: max_bands or ld out of range");
    kp.locked = false;
    if (max_bands > 0) {
        const int nb = (int)max_bands;
        // FP64 sizes cover every precision; the larger of the two local layouts
        const size_t part = (size_t)nb * std::max<size_t>((size_t)p->nzq, (size_t)p->nint * 4) * ld * 16;
        mb_status st = mb::ensure_ws(kp.ws_part, part);
        if (st == MB_OK && p->np > 0) st = mb::ensure_ws(kp.ws_proj, mb::hwork_proj_bytes(p, nb, 0));
        if (st == MB_OK && p->np > 0) st = mb::ensure_ws(kp.ws_nlpart, mb::hwork_nlpart_bytes(p, nb, 0));
        if (st == MB_OK && p->uspp) st = mb::ensure_ws(kp.ws_aux, mb::aux_bytes(p, ik, nb, (int)ld, 0));
        if (st != MB_OK) return st;
    }
    kp.locked = lock != 0;
    return MB_OK;
}

mb_status mb_autotune(mb_problem* h, int ik, int64_t nbands, mb_precision prec, void* stream, mb_tune_info* info) {
    if (mb::refuse_wire(h, "mb_autotune") != MB_OK) return MB_ERR_INVALID_ARG;
    mb::Problem* p = mb::problem_of(h);
    if (!p) return set_error(MB_ERR_INVALID_ARG, "mb_autotune: problem is NULL");
    if (p->device < 0) return set_error(MB_ERR_NO_DEVICE, "mb_autotune: host-only problem");
    if (ik < 0 || ik >= (int)p->kp.size()) return set_error(MB_ERR_INVALID_ARG, "mb_autotune: ik out of range");
    if (nbands < 1 || nbands > 4096) return set_error(MB_ERR_INVALID_ARG, "mb_autotune: nbands must be 1..4096");
    if (prec != MB_FP64 && prec != MB_FP32 && prec != MB_BF16X3)
        return set_error(MB_ERR_INVALID_ARG, "mb_autotune: unknown precision");
    if (p->order != 4) return set_error(MB_ERR_INVALID_ARG, "mb_autotune: GPU kernels support order 4 only");
    hipStream_t s = (hipStream_t)stream;
    mb::KPoint& kp = p->kp[ik];
    const int cls = prec == MB_FP64 ? 0 : 1;
    const int nb = (int)nbands, ld = kp.ld;
    const size_t csz = cls == 0 ? 16 : 8;
    void *c = nullptr, *part = nullptr, *proj = nullptr, *y = nullptr;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    mb_status st = MB_OK;
    const mb::KPoint::Tune saved = kp.tune[cls];
    auto cleanup = [&]() {
        if (c) (void)hipFree(c);
        if (part) (void)hipFree(part);
        if (proj) (void)hipFree(proj);
        if (y) (void)hipFree(y);
        if (e0) (void)hipEventDestroy(e0);
        if (e1) (void)hipEventDestroy(e1);
    };
    const size_t vbytes = (size_t)nb * p->nb * ld * csz;
    const size_t prows = std::max<size_t>((size_t)p->nzq, (size_t)p->nint * 4);  // either local layout
    if (hipMalloc(&c, vbytes) != hipSuccess || hipMalloc(&y, vbytes) != hipSuccess ||
        hipMalloc(&part, (size_t)nb * prows * ld * csz) != hipSuccess ||
        hipMalloc(&proj, std::max<size_t>(16, (size_t)nb * p->np * csz)) != hipSuccess ||
        hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) {
        (void)hipGetLastError();
        cleanup();
        return set_error(MB_ERR_OOM, "mb_autotune: scratch allocation failed");
    }
    (void)hipMemsetAsync(c, 0, vbytes, s);
    (void)hipMemsetAsync(proj, 0, std::max<size_t>(16, (size_t)nb * p->np * csz), s);
    // average time of 3 calls after one warm-up; < 0 when the configuration is unsupported
    auto timeit = [&](auto&& call) -> double {
        mb_status r = call();
        if (r == MB_ERR_INVALID_ARG) return -1.0;
        if (r != MB_OK) { st = r; return -1.0; }
        (void)hipEventRecord(e0, s);
        for (int rep = 0; rep < 3; ++rep) {
            r = call();
            if (r != MB_OK) { st = r; return -1.0; }
        }
        (void)hipEventRecord(e1, s);
        if (hipEventSynchronize(e1) != hipSuccess) { st = set_error(MB_ERR_HIP, "mb_autotune: event"); return -1.0; }
        float ms = 0.f;
        (void)hipEventElapsedTime(&ms, e0, e1);
        return ms / 3.0;
    };
    // a candidate = a local kernel (kind 0 line-per-thread at an LDS budget, 1 two-step,
    // 2 generic, 3 plane kernel in lane split var) followed by the combine pass that
    // projects its output (the plane kernel's rows per Gauss plane lengthen that pass);
    // each launcher reports a grid it cannot take
    auto candidate = [&](int kind, int budget, int var) -> mb_status {
        kp.tune[cls] = mb::KPoint::Tune{1, kind, budget, -1, var};
        mb_status r;
        if (kind == 0) r = mb::launch_local_lines(p, ik, c, part, nb, ld, cls, s, budget);
        else if (kind == 1) r = mb::launch_local_split(p, ik, c, part, nb, ld, cls, s);
        else if (kind == 2) r = mb::launch_local(p, ik, c, part, nb, ld, cls, s);
        else r = mb::launch_local_plane(p, ik, c, part, nb, ld, cls, s);
        if (r != MB_OK) return r;
        if (kind == 3) return mb::launch_zcombine(p, ik, c, part, nullptr, y, nullptr, nb, ld, cls, s);
        return mb::launch_combine(p, ik, c, part, nullptr, y, nullptr, nb, ld, cls, s);
    };
    // the untuned choice first
    kp.tune[cls] = mb::KPoint::Tune{};
    const double t_default = timeit([&]() {
        const bool planes = mb::local_uses_planes(p, ik, cls);
        mb_status r = planes ? mb::launch_local_plane(p, ik, c, part, nb, ld, cls, s)
                             : mb::launch_local(p, ik, c, part, nb, ld, cls, s);
        if (r != MB_OK) return r;
        if (planes) return mb::launch_zcombine(p, ik, c, part, nullptr, y, nullptr, nb, ld, cls, s);
        return mb::launch_combine(p, ik, c, part, nullptr, y, nullptr, nb, ld, cls, s);
    });
    int best_kind = -1, best_budget = 110, best_var = 0, ncand = 0;
    double best = 1e300;
    const int budgets[] = {22, 44, 66, 88, 110, 160};
    for (int bk : budgets) {
        const double t = timeit([&]() { return candidate(0, bk, 0); });
        if (st != MB_OK) break;
        if (t >= 0) { ++ncand; if (t < best) { best = t; best_kind = 0; best_budget = bk; } }
    }
    for (int kind = 1; kind <= 2 && st == MB_OK; ++kind) {
        const double t = timeit([&]() { return candidate(kind, 110, 0); });
        if (t >= 0) { ++ncand; if (t < best) { best = t; best_kind = kind; best_budget = 110; } }
    }
    for (int var = 0; var <= 1 && st == MB_OK; ++var) {
        const double t = timeit([&]() { return candidate(3, 110, var); });
        if (t >= 0) { ++ncand; if (t < best) { best = t; best_kind = 3; best_budget = 110; best_var = var; } }
    }
    // bands per thread of the partial-row combine pass with the projector expansion
    int combine_bb = 0;
    if (st == MB_OK && best_kind >= 0 && best_kind != 3 && p->np > 0) {
        double tb[2] = {-1.0, -1.0};
        const int bbs[2] = {1, 4};
        for (int v = 0; v < 2 && st == MB_OK; ++v) {
            kp.tune[cls] = mb::KPoint::Tune{1, best_kind, best_budget, -1, best_var, bbs[v]};
            tb[v] = timeit([&]() { return mb::launch_combine(p, ik, c, part, proj, y, nullptr, nb, ld, cls, s); });
        }
        if (st == MB_OK && tb[0] >= 0 && tb[1] >= 0) {
            combine_bb = tb[1] < tb[0] ? 4 : 1;
            ncand += 2;
        }
    }
    int nl_mfma = -1;
    double nl_best = 0.0;
    if (st == MB_OK && p->np > 0 && cls == 1) {
        const double tv = timeit([&]() { return mb::launch_nl_project(p, ik, c, proj, nb, ld, 1, s); });
        const double tm = timeit([&]() { return mb::launch_nl_project_mfma(p, ik, c, proj, nb, ld, 1, false, s); });
        if (st == MB_OK && tv >= 0 && tm >= 0) {
            nl_mfma = tm < tv ? 1 : 0;
            nl_best = std::min(tv, tm);
            ncand += 2;
        }
    }
    if (st != MB_OK || best_kind < 0) {
        kp.tune[cls] = saved;
        cleanup();
        return st != MB_OK ? st : set_error(MB_ERR_INVALID_ARG, "mb_autotune: no local kernel ran");
    }
    kp.tune[cls] = mb::KPoint::Tune{1, best_kind, best_budget, nl_mfma, best_var, combine_bb};
    if (cls == 1) kp.tune[2] = kp.tune[1];  // complex128 vectors with FP32 arithmetic (mixed solver)
    cleanup();
    if (info) {
        info->local_kernel = best_kind;
        info->lds_budget_kb = best_budget;
        info->plane_variant = best_var;
        info->nl_matrix_cores = nl_mfma;
        info->combine_bands = combine_bb;
        info->candidates = ncand;
        info->local_ms = best;
        info->local_default_ms = t_default;
        info->nl_ms = nl_best;
    }
    return MB_OK;
}

mb_status mb_tune_get(const mb_problem* h, int ik, mb_precision prec, mb_tune_info* info) {
    if (mb::refuse_wire(h, "mb_tune_get") != MB_OK) return MB_ERR_INVALID_ARG;
    if (!h || !info) return set_error(MB_ERR_INVALID_ARG, "mb_tune_get: NULL argument");
    if (ik < 0 || ik >= (int)h->p.kp.size()) return set_error(MB_ERR_INVALID_ARG, "mb_tune_get: ik out of range");
    if (prec != MB_FP64 && prec != MB_FP32 && prec != MB_BF16X3)
        return set_error(MB_ERR_INVALID_ARG, "mb_tune_get: unknown precision");
    const mb::KPoint::Tune& t = h->p.kp[ik].tune[prec == MB_FP64 ? 0 : 1];
    *info = mb_tune_info{};
    info->local_kernel = t.set ? t.kind : -1;
    info->lds_budget_kb = t.budget_kb;
    info->plane_variant = t.plane_var;
    info->nl_matrix_cores = t.nl_mfma;
    info->combine_bands = t.combine_bb;
    return MB_OK;
}

mb_status mb_tune_set(mb_problem* h, int ik, mb_precision prec, const mb_tune_info* info) {
    if (mb::refuse_wire(h, "mb_tune_set") != MB_OK) return MB_ERR_INVALID_ARG;
    if (!h || !info) return set_error(MB_ERR_INVALID_ARG, "mb_tune_set: NULL argument");
    mb::Problem& p = h->p;
    if (ik < 0 || ik >= (int)p.kp.size()) return set_error(MB_ERR_INVALID_ARG, "mb_tune_set: ik out of range");
    if (prec != MB_FP64 && prec != MB_FP32 && prec != MB_BF16X3)
        return set_error(MB_ERR_INVALID_ARG, "mb_tune_set: unknown precision");
    return mb::apply_tune(&p, ik, prec == MB_FP64 ? 0 : 1, info->local_kernel, info->lds_budget_kb,
                          info->plane_variant, info->nl_matrix_cores, info->combine_bands);
}

mb_status mb_tune_save(const mb_problem* h, const char* path) {
    if (mb::refuse_wire(h, "mb_tune_save") != MB_OK) return MB_ERR_INVALID_ARG;
    if (!h || !path) return set_error(MB_ERR_INVALID_ARG, "mb_tune_save: NULL argument");
    return mb::tune_save(&h->p, path);
}

mb_status mb_tune_load(mb_problem* h, const char* path, int* applied) {
    if (mb::refuse_wire(h, "mb_tune_load") != MB_OK) return MB_ERR_INVALID_ARG;
    if (!h || !path) return set_error(MB_ERR_INVALID_ARG, "mb_tune_load: NULL argument");
    return mb::tune_load(&h->p, path, applied);
}

mb_status spsi_apply(mb_problem* h, int ik, const void* c, void* y, int64_t nbands, int64_t ld, mb_precision prec,
                     void* stream) {
    mb_status st = mb::check_vec_args(h, ik, c, y, nbands, ld, "spsi_apply");
    if (st != MB_OK) return st;
    if (prec != MB_FP64 && prec != MB_FP32 && prec != MB_BF16X3)
        return set_error(MB_ERR_INVALID_ARG, "spsi_apply: unknown precision");
    size_t bytes = (size_t)nbands * h->p.nb * ld * (prec == MB_FP64 ? 16 : 8);
    if (nbands > 0 && mb::ranges_overlap(c, bytes, y, bytes))
        return set_error(MB_ERR_INVALID_ARG, "spsi_apply: c and y overlap");
    if (nbands == 0) return MB_OK;
    if (h->p.wire)
        return mb::wire_spsi(&h->p, ik, c, y, (int)nbands, (int)ld, prec == MB_FP64 ? 0 : 1, (hipStream_t)stream);
    return mb::launch_spsi(&h->p, ik, c, y, (int)nbands, (int)ld, prec == MB_FP64 ? 0 : 1, (hipStream_t)stream);
}

mb_status s_solve(mb_problem* h, int ik, const void* r, void* x, int64_t nbands, int64_t ld, mb_precision prec,
                  void* stream) {
    mb_status st = mb::check_vec_args(h, ik, r, x, nbands, ld, "s_solve");
    if (st != MB_OK) return st;
    if (prec != MB_FP64 && prec != MB_FP32 && prec != MB_BF16X3)
        return set_error(MB_ERR_INVALID_ARG, "s_solve: unknown precision");
    size_t bytes = (size_t)nbands * h->p.nb * ld * (prec == MB_FP64 ? 16 : 8);
    if (nbands > 0 && r != x && mb::ranges_overlap(r, bytes, x, bytes))
        return set_error(MB_ERR_INVALID_ARG, "s_solve: r and x partially overlap");
    if (nbands == 0) return MB_OK;
    if (h->p.wire)
        return mb::wire_ssolve(&h->p, ik, r, x, (int)nbands, (int)ld, prec == MB_FP64 ? 0 : 1, (hipStream_t)stream);
    return mb::launch_ssolve(&h->p, ik, r, x, (int)nbands, (int)ld, prec == MB_FP64 ? 0 : 1, (hipStream_t)stream);
}

mb_status density_accumulate(mb_problem* h, int ik, const void* c, int64_t nbands, int64_t ld, const double* w,
                             double* rho, mb_precision prec, void* stream) {
    mb_status st = mb::check_vec_args(h, ik, c, rho, nbands, ld, "density_accumulate");
    if (st != MB_OK) return st;
    if (mb::refuse_wire(h, "density_accumulate") != MB_OK) return MB_ERR_INVALID_ARG;
    if (prec != MB_FP64 && prec != MB_FP32 && prec != MB_BF16X3)
        return set_error(MB_ERR_INVALID_ARG, "density_accumulate: unknown precision");
    if (nbands > 0 && !w) return set_error(MB_ERR_INVALID_ARG, "density_accumulate: NULL weights");
    const mb::Problem& p = h->p;
    const size_t vbytes = (size_t)nbands * p.nb * ld * (prec == MB_FP64 ? 16 : 8);
    const size_t rbytes = (size_t)p.nzq * p.N1 * p.N2 * sizeof(double);
    if (nbands > 0 && mb::ranges_overlap(c, vbytes, rho, rbytes))
        return set_error(MB_ERR_INVALID_ARG, "density_accumulate: c and rho overlap");
    if (nbands == 0) return MB_OK;
    return mb::launch_density(&h->p, ik, c, (int)nbands, (int)ld, w, rho, prec == MB_FP64 ? 0 : 1,
                              (hipStream_t)stream);
}

mb_status hartree_potential(mb_problem* h, const double* rho, double* vh, void* vzg, void* stream) {
    if (mb::refuse_wire(h, "hartree_potential") != MB_OK) return MB_ERR_INVALID_ARG;
    if (!h) return set_error(MB_ERR_INVALID_ARG, "hartree_potential: problem is NULL");
    mb::Problem& p = h->p;
    if (p.device < 0) return set_error(MB_ERR_NO_DEVICE, "hartree_potential: host-only problem");
    if (!rho || !vh) return set_error(MB_ERR_INVALID_ARG, "hartree_potential: NULL density or potential");
    const size_t rbytes = (size_t)p.nzq * p.N1 * p.N2 * sizeof(double);
    if (vzg && (mb::ranges_overlap(vzg, 2 * rbytes, rho, rbytes) || mb::ranges_overlap(vzg, 2 * rbytes, vh, rbytes)))
        return set_error(MB_ERR_INVALID_ARG, "hartree_potential: vzg overlaps the density or the potential");
    if (rho != vh && mb::ranges_overlap(rho, rbytes, vh, rbytes))
        return set_error(MB_ERR_INVALID_ARG, "hartree_potential: rho and vh partially overlap");
    mb_status st = mb::ensure_ws(p.ws_hartree, mb::hartree_work_bytes(&p, vzg != nullptr));
    if (st != MB_OK) return st;
    return mb::launch_hartree(&p, rho, vh, vzg, p.ws_hartree.ptr, (hipStream_t)stream);
}

}  // extern "C"

// internal access for the eigensolver translation unit
namespace mb {
Problem* problem_of(mb_problem* h) { return h ? &h->p : nullptr; }
}  // namespace mb
