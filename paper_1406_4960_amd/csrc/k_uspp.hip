// Ultrasoft overlap (Sec. II.B.2): S = S_0 + sum_p q_p |beta_p><beta_p| with
// S_0 = I_G (x) S_z and beta_p(G, i) = F_p(G) Z_p(i).
//   S c:      projections q_p <beta_p|c> (the projection kernels of H), then the banded
//             pass with the expansion sum_p |beta_p> q_p <beta_p|c> added to its output.
//   S^{-1} r: Woodbury identity S^{-1} = S_0^{-1} - S_0^{-1} B W B^H S_0^{-1} with the
//             N_p x N_p matrix W = Q (I + B^H S_0^{-1} B Q)^{-1} built on the host:
//               x = S_0^{-1} r,  P = B^H x,  P' = -W P,  t = r + B P',  x = S_0^{-1} t
//             (the expansion B P' by the banded pass with an identity band, so that
//             only the z-windows of the projectors are touched).
// Without augmentation charges both are the banded operators alone.
#include "cplx.h"
#include "mbks_internal.h"

namespace mb {

namespace {

// Pq[b][a] = -sum_c W[a][c] P[b][c], FP64 arithmetic (W row-major, np x np)
template <typename T>
__global__ __launch_bounds__(256) void k_aug_mix(const cx<double>* W, const cx<T>* P, cx<T>* Pq, int nbands,
                                                  int np) {
    const int idx = blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= nbands * np) return;
    const int b = idx / np, a = idx - b * np;
    const cx<double>* w = W + (size_t)a * np;
    const cx<T>* pb = P + (size_t)b * np;
    double re = 0.0, im = 0.0;
    for (int c = 0; c < np; ++c) {
        const cx<double> wv = w[c];
        const cx<T> pv = pb[c];
        re += wv.x * (double)pv.x - wv.y * (double)pv.y;
        im += wv.x * (double)pv.y + wv.y * (double)pv.x;
    }
    Pq[idx] = mk<T>((T)(-re), (T)(-im));
}

size_t proj_elem(int prec) { return prec == 1 ? sizeof(cx<float>) : sizeof(cx<double>); }

}  // namespace

mb_status launch_spsi(Problem* p, int ik, const void* c, void* y, int nbands, int ld, int prec, hipStream_t s) {
    if (p->wire) return wire_spsi(p, ik, c, y, nbands, ld, prec, s);
    if (!p->uspp) return launch_spsi_banded(p, ik, c, y, nbands, ld, prec, s);
    if (nbands == 0) return MB_OK;
    KPoint& kp = p->kp[ik];
    mb_status st = ensure_hws(kp, kp.ws_proj, hwork_proj_bytes(p, nbands, prec));
    if (st != MB_OK) return st;
    void* projq = kp.ws_proj.ptr;
    st = project(p, ik, c, projq, nbands, ld, prec, s, nullptr, PROJ_Q, nullptr);
    if (st != MB_OK) return st;
    return launch_combine(p, ik, c, nullptr, nullptr, nullptr, y, nbands, ld, prec, s, false, projq, nullptr);
}

mb_status launch_ssolve(Problem* p, int ik, const void* r, void* x, int nbands, int ld, int prec, hipStream_t s) {
    if (p->wire) return wire_ssolve(p, ik, r, x, nbands, ld, prec, s);
    if (!p->uspp) return launch_ssolve_banded(p, ik, r, x, nbands, ld, prec, s);
    if (nbands == 0) return MB_OK;
    KPoint& kp = p->kp[ik];
    if (!kp.d_W) return set_error(MB_ERR_INVALID_ARG, "s_solve: ultrasoft Woodbury matrix not uploaded");
    const void* rr = r;
    if (r == x) {
        const size_t bytes = aux_bytes(p, ik, nbands, ld, prec);
        mb_status st = ensure_hws(kp, kp.ws_aux, bytes);
        if (st != MB_OK) return st;
        MB_HIP_TRY(hipMemcpyAsync(kp.ws_aux.ptr, r, bytes, hipMemcpyDeviceToDevice, s));
        rr = kp.ws_aux.ptr;
    }
    mb_status st = ensure_hws(kp, kp.ws_proj, hwork_proj_bytes(p, nbands, prec));
    if (st != MB_OK) return st;
    void* P = kp.ws_proj.ptr;
    void* Pq = (char*)kp.ws_proj.ptr + (size_t)nbands * p->np * proj_elem(prec);
    st = launch_ssolve_banded(p, ik, rr, x, nbands, ld, prec, s);
    if (st != MB_OK) return st;
    st = project(p, ik, x, P, nbands, ld, prec, s, nullptr, PROJ_ONE, nullptr);
    if (st != MB_OK) return st;
    const int tot = nbands * p->np;
    if (prec == 1)
        hipLaunchKernelGGL(k_aug_mix<float>, dim3((tot + 255) / 256), dim3(256), 0, s, (const cx<double>*)kp.d_W,
                           (const cx<float>*)P, (cx<float>*)Pq, nbands, p->np);
    else
        hipLaunchKernelGGL(k_aug_mix<double>, dim3((tot + 255) / 256), dim3(256), 0, s, (const cx<double>*)kp.d_W,
                           (const cx<double>*)P, (cx<double>*)Pq, nbands, p->np);
    MB_HIP_TRY(hipGetLastError());
    st = launch_combine(p, ik, rr, nullptr, nullptr, nullptr, x, nbands, ld, prec, s, false, Pq, p->d_iband);
    if (st != MB_OK) return st;
    return launch_ssolve_banded(p, ik, x, x, nbands, ld, prec, s);
}

}  // namespace mb
