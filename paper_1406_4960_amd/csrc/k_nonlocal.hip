// Kleinman-Bylander projections (eq. KBeq and its matrix elements, Sec. II.B.1):
//   proj[b][p] = E_p <beta_p | c_b> = E_p sum_{i in window(p)} Z_p(i) sum_G conj(F_p(G)) c_b(G, i)
// using the factorisation <G,i|beta_p> = F_p(G) Z_p(i) (the paper's Z Q split with
// the phase and normalisation folded into F).  The expansion sum_p |beta_p> proj
// is fused into the combine kernel.  The same projections serve the ultrasoft
// overlap (Sec. II.B.2): a second output q_p <beta_p|c_b>, or other scales in place of E_p.
#include "cplx.h"
#include "mbks_internal.h"

namespace mb {

namespace {

template <typename TI, typename T, int NT>
__global__ __launch_bounds__(NT) void k_nl_project(const cx<TI>* c, const cx<T>* F, const T* Z, const T* E,
                                                   const int32_t* zwin, cx<T>* proj, const T* Q, cx<T>* projq,
                                                   int nbands, int np, int ng, int nb, int ld) {
    const int p = blockIdx.x;
    const int b = blockIdx.y;
    const int lo = zwin[2 * p], hi = zwin[2 * p + 1];
    const cx<TI>* cb = c + (size_t)b * nb * ld;
    const cx<T>* Fp = F + (size_t)p * ld;
    const T* Zp = Z + (size_t)p * nb;
    cx<T> acc = mk<T>(0, 0);
    for (int g = threadIdx.x; g < ng; g += NT) {
        cx<T> f = Fp[g];
        cx<T> colsum = mk<T>(0, 0);  // sum_i Z_p(i) c(G, i)
        for (int i = lo; i <= hi; ++i) {
            cx<TI> v = cb[(size_t)i * ld + g];
            T z = Zp[i];
            colsum.x += z * (T)v.x;
            colsum.y += z * (T)v.y;
        }
        cfmac(acc, f, colsum);
    }
    __shared__ cx<T> red[NT];
    red[threadIdx.x] = acc;
    __syncthreads();
    for (int w = NT / 2; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) red[threadIdx.x] = cadd(red[threadIdx.x], red[threadIdx.x + w]);
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        proj[(size_t)b * np + p] = cscale(red[0], E[p]);
        if (projq) projq[(size_t)b * np + p] = cscale(red[0], Q[p]);
    }
}

}  // namespace

// prec: 0 = FP64, 1 = FP32 (c64), 2 = c128 vectors, FP32 arithmetic
mb_status launch_nl_project(Problem* p, int ik, const void* c, void* proj, int nbands, int ld, int prec,
                            hipStream_t s, int scale, void* projq) {
    if (p->np == 0) return MB_OK;
    const KPoint& kp = p->kp[ik];
    dim3 grid(p->np, nbands);
    const double* sc = scale == PROJ_Q ? p->d_Q : scale == PROJ_ONE ? p->d_one : p->d_E;
    const float* scf = scale == PROJ_Q ? p->d_Qf : scale == PROJ_ONE ? p->d_onef : p->d_Ef;
    StageScope ts_(MB_STAGE_NL_PROJECT, s, nbands);
    if (prec == 0)
        hipLaunchKernelGGL((k_nl_project<double, double, 256>), grid, dim3(256), 0, s, (const cx<double>*)c,
                           (const cx<double>*)kp.d_F64, p->d_Z, sc, p->d_zwin, (cx<double>*)proj, p->d_Q,
                           (cx<double>*)projq, nbands, p->np, kp.ng, p->nb, ld);
    else if (prec == 1)
        hipLaunchKernelGGL((k_nl_project<float, float, 256>), grid, dim3(256), 0, s, (const cx<float>*)c,
                           (const cx<float>*)kp.d_F32, p->d_Zf, scf, p->d_zwin, (cx<float>*)proj, p->d_Qf,
                           (cx<float>*)projq, nbands, p->np, kp.ng, p->nb, ld);
    else
        hipLaunchKernelGGL((k_nl_project<double, float, 256>), grid, dim3(256), 0, s, (const cx<double>*)c,
                           (const cx<float>*)kp.d_F32, p->d_Zf, scf, p->d_zwin, (cx<float>*)proj, p->d_Qf,
                           (cx<float>*)projq, nbands, p->np, kp.ng, p->nb, ld);
    MB_HIP_TRY(hipGetLastError());
    return MB_OK;
}

}  // namespace mb
