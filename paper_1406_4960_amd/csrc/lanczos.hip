// Generalized Lanczos-Krylov eigensolver (Sec. II.C).
#include "mbks_internal.h"

extern "C" void mb_lanczos_default_opts(mb_lanczos_opts* o) {
    if (!o) return;
    o->block = 1;
    o->krylov = 2;
    o->krylov_global = 2;
    o->max_iter = 200;
    o->tol = 1e-7;
    o->sigma = 1.0;
    o->switch_tol = 1e-4;
    o->seed = 14064960ull;
}

extern "C" mb_status lanczos_lowest(mb_problem*, int, int, mb_precision, const mb_lanczos_opts*, const void*,
                                    double*, void*, mb_lanczos_info*, void*) {
    return mb::set_error(MB_ERR_INVALID_ARG, "lanczos_lowest: not built yet");
}
