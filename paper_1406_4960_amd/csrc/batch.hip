// Many independent problems at once: the operator H applied to the vector blocks
// of a list of (problem, k-point) items of different sizes in a few launches,
// and the eigensolver run over such a list.
//
// The in-plane work (evaluate / FFT / V / FFT / project, Sec. II.B.1) of all items
// with the same grid shares one launch of the line-per-thread kernel (small grids) or
// of the two-step line kernel (larger grids); the remaining items share the generic
// kernel's launches; the banded
// combine (kinetic part, local partial sums, projector expansion) is one launch over
// every item.  Work units of a launch are laid out item after item; each block
// finds its item by binary search in a table of first units.
#include <algorithm>
#include <atomic>
#include <cstring>
#include <map>
#include <string>
#include <thread>
#include <vector>

#include "mbks_internal.h"

namespace {
constexpr size_t STAGE_BYTES = 1 << 20;        // descriptor staging per slot
constexpr size_t PART_BUDGET = size_t(4) << 30;  // local partial rows per chunk of items
}  // namespace

struct mb_batch {
    struct Item {
        mb::Problem* p;
        int ik;
    };
    std::vector<Item> items;
    int device = 0;
    mb::Workspace part, proj;
    // two staging slots used in turn; a slot is refilled only after the copies
    // that read it (recorded by `done`) have executed
    struct Slot {
        char* host = nullptr;
        char* dev = nullptr;
        hipEvent_t done = nullptr;
        bool pending = false;
    } slot[2];
    int next = 0;
    // bound vector blocks (mb_batch_bind): the arguments of every bound call, their own work
    // buffers and a staging slot of their own whose contents are the same on every call, so
    // that a captured graph's descriptor copies replay correctly
    struct Bound {
        bool on = false;
        std::vector<const void*> c;
        std::vector<void*> y;
        std::vector<int64_t> nbands, ld;
        mb_precision prec = MB_FP64;
        mb::Workspace part, proj, nlpart;
        Slot slot;
    } bound;
};

namespace mb {
namespace {

#define BT_TRY(call)                \
    do {                            \
        mb_status s_ = (call);      \
        if (s_ != MB_OK) return s_; \
    } while (0)

void free_batch(mb_batch* b) {
    for (auto& sl : b->slot) {
        if (sl.done) (void)hipEventSynchronize(sl.done);
        if (sl.done) (void)hipEventDestroy(sl.done);
        if (sl.host) (void)hipHostFree(sl.host);
        if (sl.dev) (void)hipFree(sl.dev);
    }
    if (b->part.ptr) (void)hipFree(b->part.ptr);
    if (b->proj.ptr) (void)hipFree(b->proj.ptr);
    if (b->bound.on || b->bound.slot.host) (void)hipDeviceSynchronize();
    if (b->bound.slot.host) (void)hipHostFree(b->bound.slot.host);
    if (b->bound.slot.dev) (void)hipFree(b->bound.slot.dev);
    for (mb::Workspace* w : {&b->bound.part, &b->bound.proj, &b->bound.nlpart})
        if (w->ptr) (void)hipFree(w->ptr);
    delete b;
}

// the projection path of an item inside a batch: matrix cores for BF16x3 and for FP32 /
// FP64 with at least 64 projectors, the vector kernel otherwise
bool item_uses_mfma(const mb::Problem* p, int prec) { return prec == 3 || p->np >= 64; }


mb_status apply_chunk(std::vector<BatchItem>& chunk, int prec, int lp, TableUploader& up, hipStream_t s) {
    // projections <beta_p|c> per item (a8, a9)
    for (auto& it : chunk) {
        if (it.p->np == 0 || it.nbands == 0) {
            it.proj = nullptr;
            continue;
        }
        // as in the single-item operator: matrix cores for BF16x3 and for FP32 / FP64
        // with at least 64 projectors, the vector kernel otherwise
        if (!item_uses_mfma(it.p, prec))
            BT_TRY(launch_nl_project(it.p, it.ik, it.c, it.proj, it.nbands, it.ld, lp, s));
        else
            BT_TRY(launch_nl_project_mfma(it.p, it.ik, it.c, it.proj, it.nbands, it.ld,
                                          prec == 3 ? 2 : lp == 0 ? 0 : 1, false, s, it.nlpart));
    }
    // local potential, grouped by grid
    std::map<std::pair<int, int>, std::vector<BatchItem>> by_grid;
    for (const auto& it : chunk)
        if (it.nbands > 0) by_grid[{it.p->N1, it.p->N2}].push_back(it);
    std::vector<BatchItem> generic;
    for (auto& kv : by_grid) {
        mb_status st = launch_local_lines_batch(kv.second, lp, up, s);
        if (st == MB_ERR_INVALID_ARG) st = launch_local_split_batch(kv.second, lp, up, s);
        if (st == MB_ERR_INVALID_ARG)
            generic.insert(generic.end(), kv.second.begin(), kv.second.end());
        else if (st != MB_OK)
            return st;
    }
    if (!generic.empty()) BT_TRY(launch_local_batch(generic, lp, up, s));
    std::vector<BatchItem> live;
    for (const auto& it : chunk)
        if (it.nbands > 0) live.push_back(it);
    return launch_combine_batch(live, lp, up, s);
}

// bytes of the bound work buffers for the bound arguments (proj, partial rows, matrix-core
// partials); the same arithmetic as apply_batched's
struct BatchSizes {
    size_t proj = 0, part = 0, nlpart = 0;
};

mb_status apply_batched(mb_batch* b, const void* const* c, void* const* y, const int64_t* nbands,
                        const int64_t* ld, mb_precision prec, hipStream_t s, bool bound = false,
                        BatchSizes* sizes_only = nullptr) {
    const int n = (int)b->items.size();
    const int lp = prec == MB_FP64 ? 0 : 1;               // local / combine precision
    const int kprec = prec == MB_FP64 ? 0 : prec == MB_FP32 ? 1 : 3;
    const size_t csz = lp == 0 ? 16 : 8;
    std::vector<BatchItem> all(n);
    size_t proj_total = 0, part_max = 0, part_total = 0, nl_total = 0;
    for (int t = 0; t < n; ++t) {
        Problem* p = b->items[t].p;
        const int ik = b->items[t].ik;
        const int64_t nbt = nbands[t];
        const int64_t ldt = ld ? ld[t] : recommended_ld(p->kp[ik].ng);
        const std::string what = "hpsi_apply_batched: item " + std::to_string(t);
        if (nbt < 0 || nbt > (1 << 20)) return set_error(MB_ERR_INVALID_ARG, what + ": nbands");
        if (ldt < p->kp[ik].ng || ldt > (1 << 24)) return set_error(MB_ERR_INVALID_ARG, what + ": ld < N_G");
        if (nbt > 0 && (!c[t] || !y[t])) return set_error(MB_ERR_INVALID_ARG, what + ": NULL vector");
        const size_t bytes = (size_t)nbt * p->nb * ldt * csz;
        if (nbt > 0 && ranges_overlap(c[t], bytes, y[t], bytes))
            return set_error(MB_ERR_INVALID_ARG, what + ": c and y overlap");
        all[t] = BatchItem{p, ik, c[t], y[t], nullptr, nullptr, (int)nbt, (int)ldt};
        const size_t pb = ((size_t)nbt * p->nint * 4 * ldt * csz + 255) / 256 * 256;
        if (pb > PART_BUDGET) return set_error(MB_ERR_INVALID_ARG, what + ": block too large for one launch");
        part_max = std::max(part_max, pb);
        part_total += pb;
        proj_total += ((size_t)nbt * p->np * csz + 255) / 256 * 256;
        if (bound && p->np > 0 && nbt > 0 && item_uses_mfma(p, kprec))
            nl_total += (nl_mfma_part_bytes(p, (int)nbt, kprec == 3 ? 2 : lp == 0 ? 0 : 1) + 255) / 256 * 256;
    }
    const size_t proj_need = std::max<size_t>(proj_total, 256);
    const size_t part_need = std::max<size_t>(std::min(PART_BUDGET, part_total), 256);
    if (sizes_only) {
        sizes_only->proj = proj_need;
        sizes_only->part = part_need;
        sizes_only->nlpart = std::max<size_t>(nl_total, 256);
        return MB_OK;
    }
    mb::Workspace& wproj = bound ? b->bound.proj : b->proj;
    mb::Workspace& wpart = bound ? b->bound.part : b->part;
    if (bound) {
        // the bound call allocates nothing: its buffers were sized by mb_batch_bind
        if (wproj.bytes < proj_need || wpart.bytes < part_need || b->bound.nlpart.bytes < nl_total)
            return set_error(MB_ERR_INVALID_ARG, "hpsi_apply_batched_bound: bound work buffers too small");
    } else {
        BT_TRY(ensure_ws(wproj, proj_need));
        // partial rows of as many consecutive items as fit the budget (at least the largest item)
        BT_TRY(ensure_ws(wpart, part_need));
    }
    const size_t part_cap = wpart.bytes;
    {
        size_t off = 0, noff = 0;
        for (auto& it : all) {
            it.proj = (char*)wproj.ptr + off;
            off += ((size_t)it.nbands * it.p->np * csz + 255) / 256 * 256;
            if (bound && it.p->np > 0 && it.nbands > 0 && item_uses_mfma(it.p, kprec)) {
                it.nlpart = (char*)b->bound.nlpart.ptr + noff;
                noff += (nl_mfma_part_bytes(it.p, it.nbands, kprec == 3 ? 2 : lp == 0 ? 0 : 1) + 255) / 256 * 256;
            }
        }
    }
    TableUploader up;
    up.cap = STAGE_BYTES;
    mb_batch::Slot* slp = nullptr;
    if (bound) {
        up.host = b->bound.slot.host;
        up.dev = b->bound.slot.dev;
    } else {
        slp = &b->slot[b->next];
        b->next ^= 1;
        if (slp->pending) {
            MB_HIP_TRY(hipEventSynchronize(slp->done));
            slp->pending = false;
        }
        up.host = slp->host;
        up.dev = slp->dev;
    }
    struct MaybeGuard {
        mb_batch::Slot* sl;
        hipStream_t s;
        ~MaybeGuard() {
            if (sl && hipEventRecord(sl->done, s) == hipSuccess) sl->pending = true;
        }
    } guard{slp, s};
    // chunks of consecutive items whose partial rows fit the workspace together
    std::vector<BatchItem> chunk;
    size_t used = 0;
    for (auto& it : all) {
        const size_t pb = ((size_t)it.nbands * it.p->nint * 4 * it.ld * csz + 255) / 256 * 256;
        if (!chunk.empty() && used + pb > part_cap) {
            BT_TRY(apply_chunk(chunk, kprec, lp, up, s));
            chunk.clear();
            used = 0;
        }
        it.part = (char*)wpart.ptr + used;
        used += pb;
        chunk.push_back(it);
    }
    if (!chunk.empty()) BT_TRY(apply_chunk(chunk, kprec, lp, up, s));
    return MB_OK;
}

struct SolveJob {
    std::vector<int> items;  // of one (problem, k-point), solved in order
};

}  // namespace
}  // namespace mb

using mb::set_error;

extern "C" {

mb_status mb_batch_create(mb_problem* const* probs, const int* iks, int nitems, mb_batch** out) {
    if (!out) return set_error(MB_ERR_INVALID_ARG, "mb_batch_create: out is NULL");
    *out = nullptr;
    if (!probs || !iks || nitems < 1 || nitems > 65536)
        return set_error(MB_ERR_INVALID_ARG, "mb_batch_create: need 1..65536 items");
    auto* b = new mb_batch();
    for (int t = 0; t < nitems; ++t) {
        mb::Problem* p = mb::problem_of(probs[t]);
        const std::string what = "mb_batch_create: item " + std::to_string(t);
        mb_status st = MB_OK;
        if (!p)
            st = set_error(MB_ERR_INVALID_ARG, what + ": problem is NULL");
        else if (p->wire)
            st = set_error(MB_ERR_INVALID_ARG, what + ": not available for the 1D-periodic form");
        else if (p->device < 0)
            st = set_error(MB_ERR_NO_DEVICE, what + ": host-only problem");
        else if (iks[t] < 0 || iks[t] >= (int)p->kp.size())
            st = set_error(MB_ERR_INVALID_ARG, what + ": ik out of range");
        else if (p->order != 4)
            st = set_error(MB_ERR_INVALID_ARG, what + ": GPU kernels support order 4 only");
        else if (t > 0 && p->device != b->device)
            st = set_error(MB_ERR_INVALID_ARG, what + ": problems on different devices");
        if (st != MB_OK) {
            delete b;
            return st;
        }
        if (t == 0) b->device = p->device;
        b->items.push_back({p, iks[t]});
    }
    if (hipSetDevice(b->device) != hipSuccess) {
        delete b;
        return set_error(MB_ERR_HIP, "mb_batch_create: hipSetDevice failed");
    }
    for (auto& sl : b->slot) {
        if (hipHostMalloc((void**)&sl.host, STAGE_BYTES, hipHostMallocDefault) != hipSuccess ||
            hipMalloc((void**)&sl.dev, STAGE_BYTES) != hipSuccess ||
            hipEventCreateWithFlags(&sl.done, hipEventDisableTiming) != hipSuccess) {
            (void)hipGetLastError();
            mb::free_batch(b);
            return set_error(MB_ERR_OOM, "mb_batch_create: staging allocation failed");
        }
    }
    *out = b;
    return MB_OK;
}

mb_status mb_batch_destroy(mb_batch* b) {
    if (!b) return MB_OK;
    mb::free_batch(b);
    return MB_OK;
}

mb_status hpsi_apply_batched(mb_batch* b, const void* const* c, void* const* y, const int64_t* nbands,
                             const int64_t* ld, mb_precision prec, void* stream) {
    if (!b || !c || !y || !nbands) return set_error(MB_ERR_INVALID_ARG, "hpsi_apply_batched: NULL argument");
    if (prec != MB_FP64 && prec != MB_FP32 && prec != MB_BF16X3)
        return set_error(MB_ERR_INVALID_ARG, "hpsi_apply_batched: unknown precision");
    return mb::apply_batched(b, c, y, nbands, ld, prec, (hipStream_t)stream);
}

mb_status mb_batch_bind(mb_batch* b, const void* const* c, void* const* y, const int64_t* nbands,
                        const int64_t* ld, mb_precision prec) {
    if (!b || !c || !y || !nbands) return set_error(MB_ERR_INVALID_ARG, "mb_batch_bind: NULL argument");
    if (prec != MB_FP64 && prec != MB_FP32 && prec != MB_BF16X3)
        return set_error(MB_ERR_INVALID_ARG, "mb_batch_bind: unknown precision");
    const int n = (int)b->items.size();
    mb::BatchSizes sz;
    mb_status st = mb::apply_batched(b, c, y, nbands, ld, prec, nullptr, true, &sz);  // validates
    if (st != MB_OK) return st;
    if (hipSetDevice(b->device) != hipSuccess) return set_error(MB_ERR_HIP, "mb_batch_bind: hipSetDevice failed");
    auto& bd = b->bound;
    bd.on = false;
    MB_HIP_TRY(hipDeviceSynchronize());  // no bound call may still read the old buffers
    for (mb::Workspace* w : {&bd.part, &bd.proj, &bd.nlpart}) {
        if (w->ptr) MB_HIP_TRY(hipFree(w->ptr));
        w->ptr = nullptr;
        w->bytes = 0;
    }
    if (mb::ensure_ws(bd.proj, sz.proj) != MB_OK || mb::ensure_ws(bd.part, sz.part) != MB_OK ||
        mb::ensure_ws(bd.nlpart, sz.nlpart) != MB_OK)
        return set_error(MB_ERR_OOM, "mb_batch_bind: work buffer allocation failed");
    if (!bd.slot.host) {
        if (hipHostMalloc((void**)&bd.slot.host, STAGE_BYTES, hipHostMallocDefault) != hipSuccess ||
            hipMalloc((void**)&bd.slot.dev, STAGE_BYTES) != hipSuccess) {
            (void)hipGetLastError();
            return set_error(MB_ERR_OOM, "mb_batch_bind: staging allocation failed");
        }
    }
    bd.c.assign(c, c + n);
    bd.y.assign(y, y + n);
    bd.nbands.assign(nbands, nbands + n);
    bd.ld.resize(n);
    for (int t = 0; t < n; ++t) bd.ld[t] = ld ? ld[t] : mb::recommended_ld(b->items[t].p->kp[b->items[t].ik].ng);
    bd.prec = prec;
    bd.on = true;
    return MB_OK;
}

mb_status hpsi_apply_batched_bound(mb_batch* b, void* stream) {
    if (!b) return set_error(MB_ERR_INVALID_ARG, "hpsi_apply_batched_bound: NULL batch");
    if (!b->bound.on) return set_error(MB_ERR_INVALID_ARG, "hpsi_apply_batched_bound: no blocks bound (mb_batch_bind)");
    auto& bd = b->bound;
    return mb::apply_batched(b, bd.c.data(), bd.y.data(), bd.nbands.data(), bd.ld.data(), bd.prec,
                             (hipStream_t)stream, true);
}

mb_status lanczos_lowest_batched(mb_batch* b, const int* nev, mb_precision prec, const mb_lanczos_opts* opts,
                                 double* const* eig, void* const* x, mb_lanczos_info* info, void* stream) {
    if (!b || !nev || !eig || !x) return set_error(MB_ERR_INVALID_ARG, "lanczos_lowest_batched: NULL argument");
    if (prec != MB_FP64 && prec != MB_FP32 && prec != MB_BF16X3)
        return set_error(MB_ERR_INVALID_ARG, "lanczos_lowest_batched: unknown precision");
    mb_lanczos_opts o;
    mb_lanczos_default_opts(&o);
    if (opts) o = *opts;
    if (o.max_iter < 1 || o.krylov < 1 || o.block < 1 || o.krylov_global < 0 || !(o.tol > 0))
        return set_error(MB_ERR_INVALID_ARG, "lanczos_lowest_batched: bad options");
    const int n = (int)b->items.size();
    for (int t = 0; t < n; ++t) {
        if (nev[t] < 0) return set_error(MB_ERR_INVALID_ARG, "lanczos_lowest_batched: nev < 0");
        if (nev[t] > 0 && (!eig[t] || !x[t]))
            return set_error(MB_ERR_INVALID_ARG, "lanczos_lowest_batched: NULL output");
    }
    hipStream_t caller = (hipStream_t)stream;
    // calls on one k-point of a problem share its workspaces: one job per (problem, k-point)
    std::vector<mb::SolveJob> jobs;
    {
        std::map<std::pair<mb::Problem*, int>, int> idx;
        for (int t = 0; t < n; ++t) {
            if (nev[t] == 0) continue;
            const std::pair<mb::Problem*, int> key{b->items[t].p, b->items[t].ik};
            auto f = idx.find(key);
            if (f == idx.end()) {
                idx[key] = (int)jobs.size();
                jobs.push_back({{t}});
            } else {
                jobs[f->second].items.push_back(t);
            }
        }
    }
    // the solves start after the caller's earlier work on `stream`
    hipEvent_t ready;
    MB_HIP_TRY(hipEventCreateWithFlags(&ready, hipEventDisableTiming));
    MB_HIP_TRY(hipEventRecord(ready, caller));
    int nthreads = mb::timer_enabled() ? 1 : std::max(1, std::min<int>(16, (int)jobs.size()));
    {
        // as many concurrent solves as the free device memory holds (each solve of a
        // large slab takes tens of GB of vectors, released when it ends)
        size_t need = 0;
        for (const auto& jb : jobs)
            for (int t : jb.items)
                need = std::max(need, mb::lanczos_device_bytes(b->items[t].p, b->items[t].ik, nev[t], o));
        size_t freeb = 0, totb = 0;
        if (need > 0 && hipMemGetInfo(&freeb, &totb) == hipSuccess) {
            const size_t fit = (size_t)(0.85 * (double)freeb) / (need + need / 8);
            nthreads = std::max(1, std::min<int>(nthreads, (int)std::min<size_t>(fit, 16)));
        } else {
            (void)hipGetLastError();
        }
    }
    std::vector<mb_status> status(n, MB_OK);
    std::vector<std::string> message(n);
    std::atomic<int> next_job{0};
    std::vector<hipStream_t> streams(nthreads, nullptr);
    std::vector<hipEvent_t> finished(nthreads, nullptr);
    mb_status setup = MB_OK;
    for (int w = 0; w < nthreads && setup == MB_OK; ++w) {
        if (hipStreamCreateWithFlags(&streams[w], hipStreamNonBlocking) != hipSuccess ||
            hipEventCreateWithFlags(&finished[w], hipEventDisableTiming) != hipSuccess)
            setup = set_error(MB_ERR_HIP, "lanczos_lowest_batched: stream creation failed");
    }
    auto worker = [&](int w) {
        (void)hipSetDevice(b->device);
        hipStream_t s = streams[w];
        (void)hipStreamWaitEvent(s, ready, 0);
        for (;;) {
            const int j = next_job.fetch_add(1);
            if (j >= (int)jobs.size()) break;
            for (int t : jobs[j].items) {
                mb_lanczos_info inf{};
                status[t] = mb::lanczos_impl(b->items[t].p, b->items[t].ik, nev[t], prec, o, nullptr, eig[t], x[t],
                                             &inf, s);
                if (status[t] != MB_OK) message[t] = mb_last_error();
                if (info) info[t] = inf;
            }
        }
        (void)hipEventRecord(finished[w], s);
    };
    if (setup == MB_OK) {
        if (nthreads == 1) {
            worker(0);
        } else {
            std::vector<std::thread> pool;
            for (int w = 0; w < nthreads; ++w) pool.emplace_back(worker, w);
            for (auto& th : pool) th.join();
        }
        for (int w = 0; w < nthreads; ++w) (void)hipStreamWaitEvent(caller, finished[w], 0);
    }
    for (int w = 0; w < nthreads; ++w) {
        if (streams[w]) {
            (void)hipStreamSynchronize(streams[w]);
            (void)hipStreamDestroy(streams[w]);
        }
        if (finished[w]) (void)hipEventDestroy(finished[w]);
    }
    (void)hipEventDestroy(ready);
    if (setup != MB_OK) return setup;
    mb_status first = MB_OK;
    for (int t = 0; t < n; ++t) {
        if (status[t] != MB_OK && status[t] != MB_ERR_NOT_CONVERGED) {
            return set_error(status[t], "lanczos_lowest_batched: item " + std::to_string(t) + ": " + message[t]);
        }
        if (status[t] == MB_ERR_NOT_CONVERGED && first == MB_OK) first = MB_ERR_NOT_CONVERGED;
    }
    if (first != MB_OK) return set_error(first, "lanczos_lowest_batched: some items did not converge");
    return MB_OK;
}

}  // extern "C"
