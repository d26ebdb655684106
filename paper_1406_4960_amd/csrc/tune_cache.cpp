// Kernel choices per k-point and precision class: validation, and a persisted cache of
// the autotuner's results in a small JSON file (one entry per line, merged on save).
// An entry is keyed by everything the choice depends on: the GPU architecture and the
// sizes of the k-point's problem (grid, spline order, splines, knot intervals, Gauss
// points per interval, G vectors, projectors, row stride); never by values such as the
// atom positions or the potential, which do not change which kernel is fastest.
#include <cstdio>
#include <cstring>
#include <fstream>
#include <map>
#include <sstream>
#include <string>
#include <vector>

#include "mbks_internal.h"

namespace mb {

namespace {

constexpr const char* kFormat = "mbks-tune-1";

struct Entry {
    std::string key;
    int cls = 0, kind = -1, budget = 110, var = 0, nl = -1, bb = 0;
};

std::string arch_of(const Problem* p) {
    if (p->device < 0) return "host";
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, p->device) != hipSuccess) {
        (void)hipGetLastError();
        return "unknown";
    }
    std::string a = prop.gcnArchName;  // e.g. "gfx950:sramecc+:xnack-"
    const size_t colon = a.find(':');
    return colon == std::string::npos ? a : a.substr(0, colon);
}

std::string key_of(const Problem* p, const KPoint& kp, const std::string& arch) {
    char buf[256];
    std::snprintf(buf, sizeof buf, "%s/grid%dx%d/order%d/nb%d/nint%d/nq%d/ng%d/np%d/ld%d", arch.c_str(), p->N1,
                  p->N2, p->order, p->nb, p->nint, p->nq, kp.ng, p->np, kp.ld);
    return buf;
}

std::string format_entry(const Entry& e) {
    char buf[512];
    std::snprintf(buf, sizeof buf,
                  "  {\"key\": \"%s\", \"class\": %d, \"local_kernel\": %d, \"lds_budget_kb\": %d, "
                  "\"plane_variant\": %d, \"nl_matrix_cores\": %d, \"combine_bands\": %d}",
                  e.key.c_str(), e.cls, e.kind, e.budget, e.var, e.nl, e.bb);
    return buf;
}

bool parse_entry(const std::string& line, Entry& e) {
    char key[256] = {0};
    const int n = std::sscanf(line.c_str(),
                              " {\"key\": \"%255[^\"]\", \"class\": %d, \"local_kernel\": %d, \"lds_budget_kb\": %d, "
                              "\"plane_variant\": %d, \"nl_matrix_cores\": %d, \"combine_bands\": %d",
                              key, &e.cls, &e.kind, &e.budget, &e.var, &e.nl, &e.bb);
    if (n != 7) return false;
    e.key = key;
    return true;
}

// reads the entries of an existing cache file; missing file = no entries
mb_status read_cache(const char* path, std::vector<Entry>& out, bool* exists) {
    out.clear();
    std::ifstream f(path);
    *exists = (bool)f;
    if (!f) return MB_OK;
    std::string line;
    bool format_ok = false;
    while (std::getline(f, line)) {
        if (line.find("\"format\"") != std::string::npos) {
            format_ok = line.find(kFormat) != std::string::npos;
            continue;
        }
        if (line.find("\"key\"") == std::string::npos) continue;
        Entry e;
        if (!parse_entry(line, e)) return set_error(MB_ERR_INVALID_ARG, "tune cache: malformed entry: " + line);
        out.push_back(e);
    }
    if (!format_ok) return set_error(MB_ERR_INVALID_ARG, std::string("tune cache: not a ") + kFormat + " file");
    return MB_OK;
}

}  // namespace

mb_status apply_tune(Problem* p, int ik, int cls, int kind, int budget_kb, int plane_var, int nl_mfma,
                     int combine_bb) {
    if (ik < 0 || ik >= (int)p->kp.size() || cls < 0 || cls > 1)
        return set_error(MB_ERR_INVALID_ARG, "tune: k-point or precision class out of range");
    KPoint& kp = p->kp[ik];
    if (kind == -1) {
        kp.tune[cls] = KPoint::Tune{};
        if (cls == 1) kp.tune[2] = KPoint::Tune{};
        return MB_OK;
    }
    if (kind < 0 || kind > 3) return set_error(MB_ERR_INVALID_ARG, "tune: local_kernel must be -1..3");
    if (budget_kb < 22 || budget_kb > 160) return set_error(MB_ERR_INVALID_ARG, "tune: lds_budget_kb must be 22..160");
    if (plane_var != 0 && plane_var != 1) return set_error(MB_ERR_INVALID_ARG, "tune: plane_variant must be 0 or 1");
    if (nl_mfma < -1 || nl_mfma > 1) return set_error(MB_ERR_INVALID_ARG, "tune: nl_matrix_cores must be -1..1");
    if (combine_bb != 0 && combine_bb != 1 && combine_bb != 4)
        return set_error(MB_ERR_INVALID_ARG, "tune: combine_bands must be 0, 1 or 4");
    if (kind == 3 && !plane_kernel_grid(p))
        return set_error(MB_ERR_INVALID_ARG, "tune: the plane kernel does not support this grid");
    kp.tune[cls] = KPoint::Tune{1, kind, budget_kb, nl_mfma, plane_var, combine_bb};
    if (cls == 1) kp.tune[2] = kp.tune[1];
    return MB_OK;
}

mb_status tune_save(const Problem* p, const char* path) {
    std::vector<Entry> entries;
    bool exists = false;
    mb_status st = read_cache(path, entries, &exists);
    if (st != MB_OK) return st;
    std::map<std::string, size_t> pos;
    for (size_t i = 0; i < entries.size(); ++i) pos[entries[i].key + "#" + std::to_string(entries[i].cls)] = i;
    const std::string arch = arch_of(p);
    for (const KPoint& kp : p->kp)
        for (int cls = 0; cls < 2; ++cls) {
            const KPoint::Tune& t = kp.tune[cls];
            if (!t.set) continue;
            Entry e;
            e.key = key_of(p, kp, arch);
            e.cls = cls;
            e.kind = t.kind;
            e.budget = t.budget_kb;
            e.var = t.plane_var;
            e.nl = t.nl_mfma;
            e.bb = t.combine_bb;
            const std::string k = e.key + "#" + std::to_string(cls);
            auto it = pos.find(k);
            if (it != pos.end()) {
                entries[it->second] = e;
            } else {
                pos[k] = entries.size();
                entries.push_back(e);
            }
        }
    std::ostringstream o;
    o << "{\n \"format\": \"" << kFormat << "\",\n \"entries\": [\n";
    for (size_t i = 0; i < entries.size(); ++i) o << format_entry(entries[i]) << (i + 1 < entries.size() ? ",\n" : "\n");
    o << " ]\n}\n";
    const std::string tmp = std::string(path) + ".tmp";
    {
        std::ofstream f(tmp, std::ios::trunc);
        if (!f) return set_error(MB_ERR_INVALID_ARG, std::string("tune cache: cannot write ") + tmp);
        f << o.str();
        if (!f) return set_error(MB_ERR_INVALID_ARG, std::string("tune cache: write failed: ") + tmp);
    }
    if (std::rename(tmp.c_str(), path) != 0)
        return set_error(MB_ERR_INVALID_ARG, std::string("tune cache: cannot replace ") + path);
    return MB_OK;
}

mb_status tune_load(Problem* p, const char* path, int* applied) {
    if (applied) *applied = 0;
    std::vector<Entry> entries;
    bool exists = false;
    mb_status st = read_cache(path, entries, &exists);
    if (st != MB_OK || !exists) return st;
    const std::string arch = arch_of(p);
    int n = 0;
    for (int ik = 0; ik < (int)p->kp.size(); ++ik) {
        const std::string key = key_of(p, p->kp[ik], arch);
        for (const Entry& e : entries) {
            if (e.key != key) continue;
            st = apply_tune(p, ik, e.cls, e.kind, e.budget, e.var, e.nl, e.bb);
            if (st != MB_OK) return st;
            ++n;
        }
    }
    if (applied) *applied = n;
    return MB_OK;
}

}  // namespace mb
