// C ABI of the batched ensemble (include/cdbm.h): independent grids with
// their own sizes, gamma, tau, dt, spacings and boundary conditions, sharing
// one velocity set, advanced by one persistent launch per step.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdio>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "../../include/cdbm.h"
#include "api_internal.hpp"
#include "launch.hpp"
#include "step_fused.hpp"

using namespace cdbm;

struct cdbm_batch {
    std::vector<cdbm_params> p;
    std::vector<KParams> k;
    std::vector<int64_t> off;
    int device = 0;
    int precision = CDBM_FP64;
    size_t elem = 8;
    int64_t total_elems = 0;    // extent of the batch buffers (elements)
    KParams* d_k = nullptr;
    int64_t* d_off = nullptr;
    int64_t* d_work = nullptr;
    int* flag = nullptr;
    void* scratch = nullptr;
    int nblocks = 1;
    bool chunked = false;   // every width and offset is a multiple of the 16-byte chunk
    cdbm_batch_launch launch{CDBM_BATCH_CONTIGUOUS, BATCH_FILL, 0, 0};
    // row-piece form: the unit table (four ints per unit), its capacity in
    // units, the counter ranges and the counters themselves
    int* d_units = nullptr;
    int64_t units_cap = 0;
    int64_t* d_range = nullptr;
    int* d_counters = nullptr;
    int nq = 1;
    StepGraph graph;
};

namespace {

void release(cdbm_batch* b) {
    b->graph.release();
    if (b->d_k) (void)hipFree(b->d_k);
    if (b->d_off) (void)hipFree(b->d_off);
    if (b->d_work) (void)hipFree(b->d_work);
    if (b->flag) (void)hipFree(b->flag);
    if (b->scratch) (void)hipFree(b->scratch);
    if (b->d_units) (void)hipFree(b->d_units);
    if (b->d_range) (void)hipFree(b->d_range);
    if (b->d_counters) (void)hipFree(b->d_counters);
    delete b;
}

hipError_t batch_step_once(const void* ctx, const void* fin, void* fout, hipStream_t st) {
    const cdbm_batch* b = (const cdbm_batch*)ctx;
    const int n = (int)b->p.size();
    if (b->launch.layout == CDBM_BATCH_ROW_PIECES)
        return b->precision == CDBM_MIXED
                   ? launch_batch_step_rows<float>(fin, fout, b->d_k, b->d_off, b->d_units,
                                                   b->d_range, b->nq, b->d_counters, b->nblocks,
                                                   b->chunked, st)
                   : launch_batch_step_rows<double>(fin, fout, b->d_k, b->d_off, b->d_units,
                                                    b->d_range, b->nq, b->d_counters, b->nblocks,
                                                    b->chunked, st);
    return b->precision == CDBM_MIXED
               ? launch_batch_step<float>(fin, fout, b->d_k, b->d_off, b->d_work, n,
                                          b->launch.fill_rows, b->nblocks, b->chunked, st)
               : launch_batch_step<double>(fin, fout, b->d_k, b->d_off, b->d_work, n,
                                           b->launch.fill_rows, b->nblocks, b->chunked, st);
}

int check_launch(const cdbm_batch_launch& l) {
    if (l.layout != CDBM_BATCH_CONTIGUOUS && l.layout != CDBM_BATCH_ROW_PIECES)
        return fail(CDBM_EINVAL, "layout must be CDBM_BATCH_CONTIGUOUS or CDBM_BATCH_ROW_PIECES");
    if (l.layout == CDBM_BATCH_CONTIGUOUS && (l.fill_rows < 0 || l.fill_rows > 1024))
        return fail(CDBM_EINVAL, "fill_rows must lie in [0, 1024]");
    if (l.layout == CDBM_BATCH_ROW_PIECES && (l.piece_rows < 16 || l.piece_rows > 65536))
        return fail(CDBM_EINVAL, "piece_rows must lie in [16, 65536]");
    if (l.layout == CDBM_BATCH_ROW_PIECES && l.tail_rows != 0 &&
        (l.tail_rows < 8 || l.tail_rows > 65536))
        return fail(CDBM_EINVAL, "tail_rows must be 0 or lie in [8, 65536]");
    if (l.layout == CDBM_BATCH_CONTIGUOUS && l.tail_rows != 0)
        return fail(CDBM_EINVAL, "tail_rows must be 0 in the contiguous layout");
    return CDBM_OK;
}

// Upload the tables of a launch configuration (synchronous).  Contiguous
// form: the prefix sums of strips * (ny + fill).  Row-piece form: each grid
// cut into pieces of about piece_rows rows; the units (grid, piece, strip)
// split into nq ranges of about equal weight (rows + BATCH_FILL per unit),
// nq = min(8, blocks): one counter per XCD.
int apply_launch(cdbm_batch* b, const cdbm_batch_launch& l) {
    int rc = check_launch(l);
    if (rc != CDBM_OK) return rc;
    // the captured graphs hold the old kernel and its arguments
    b->graph.release();
    const int n = (int)b->p.size();
    const int tx = strip_width(b->precision);
    hipError_t e;
    if (l.layout == CDBM_BATCH_CONTIGUOUS) {
        std::vector<int64_t> work(n + 1, 0);
        for (int g = 0; g < n; ++g) {
            const int64_t strips = (b->p[g].nx + tx - 1) / tx;
            work[g + 1] = work[g] + strips * (b->p[g].ny + l.fill_rows);
        }
        e = hipMemcpy(b->d_work, work.data(), sizeof(int64_t) * (n + 1), hipMemcpyHostToDevice);
        if (e != hipSuccess) return hip_fail(e, "hipMemcpy of the batch work table");
    } else {
        // units (grid, strip column, first row, end row): each grid's rows
        // above its tail cut into pieces of about piece_rows rows, strip by
        // strip within a piece; the tail (the last tail_rows rows of a grid
        // taller than twice that) as one unit per strip, placed after the
        // pieces of the range that holds the grid's last piece, so that every
        // range ends with small units
        struct Unit {
            int g, x0, ya, yb;
        };
        std::vector<Unit> body;
        std::vector<int64_t> last(n, -1);   // index in body of each grid's last unit
        std::vector<std::vector<Unit>> tails(n);
        double total = 0.0;
        for (int g = 0; g < n; ++g) {
            const int ny = b->p[g].ny;
            const int strips = (b->p[g].nx + tx - 1) / tx;
            const int tail = (l.tail_rows > 0 && ny > 2 * l.tail_rows) ? l.tail_rows : 0;
            const int nb = ny - tail;
            int pieces = std::max(1, (nb + l.piece_rows / 2) / l.piece_rows);
            const int rows = (nb + pieces - 1) / pieces;
            pieces = (nb + rows - 1) / rows;
            for (int p = 0; p < pieces; ++p) {
                const int ya = p * rows, yb = std::min(nb, ya + rows);
                for (int s = 0; s < strips; ++s) body.push_back(Unit{g, s * tx, ya, yb});
                total += (double)strips * (yb - ya + BATCH_FILL);
            }
            last[g] = (int64_t)body.size() - 1;
            for (int s = 0; tail > 0 && s < strips; ++s) tails[g].push_back(Unit{g, s * tx, nb, ny});
            total += (double)tails[g].size() * (tail + BATCH_FILL);
        }
        if ((int64_t)body.size() >= (int64_t(1) << 30)) return fail(CDBM_EINVAL, "too many work units");
        const int nq = std::max(1, std::min(8, b->nblocks));
        // cut the pieces into nq ranges of about equal weight, a grid's tail
        // counted with its last piece; then each range's pieces followed by
        // the tails of the grids whose last piece it holds
        std::vector<Unit> table;
        table.reserve(body.size() + 64);
        std::vector<int64_t> range(nq + 1, 0);
        double acc = 0.0;
        int k = 0;
        std::vector<int> ended;   // grids whose last piece the current range holds
        auto close_range = [&]() {
            for (int g : ended) table.insert(table.end(), tails[g].begin(), tails[g].end());
            ended.clear();
            range[++k] = (int64_t)table.size();
        };
        for (int64_t u = 0; u < (int64_t)body.size(); ++u) {
            const Unit& t = body[u];
            table.push_back(t);
            acc += t.yb - t.ya + BATCH_FILL;
            if (last[t.g] == u) {
                ended.push_back(t.g);
                acc += (double)tails[t.g].size() * (l.tail_rows + BATCH_FILL);
            }
            if (k < nq - 1 && acc >= total * (k + 1) / nq) close_range();
        }
        while (k < nq) close_range();
        const int64_t nunits = (int64_t)table.size();
        if (!b->d_range &&
            (hipMalloc(&b->d_range, sizeof(int64_t) * 9) != hipSuccess ||
             hipMalloc(&b->d_counters, sizeof(int) * 9) != hipSuccess))
            return fail(CDBM_ENOMEM, "device allocation of the row-piece tables failed");
        if (nunits > b->units_cap) {
            if (b->d_units) (void)hipFree(b->d_units);
            b->d_units = nullptr;
            b->units_cap = 0;
            if (hipMalloc(&b->d_units, sizeof(int) * 4 * nunits) != hipSuccess)
                return fail(CDBM_ENOMEM, "device allocation of the unit table failed");
            b->units_cap = nunits;
        }
        std::vector<int> flat(4 * nunits);
        for (int64_t u = 0; u < nunits; ++u) {
            flat[4 * u] = table[u].g;
            flat[4 * u + 1] = table[u].x0;
            flat[4 * u + 2] = table[u].ya;
            flat[4 * u + 3] = table[u].yb;
        }
        if ((e = hipMemcpy(b->d_units, flat.data(), sizeof(int) * 4 * nunits,
                           hipMemcpyHostToDevice)) != hipSuccess ||
            (e = hipMemcpy(b->d_range, range.data(), sizeof(int64_t) * (nq + 1),
                           hipMemcpyHostToDevice)) != hipSuccess ||
            (e = hipMemset(b->d_counters, 0, sizeof(int) * 9)) != hipSuccess ||
            (e = hipDeviceSynchronize()) != hipSuccess)
            return hip_fail(e, "upload of the row-piece tables");
        b->nq = nq;
    }
    b->launch = l;
    return CDBM_OK;
}

// --- autotuning ----------------------------------------------------------
//
// The cache is a JSON object with one entry per line, keyed by
// "<gfx arch>|<precision>|cells2^<k>|grids2^<m>" (k, m: floor of log2 of the
// batch's cell and grid counts), each value the chosen launch and its time:
//   "gfx950|mixed|cells2^25|grids2^6": {"layout": 1, "fill_rows": 0, "piece_rows": 192, "tail_rows": 64, "ms_per_step": 1.512},
// (an entry without tail_rows reads as tail_rows 0).

struct TuneEntry {
    cdbm_batch_launch l;
    double ms;
};

int floor_log2(int64_t v) {
    int k = 0;
    while (v > 1) {
        v >>= 1;
        ++k;
    }
    return k;
}

std::string tune_key(const cdbm_batch* b) {
    hipDeviceProp_t prop;
    std::string arch = "unknown";
    if (hipGetDeviceProperties(&prop, b->device) == hipSuccess) {
        arch = prop.gcnArchName;
        const size_t c = arch.find(':');
        if (c != std::string::npos) arch = arch.substr(0, c);
    }
    int64_t cells = 0;
    for (const cdbm_params& q : b->p) cells += (int64_t)q.nx * q.ny;
    char buf[160];
    std::snprintf(buf, sizeof buf, "%s|%s|cells2^%d|grids2^%d", arch.c_str(),
                  b->precision == CDBM_MIXED ? "mixed" : "fp64", floor_log2(cells),
                  floor_log2((int64_t)b->p.size()));
    return buf;
}

std::vector<std::pair<std::string, TuneEntry>> read_cache(const char* path) {
    std::vector<std::pair<std::string, TuneEntry>> out;
    FILE* fh = path ? std::fopen(path, "r") : nullptr;
    if (!fh) return out;
    char line[512];
    while (std::fgets(line, sizeof line, fh)) {
        const char* q0 = std::strchr(line, '"');
        const char* q1 = q0 ? std::strchr(q0 + 1, '"') : nullptr;
        const char* brace = q1 ? std::strchr(q1, '{') : nullptr;
        if (!brace) continue;
        TuneEntry e{};
        if (std::sscanf(brace, "{\"layout\": %d, \"fill_rows\": %d, \"piece_rows\": %d, "
                               "\"tail_rows\": %d, \"ms_per_step\": %lf",
                        &e.l.layout, &e.l.fill_rows, &e.l.piece_rows, &e.l.tail_rows, &e.ms) != 5) {
            e = TuneEntry{};
            if (std::sscanf(brace, "{\"layout\": %d, \"fill_rows\": %d, \"piece_rows\": %d, "
                                   "\"ms_per_step\": %lf",
                            &e.l.layout, &e.l.fill_rows, &e.l.piece_rows, &e.ms) != 4)
                continue;
        }
        out.emplace_back(std::string(q0 + 1, q1), e);
    }
    std::fclose(fh);
    return out;
}

void write_cache(const char* path, const std::vector<std::pair<std::string, TuneEntry>>& ents) {
    const std::string tmp = std::string(path) + ".tmp";
    FILE* fh = std::fopen(tmp.c_str(), "w");
    if (!fh) return;   // an unwritable cache only costs a re-tune next time
    std::fprintf(fh, "{\n");
    for (size_t k = 0; k < ents.size(); ++k) {
        const TuneEntry& e = ents[k].second;
        std::fprintf(fh,
                     "\"%s\": {\"layout\": %d, \"fill_rows\": %d, \"piece_rows\": %d, "
                     "\"tail_rows\": %d, \"ms_per_step\": %.6f}%s\n",
                     ents[k].first.c_str(), e.l.layout, e.l.fill_rows, e.l.piece_rows,
                     e.l.tail_rows, e.ms, k + 1 < ents.size() ? "," : "");
    }
    std::fprintf(fh, "}\n");
    std::fclose(fh);
    std::rename(tmp.c_str(), path);
}

// Milliseconds per step of the current launch: the fastest of three runs of
// TUNE_STEPS single launches (f_in -> f_out, then ping-pong with the batch's
// scratch), after two untimed steps.
constexpr int TUNE_STEPS = 8;

int time_launch(cdbm_batch* b, const void* f_in, void* f_out, hipStream_t st, double* ms) {
    hipEvent_t e0 = nullptr, e1 = nullptr;
    hipError_t e = hipEventCreate(&e0);
    if (e == hipSuccess) e = hipEventCreate(&e1);
    int rc = CDBM_OK;
    double best = -1.0;
    if (e != hipSuccess) rc = hip_fail(e, "hipEventCreate");
    for (int rep = 0; rc == CDBM_OK && rep < 4; ++rep) {
        // rep 0 is the warm-up
        if (rep > 0 && (e = hipEventRecord(e0, st)) != hipSuccess) {
            rc = hip_fail(e, "hipEventRecord");
            break;
        }
        const int n = rep == 0 ? 2 : TUNE_STEPS;
        e = batch_step_once(b, f_in, f_out, st);
        for (int k = 1; e == hipSuccess && k < n; ++k)
            e = (k % 2) ? batch_step_once(b, f_out, b->scratch, st)
                        : batch_step_once(b, b->scratch, f_out, st);
        if (e != hipSuccess) {
            rc = hip_fail(e, "batch step launch");
            break;
        }
        if (rep == 0) continue;
        float t = 0.0f;
        if ((e = hipEventRecord(e1, st)) != hipSuccess || (e = hipEventSynchronize(e1)) != hipSuccess ||
            (e = hipEventElapsedTime(&t, e0, e1)) != hipSuccess) {
            rc = hip_fail(e, "timing the batch step");
            break;
        }
        const double per = (double)t / n;
        if (best < 0.0 || per < best) best = per;
    }
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    *ms = best;
    return rc;
}

int autotune(cdbm_batch* b, const void* f_in, void* f_out, const char* cache_path,
             cdbm_batch_launch* chosen, hipStream_t st) {
    const std::string key = tune_key(b);
    auto ents = read_cache(cache_path);
    for (const auto& kv : ents)
        if (kv.first == key && check_launch(kv.second.l) == CDBM_OK) {
            int rc = apply_launch(b, kv.second.l);
            if (rc == CDBM_OK && chosen) *chosen = b->launch;
            return rc;
        }
    // candidates: the contiguous split with three fill weights (the default
    // first), the row-piece form with three piece heights, and three
    // row-piece forms with tails
    // (on the 96-grid ensemble of 128^2 .. 1024^2 grids, mixed: 1.75-1.80 ms
    // contiguous, 1.52-1.55 plain pieces of 128 or 192 rows, 1.44-1.46 with
    // tails over the range of pieces below, within timing noise of each other)
    const cdbm_batch_launch cands[] = {
        {CDBM_BATCH_CONTIGUOUS, BATCH_FILL, 0, 0}, {CDBM_BATCH_CONTIGUOUS, 0, 0, 0},
        {CDBM_BATCH_CONTIGUOUS, 2 * BATCH_FILL, 0, 0}, {CDBM_BATCH_ROW_PIECES, 0, 128, 0},
        {CDBM_BATCH_ROW_PIECES, 0, 192, 0},           {CDBM_BATCH_ROW_PIECES, 0, 160, 64},
        {CDBM_BATCH_ROW_PIECES, 0, 192, 64},          {CDBM_BATCH_ROW_PIECES, 0, 320, 96},
        {CDBM_BATCH_ROW_PIECES, 0, 320, 128},         {CDBM_BATCH_ROW_PIECES, 0, 384, 160},
        {CDBM_BATCH_ROW_PIECES, 0, 448, 160},
    };
    TuneEntry best{cands[0], -1.0};
    for (const cdbm_batch_launch& c : cands) {
        int rc = apply_launch(b, c);
        double ms = 0.0;
        if (rc == CDBM_OK) rc = time_launch(b, f_in, f_out, st, &ms);
        if (rc != CDBM_OK) return rc;
        if (best.ms < 0.0 || ms < best.ms) best = TuneEntry{c, ms};
    }
    int rc = apply_launch(b, best.l);
    if (rc != CDBM_OK) return rc;
    if (cache_path) {
        ents.emplace_back(key, best);
        write_cache(cache_path, ents);
    }
    if (chosen) *chosen = b->launch;
    return CDBM_OK;
}

int check_batch_device(const cdbm_batch* b) {
    int dev = -1;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
    if (dev != b->device) return fail(CDBM_EINVAL, "batch was created on another device");
    return CDBM_OK;
}

}  // namespace

extern "C" {

int cdbm_batch_create(const cdbm_params* per_grid, int32_t ngrids, const int64_t* f_offsets,
                      cdbm_batch** out) {
    if (!per_grid || !f_offsets || !out) return fail(CDBM_EINVAL, "null argument");
    *out = nullptr;
    if (ngrids < 1 || ngrids > (1 << 20)) return fail(CDBM_EINVAL, "ngrids out of range");
    auto* b = new (std::nothrow) cdbm_batch();
    if (!b) return fail(CDBM_ENOMEM, "host allocation failed");
    b->p.assign(per_grid, per_grid + ngrids);
    b->k.resize(ngrids);
    b->off.assign(f_offsets, f_offsets + ngrids);
    b->precision = per_grid[0].precision;
    if (b->precision == CDBM_MIXED_COMP) {
        delete b;
        return fail(CDBM_EINVAL, "the batched form does not take CDBM_MIXED_COMP");
    }
    char buf[160];
    for (int g = 0; g < ngrids; ++g) {
        const cdbm_params& q = per_grid[g];
        std::string err;
        int rc = build_params(q, b->k[g], err);
        if (rc != CDBM_OK) {
            std::snprintf(buf, sizeof buf, "grid %d: ", g);
            delete b;
            return fail(rc, buf + err);
        }
        if (std::memcmp(q.v, per_grid[0].v, sizeof q.v) != 0 ||
            std::memcmp(q.eta, per_grid[0].eta, sizeof q.eta) != 0 ||
            q.precision != per_grid[0].precision) {
            std::snprintf(buf, sizeof buf,
                          "grid %d: v, eta and precision must be the same for every grid", g);
            delete b;
            return fail(CDBM_EINVAL, buf);
        }
        if (f_offsets[g] < 0) {
            delete b;
            return fail(CDBM_EINVAL, "negative f offset");
        }
    }
    // the grids' blocks must not overlap
    std::vector<int> order(ngrids);
    for (int g = 0; g < ngrids; ++g) order[g] = g;
    std::sort(order.begin(), order.end(), [&](int x, int y) { return f_offsets[x] < f_offsets[y]; });
    int64_t end = 0;
    for (int idx = 0; idx < ngrids; ++idx) {
        const int g = order[idx];
        const int64_t sz = (int64_t)NV * per_grid[g].nx * per_grid[g].ny;
        if (f_offsets[g] < end) {
            delete b;
            return fail(CDBM_EINVAL, "f blocks of the grids overlap");
        }
        end = f_offsets[g] + sz;
    }
    b->total_elems = end;
    b->elem = b->precision == CDBM_MIXED ? sizeof(float) : sizeof(double);

    int64_t strip_rows = 0;
    for (int g = 0; g < ngrids; ++g) {
        const int tx = strip_width(b->precision);
        const int64_t strips = (per_grid[g].nx + tx - 1) / tx;
        strip_rows += strips * per_grid[g].ny;
    }
    hipError_t e = hipGetDevice(&b->device);
    if (e != hipSuccess) {
        delete b;
        return hip_fail(e, "hipGetDevice");
    }
    if (hipMalloc(&b->d_k, sizeof(KParams) * ngrids) != hipSuccess ||
        hipMalloc(&b->d_off, sizeof(int64_t) * ngrids) != hipSuccess ||
        hipMalloc(&b->d_work, sizeof(int64_t) * (ngrids + 1)) != hipSuccess ||
        hipMalloc(&b->flag, sizeof(int)) != hipSuccess ||
        hipMalloc(&b->scratch, (size_t)b->total_elems * b->elem) != hipSuccess) {
        release(b);
        return fail(CDBM_ENOMEM, "device allocation failed");
    }
    if ((e = hipMemcpy(b->d_k, b->k.data(), sizeof(KParams) * ngrids, hipMemcpyHostToDevice)) !=
            hipSuccess ||
        (e = hipMemcpy(b->d_off, f_offsets, sizeof(int64_t) * ngrids, hipMemcpyHostToDevice)) !=
            hipSuccess) {
        release(b);
        return hip_fail(e, "hipMemcpy of the batch tables");
    }
    const int64_t cap = (strip_rows + 31) / 32;
    int64_t nb = b->precision == CDBM_MIXED ? batch_blocks<float>() : batch_blocks<double>();
    b->nblocks = (int)std::max<int64_t>(1, std::min(nb, cap));
    int rc = apply_launch(b, b->launch);
    if (rc != CDBM_OK) {
        release(b);
        return rc;
    }
    // the chunked form of the step (16-byte chunks, 32-bit offsets within a grid)
    const int cw = b->precision == CDBM_MIXED ? 4 : 2;
    const uint64_t esz = b->precision == CDBM_MIXED ? 4 : 8;
    b->chunked = true;
    for (int g = 0; g < ngrids; ++g)
        b->chunked = b->chunked && per_grid[g].nx % cw == 0 && f_offsets[g] % cw == 0 &&
                     (uint64_t)NV * per_grid[g].nx * per_grid[g].ny * esz <= (uint64_t(1) << 32);
    *out = b;
    return CDBM_OK;
}

int cdbm_batch_destroy(cdbm_batch* b) {
    if (!b) return CDBM_OK;
    (void)hipDeviceSynchronize();
    release(b);
    return CDBM_OK;
}

int cdbm_batch_init(cdbm_batch* b, const double* rho, const double* ux, const double* uy,
                    const double* T, void* f_out, void* stream) {
    if (!b || !rho || !ux || !uy || !T || !f_out) return fail(CDBM_EINVAL, "null argument");
    int rc = check_batch_device(b);
    if (rc != CDBM_OK) return rc;
    hipStream_t st = (hipStream_t)stream;
    for (size_t g = 0; g < b->p.size(); ++g) {
        if (b->off[g] % NV != 0)
            return fail(CDBM_EINVAL, "cdbm_batch_init needs f offsets that are multiples of 16");
        const int64_t c0 = b->off[g] / NV;
        const int64_t cells = (int64_t)b->p[g].nx * b->p[g].ny;
        rc = check_fields_range(b->flag, rho + c0, ux + c0, uy + c0, T + c0, cells, st);
        if (rc != CDBM_OK) return rc;
    }
    for (size_t g = 0; g < b->p.size(); ++g) {
        const int64_t c0 = b->off[g] / NV;
        char* dst = (char*)f_out + (size_t)b->off[g] * b->elem;
        hipError_t e =
            b->precision == CDBM_MIXED
                ? launch_init<float>(rho + c0, ux + c0, uy + c0, T + c0, dst, b->k[g], st)
                : launch_init<double>(rho + c0, ux + c0, uy + c0, T + c0, dst, b->k[g], st);
        if (e != hipSuccess) return hip_fail(e, "init launch");
    }
    return CDBM_OK;
}

int cdbm_batch_step(cdbm_batch* b, const void* f_in, void* f_out, int32_t nsteps, void* stream) {
    if (!b || !f_in || !f_out) return fail(CDBM_EINVAL, "null argument");
    if (nsteps < 0) return fail(CDBM_EINVAL, "nsteps must be >= 0");
    const size_t bytes = (size_t)b->total_elems * b->elem;
    const char* x = (const char*)f_in;
    const char* y = (const char*)f_out;
    if (x < y + bytes && y < x + bytes) return fail(CDBM_EINVAL, "f_in and f_out overlap");
    int rc = check_batch_device(b);
    if (rc != CDBM_OK) return rc;
    hipStream_t st = (hipStream_t)stream;
    if (nsteps == 0) {
        hipError_t e = hipMemcpyAsync(f_out, f_in, bytes, hipMemcpyDeviceToDevice, st);
        return e == hipSuccess ? CDBM_OK : hip_fail(e, "hipMemcpyAsync");
    }
    return run_steps(batch_step_once, b, f_in, f_out, b->scratch, nsteps, st, b->graph);
}

int cdbm_batch_get_launch(const cdbm_batch* b, cdbm_batch_launch* out) {
    if (!b || !out) return fail(CDBM_EINVAL, "null argument");
    *out = b->launch;
    return CDBM_OK;
}

int cdbm_batch_set_launch(cdbm_batch* b, const cdbm_batch_launch* l) {
    if (!b || !l) return fail(CDBM_EINVAL, "null argument");
    int rc = check_batch_device(b);
    if (rc != CDBM_OK) return rc;
    return apply_launch(b, *l);
}

int cdbm_batch_autotune(cdbm_batch* b, const void* f_in, void* f_out, const char* cache_path,
                        cdbm_batch_launch* chosen, void* stream) {
    if (!b || !f_in || !f_out) return fail(CDBM_EINVAL, "null argument");
    int rc = check_batch_device(b);
    if (rc != CDBM_OK) return rc;
    return autotune(b, f_in, f_out, cache_path, chosen, (hipStream_t)stream);
}

}  // extern "C"
