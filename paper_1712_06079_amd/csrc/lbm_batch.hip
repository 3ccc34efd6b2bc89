// Batched sweep: many independent periodic domains of uneven size, EOS and
// temperature (the coexistence-curve sweep of Sec. 5.2) advanced by one
// launch per step of a worklist kernel (k_batch), replayed from a hipGraph.
// A scheduler setting (tile height, worklist order, persistent grid size) is
// chosen by lbm_batch_autotune from timed candidates.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdio>
#include <cstring>
#include <map>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "../../include/lbm.h"
#include "lbm_fused.hpp"
#include "lbm_internal.hpp"

using namespace lbm_internal;

struct lbm_batch {
    int n;
    int prec, force, grad9;
    std::vector<lbm_domain*> doms;
    std::vector<size_t> dom_off, dom_bytes;
    char* ws;
    size_t ws_bytes;
    size_t off_desc[2], off_tiles, off_flags, off_snap, desc_bytes, tiles_cap;
    int cur;            // buffer parity shared by all domains
    int64_t steps;
    int tile_y, order, grid, ry;
    int ntiles;
    hipStream_t cap;
    hipGraphExec_t exec;
    bool graph_ok;
    int graph_steps;
};

namespace {

// Fill n ints with v (clears the per-domain flags on the stream, also where a
// memset node would not be wanted).
__global__ void k_fill_int(int* __restrict__ p, int n, int v) {
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) p[i] = v;
}

constexpr int GRAPH_STEPS = 16;  // launches per captured graph (even: parity is restored)

size_t desc_size(int prec) { return prec == LBM_F32 ? sizeof(lbm::StepArgs<float>) : sizeof(lbm::StepArgs<double>); }

// Worklist of (domain, x0, y0) tiles in the requested order.  Worklist
// position p is taken by workgroup p mod G of a grid of G workgroups, and
// workgroup w runs on XCD w mod 8: order 3 places each domain's tiles at
// positions of one XCD (domains largest first, each to the XCD with the most
// free positions; what does not fit fills the remaining positions), so the
// potential halos that neighbouring tiles share are read into one L2.
std::vector<lbm::BatchTile> make_tiles(const lbm_batch* b, int ty, int order, int grid) {
    std::vector<std::vector<lbm::BatchTile>> per(b->n);
    for (int d = 0; d < b->n; ++d) {
        const lbm_params& p = b->doms[d]->p;
        for (int y0 = 0; y0 < p.ny; y0 += ty)
            for (int x0 = 0; x0 < p.nx; x0 += lbm::BX) per[d].push_back(lbm::BatchTile{d, x0, y0, 0});
    }
    std::vector<int> idx(b->n);
    for (int d = 0; d < b->n; ++d) idx[d] = d;
    if (order == 1 || order == 3)  // largest domains first (longest-processing-time order)
        std::stable_sort(idx.begin(), idx.end(), [&](int a, int c) { return per[a].size() > per[c].size(); });
    std::vector<lbm::BatchTile> out;
    if (order == 3) {
        size_t total = 0;
        for (const auto& v : per) total += v.size();
        const size_t G = grid > 0 ? std::min<size_t>((size_t)grid, total) : total;
        std::vector<std::vector<size_t>> pos(lbm::NXCD);
        for (size_t p = 0; p < total; ++p) pos[(p % G) % lbm::NXCD].push_back(p);
        out.assign(total, lbm::BatchTile{0, 0, 0, 0});
        std::vector<char> used(total, 0);
        std::vector<size_t> fill(lbm::NXCD, 0);
        std::vector<lbm::BatchTile> spill;
        for (int d : idx) {
            int x = 0;
            for (int k = 1; k < lbm::NXCD; ++k)
                if (pos[k].size() - fill[k] > pos[x].size() - fill[x]) x = k;
            for (const auto& t : per[d]) {
                if (fill[x] < pos[x].size()) {
                    const size_t p = pos[x][fill[x]++];
                    out[p] = t;
                    used[p] = 1;
                } else {
                    spill.push_back(t);
                }
            }
        }
        size_t k = 0;
        for (size_t p = 0; p < total; ++p)
            if (!used[p]) out[p] = spill[k++];
    } else if (order == 2) {  // round robin: one tile of each domain in turn
        size_t k = 0;
        bool any = true;
        while (any) {
            any = false;
            for (int d = 0; d < b->n; ++d)
                if (k < per[d].size()) { out.push_back(per[d][k]); any = true; }
            ++k;
        }
    } else {
        for (int d : idx) out.insert(out.end(), per[d].begin(), per[d].end());
    }
    return out;
}

int max_tiles(const lbm_params* params, int n) {
    long t = 0;
    for (int i = 0; i < n; ++i)
        t += (long)((params[i].nx + lbm::BX - 1) / lbm::BX) * ((params[i].ny + 3) / 4);
    return (int)t;
}

template <typename Real, int FORCE, int TY, int RY>
void launch_batch_t(const lbm_batch* b, int parity, hipStream_t s) {
    const auto* descs = reinterpret_cast<const lbm::StepArgs<Real>*>(b->ws + b->off_desc[parity]);
    const auto* tiles = reinterpret_cast<const lbm::BatchTile*>(b->ws + b->off_tiles);
    const int grid = b->grid > 0 ? std::min(b->grid, b->ntiles) : b->ntiles;
    if (b->grad9)
        hipLaunchKernelGGL((lbm::k_batch<Real, FORCE, TY, 16, true>), dim3(grid), dim3(lbm::NT), 0, s, descs, tiles,
                           b->ntiles);
    else
        hipLaunchKernelGGL((lbm::k_batch<Real, FORCE, TY, RY>), dim3(grid), dim3(lbm::NT), 0, s, descs, tiles,
                           b->ntiles);
}

template <typename Real, int FORCE>
void launch_batch_f(const lbm_batch* b, int parity, hipStream_t s) {
    constexpr int R = lbm::Radius<Real>::value;
    const bool small = b->ry <= 16;
    if (b->tile_y == 4) {
        if (small) launch_batch_t<Real, FORCE, 4, 16>(b, parity, s);
        else launch_batch_t<Real, FORCE, 4, R>(b, parity, s);
    } else {
        if (small) launch_batch_t<Real, FORCE, 8, 16>(b, parity, s);
        else launch_batch_t<Real, FORCE, 8, R>(b, parity, s);
    }
}

void launch_batch(const lbm_batch* b, int parity, hipStream_t s) {
    const bool f32 = b->prec == LBM_F32;
    switch (b->force) {
        case LBM_FORCE_SC:
            if (f32) launch_batch_f<float, lbm::FORCE_SC>(b, parity, s); else launch_batch_f<double, lbm::FORCE_SC>(b, parity, s);
            break;
        case LBM_FORCE_ZC:
            if (f32) launch_batch_f<float, lbm::FORCE_ZC>(b, parity, s); else launch_batch_f<double, lbm::FORCE_ZC>(b, parity, s);
            break;
        default:
            if (f32) launch_batch_f<float, lbm::FORCE_HYBRID>(b, parity, s); else launch_batch_f<double, lbm::FORCE_HYBRID>(b, parity, s);
    }
}

void set_parity(lbm_batch* b, int cur) {
    b->cur = cur;
    for (auto* d : b->doms) d->cur = cur;
}

// Replace the worklist (copied on stream s, which is then synchronised, so
// launches queued on s before the call have read the old list) and drop the
// captured graph.
lbm_status upload_tiles(lbm_batch* b, hipStream_t s) {
    std::vector<lbm::BatchTile> t = make_tiles(b, b->tile_y, b->order, b->grid);
    if (t.size() > b->tiles_cap) return fail(LBM_EINVAL, "tile list exceeds its workspace area");
    b->ntiles = (int)t.size();
    HIP_TRY(hipMemcpyAsync(b->ws + b->off_tiles, t.data(), t.size() * sizeof(lbm::BatchTile), hipMemcpyHostToDevice, s));
    HIP_TRY(hipStreamSynchronize(s));
    if (b->graph_ok) {
        (void)hipGraphExecDestroy(b->exec);
        b->graph_ok = false;
    }
    return LBM_OK;
}

lbm_status ensure_graph(lbm_batch* b) {
    if (b->graph_ok) return LBM_OK;
    hipGraph_t g;
    HIP_TRY(hipStreamBeginCapture(b->cap, hipStreamCaptureModeThreadLocal));
    for (int s = 0; s < b->graph_steps; ++s) launch_batch(b, s & 1, b->cap);
    hipError_t e = hipStreamEndCapture(b->cap, &g);
    if (e != hipSuccess) return fail(LBM_EDEVICE, "graph capture: %s", hipGetErrorString(e));
    e = hipGraphInstantiate(&b->exec, g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    if (e != hipSuccess) return fail(LBM_EDEVICE, "graph instantiate: %s", hipGetErrorString(e));
    b->graph_ok = true;
    return LBM_OK;
}

// Autotuner results of this process, keyed by what the timing depends on:
// the device's architecture, the batch's precision, force and use of Eq. 15,
// and its domains in order: shape, gradient, walls (the tile list and the
// per-tile work are built from them).
struct TuneChoice {
    int tile_y, order, grid;
};
std::mutex tune_mutex;
std::map<std::string, TuneChoice> tune_cache;

lbm_status tune_key(const lbm_batch* b, std::string* key) {
    int dev = 0;
    HIP_TRY(hipGetDevice(&dev));
    hipDeviceProp_t prop;
    HIP_TRY(hipGetDeviceProperties(&prop, dev));
    char buf[96];
    snprintf(buf, sizeof(buf), "%s|p%d|f%d|g%d|n%d|", prop.gcnArchName, b->prec, b->force, b->grad9, b->n);
    *key = buf;
    for (const auto* d : b->doms) {
        snprintf(buf, sizeof(buf), "%dx%dg%d%s,", d->p.nx, d->p.ny, d->p.grad, d->p.walls ? "w" : "");
        *key += buf;
    }
    return LBM_OK;
}

struct BatchLayout {
    std::vector<size_t> off, bytes;
    size_t desc, tiles, flags, snap, total;
};

lbm_status batch_layout(const lbm_params* params, int n, BatchLayout* L) {
    size_t pos = 0, snap = 0;
    L->off.resize(n);
    L->bytes.resize(n);
    for (int i = 0; i < n; ++i) {
        size_t nb = 0;
        lbm_status st = lbm_workspace_bytes(&params[i], &nb);
        if (st != LBM_OK) return st;
        L->off[i] = pos;
        L->bytes[i] = nb;
        pos += align256(nb);
        const size_t es = params[i].prec == LBM_F32 ? 4 : 8;
        snap += align256((size_t)lbm::Q * ((params[i].nx + lbm::BX - 1) / lbm::BX) * lbm::BX * params[i].ny * es);
    }
    L->desc = align256((size_t)n * desc_size(params[0].prec));
    L->tiles = align256((size_t)max_tiles(params, n) * sizeof(lbm::BatchTile));
    L->flags = align256((size_t)n * sizeof(int));
    L->snap = snap;
    L->total = pos + 2 * L->desc + L->tiles + L->flags + L->snap;
    return LBM_OK;
}

}  // namespace

extern "C" {

lbm_status lbm_batch_workspace_bytes(const lbm_params* params, int32_t n, size_t* bytes) {
    if (!params || !bytes || n < 1) return fail(LBM_EINVAL, "invalid batch arguments");
    BatchLayout L;
    lbm_status st = batch_layout(params, n, &L);
    if (st != LBM_OK) return st;
    *bytes = L.total;
    return LBM_OK;
}

lbm_status lbm_batch_create(const lbm_params* params, int32_t n, void* workspace, size_t workspace_bytes,
                            const double* const* rho0s, hipStream_t stream, lbm_batch** out) {
    if (!params || !workspace || !rho0s || !out || n < 1) return fail(LBM_EINVAL, "invalid batch arguments");
    if (((uintptr_t)workspace & 255) != 0) return fail(LBM_EINVAL, "workspace must be 256-byte aligned");
    for (int i = 1; i < n; ++i)
        if (params[i].prec != params[0].prec || params[i].force != params[0].force ||
            (params[i].grad == LBM_GRAD_CDM9) != (params[0].grad == LBM_GRAD_CDM9))
            return fail(LBM_EINVAL, "all domains of a batch share precision, force and (Eq. 15 or not) gradient");
    BatchLayout L;
    lbm_status st = batch_layout(params, n, &L);
    if (st != LBM_OK) return st;
    if (workspace_bytes < L.total) return fail(LBM_ENOMEM, "batch workspace %zu < %zu bytes", workspace_bytes, L.total);
    lbm_batch* b = new (std::nothrow) lbm_batch();
    if (!b) return fail(LBM_ENOMEM, "out of host memory");
    b->n = n;
    b->prec = params[0].prec;
    b->force = params[0].force;
    b->grad9 = params[0].grad == LBM_GRAD_CDM9 ? 1 : 0;
    b->ws = static_cast<char*>(workspace);
    b->ws_bytes = workspace_bytes;
    size_t pos = L.off.empty() ? 0 : L.off[n - 1] + align256(L.bytes[n - 1]);
    b->desc_bytes = L.desc;
    b->off_desc[0] = pos;
    b->off_desc[1] = pos + L.desc;
    b->off_tiles = pos + 2 * L.desc;
    b->tiles_cap = L.tiles / sizeof(lbm::BatchTile);
    b->off_flags = b->off_tiles + L.tiles;
    b->off_snap = b->off_flags + L.flags;
    b->cur = 0;
    b->steps = 0;
    b->tile_y = 8;
    b->order = 1;
    b->grid = 0;
    b->graph_ok = false;
    b->graph_steps = GRAPH_STEPS;
    b->dom_off = L.off;
    b->dom_bytes = L.bytes;
    int ry = 0;
    for (int i = 0; i < n; ++i) {
        lbm_domain* d = nullptr;
        st = lbm_init(&params[i], b->ws + L.off[i], L.bytes[i], rho0s[i], nullptr, nullptr, stream, &d);
        if (st != LBM_OK) {
            for (auto* q : b->doms) lbm_destroy(q);
            delete b;
            return st;
        }
        b->doms.push_back(d);
        ry = std::max(ry, d->ty);
    }
    b->ry = ry;
    // descriptors for both buffer parities
    std::vector<char> host(L.desc);
    for (int par = 0; par < 2; ++par) {
        for (int i = 0; i < n; ++i) {
            if (b->prec == LBM_F32) {
                auto a = make_args<float>(b->doms[i], par, 1 - par);
                std::memcpy(host.data() + i * sizeof(a), &a, sizeof(a));
            } else {
                auto a = make_args<double>(b->doms[i], par, 1 - par);
                std::memcpy(host.data() + i * sizeof(a), &a, sizeof(a));
            }
        }
        hipError_t e = hipMemcpyAsync(b->ws + b->off_desc[par], host.data(), n * desc_size(b->prec),
                                      hipMemcpyHostToDevice, stream);
        if (e == hipSuccess) e = hipStreamSynchronize(stream);
        if (e != hipSuccess) {
            lbm_batch_destroy(b);
            return fail(LBM_EDEVICE, "descriptor upload: %s", hipGetErrorString(e));
        }
    }
    if (hipStreamCreateWithFlags(&b->cap, hipStreamNonBlocking) != hipSuccess) {
        b->cap = nullptr;
        lbm_batch_destroy(b);
        return fail(LBM_EDEVICE, "capture stream creation failed");
    }
    st = upload_tiles(b, stream);
    if (st != LBM_OK) {
        lbm_batch_destroy(b);
        return st;
    }
    *out = b;
    return LBM_OK;
}

lbm_status lbm_batch_step(lbm_batch* b, int64_t nsteps, hipStream_t stream) {
    if (!b || nsteps < 0) return fail(LBM_EINVAL, "invalid arguments");
    int64_t left = nsteps;
    if (left >= b->graph_steps) {
        if (b->cur == 1) {  // align to the captured parity
            launch_batch(b, 1, stream);
            HIP_TRY(hipGetLastError());
            set_parity(b, 0);
            --left;
        }
        lbm_status st = ensure_graph(b);
        if (st != LBM_OK) return st;
        while (left >= b->graph_steps) {
            HIP_TRY(hipGraphLaunch(b->exec, stream));
            left -= b->graph_steps;
        }
    }
    for (; left > 0; --left) {
        launch_batch(b, b->cur, stream);
        HIP_TRY(hipGetLastError());
        set_parity(b, 1 - b->cur);
    }
    b->steps += nsteps;
    for (auto* d : b->doms) d->steps = b->steps;
    return LBM_OK;
}

lbm_status lbm_batch_step_separate(lbm_batch* b, int64_t nsteps, hipStream_t stream) {
    if (!b || nsteps < 0) return fail(LBM_EINVAL, "invalid arguments");
    for (int64_t s = 0; s < nsteps; ++s) {
        for (auto* d : b->doms) {
            lbm_status st = lbm_step(d, 1, stream);
            if (st != LBM_OK) return st;
        }
        b->cur = 1 - b->cur;
    }
    b->steps += nsteps;
    for (auto* d : b->doms) d->steps = b->steps;
    return LBM_OK;
}

lbm_domain* lbm_batch_domain(lbm_batch* b, int32_t i) {
    if (!b || i < 0 || i >= b->n) return nullptr;
    return b->doms[i];
}

lbm_status lbm_batch_set_schedule(lbm_batch* b, int32_t tile_y, int32_t order, int32_t grid, hipStream_t stream) {
    if (!b) return fail(LBM_EINVAL, "NULL batch");
    if ((tile_y != 4 && tile_y != 8) || order < 0 || order > 3 || grid < 0)
        return fail(LBM_EINVAL, "schedule tile_y %d, order %d, grid %d", tile_y, order, grid);
    b->tile_y = tile_y;
    b->order = order;
    b->grid = grid;
    // the new worklist is copied on `stream`, behind every launch already
    // queued there, and the stream is synchronised before the graph that
    // reads the old worklist is destroyed
    return upload_tiles(b, stream);
}

lbm_status lbm_batch_get_schedule(const lbm_batch* b, int32_t* tile_y, int32_t* order, int32_t* grid) {
    if (!b || !tile_y || !order || !grid) return fail(LBM_EINVAL, "NULL argument");
    *tile_y = b->tile_y;
    *order = b->order;
    *grid = b->grid;
    return LBM_OK;
}

lbm_status lbm_batch_autotune(lbm_batch* b, int32_t probe_steps, hipStream_t stream, char* report, size_t report_len) {
    if (!b || probe_steps < 1) return fail(LBM_EINVAL, "invalid arguments");
    HIP_TRY(hipStreamSynchronize(stream));
    std::string key;
    lbm_status kst = tune_key(b, &key);
    if (kst != LBM_OK) return kst;
    bool cached = false;
    TuneChoice kept{};
    {
        std::lock_guard<std::mutex> lock(tune_mutex);
        auto it = tune_cache.find(key);
        if (it != tune_cache.end()) {
            cached = true;
            kept = it->second;
        }
    }
    if (cached) {  // (the lock is released: the upload synchronises the stream)
        b->tile_y = kept.tile_y;
        b->order = kept.order;
        b->grid = kept.grid;
        lbm_status st = upload_tiles(b, stream);
        if (st != LBM_OK) return st;
        if (report && report_len) {
            char buf[128];
            snprintf(buf, sizeof(buf), "{\"cached\": true, \"best\": \"ty%d_o%d_g%d\"}", b->tile_y, b->order, b->grid);
            std::strncpy(report, buf, report_len - 1);
            report[report_len - 1] = 0;
        }
        return LBM_OK;
    }
    // snapshot every domain's current populations
    const int cur0 = b->cur;
    std::vector<size_t> soff(b->n);
    size_t pos = 0;
    for (int i = 0; i < b->n; ++i) {
        soff[i] = b->off_snap + pos;
        HIP_TRY(hipMemcpyAsync(b->ws + soff[i], b->doms[i]->ws + b->doms[i]->off_f[cur0], b->doms[i]->off_f[1],
                               hipMemcpyDeviceToDevice, stream));
        pos += align256(b->doms[i]->off_f[1]);
    }
    hipEvent_t e0, e1;
    HIP_TRY(hipEventCreate(&e0));
    HIP_TRY(hipEventCreate(&e1));
    const int tys[2] = {4, 8};
    const int grids[5] = {0, 256, 512, 1024, 2048};
    constexpr int NORDER = 4;
    float best = 1e30f;
    int bt = b->tile_y, bo = b->order, bg = b->grid;
    std::string rep = "{";
    for (int ty : tys)
        for (int order = 0; order < NORDER; ++order)
            for (int grid : grids) {
                b->tile_y = ty;
                b->order = order;
                b->grid = grid;
                lbm_status st = upload_tiles(b, stream);
                if (st != LBM_OK) return st;
                for (int w = 0; w < 2; ++w) {
                    launch_batch(b, b->cur, stream);
                    set_parity(b, 1 - b->cur);
                }
                HIP_TRY(hipEventRecord(e0, stream));
                for (int s = 0; s < probe_steps; ++s) {
                    launch_batch(b, b->cur, stream);
                    set_parity(b, 1 - b->cur);
                }
                HIP_TRY(hipEventRecord(e1, stream));
                HIP_TRY(hipEventSynchronize(e1));
                HIP_TRY(hipGetLastError());
                float ms = 0;
                HIP_TRY(hipEventElapsedTime(&ms, e0, e1));
                char buf[96];
                snprintf(buf, sizeof(buf), "%s\"ty%d_o%d_g%d\": %.5f", rep.size() > 1 ? ", " : "", ty, order, grid,
                         ms / probe_steps);
                rep += buf;
                if (ms < best) { best = ms; bt = ty; bo = order; bg = grid; }
            }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    char buf[128];
    snprintf(buf, sizeof(buf), ", \"cached\": false, \"best\": \"ty%d_o%d_g%d\"}", bt, bo, bg);
    rep += buf;
    {
        std::lock_guard<std::mutex> lock(tune_mutex);
        tune_cache[key] = TuneChoice{bt, bo, bg};
    }
    // restore the snapshot into the original parity and rebuild the potential fields
    set_parity(b, cur0);
    for (int i = 0; i < b->n; ++i) {
        HIP_TRY(hipMemcpyAsync(b->doms[i]->ws + b->doms[i]->off_f[cur0], b->ws + soff[i], b->doms[i]->off_f[1],
                               hipMemcpyDeviceToDevice, stream));
        lbm_status st = launch_phi(b->doms[i], cur0, stream);
        if (st != LBM_OK) return st;
    }
    b->tile_y = bt;
    b->order = bo;
    b->grid = bg;
    lbm_status st = upload_tiles(b, stream);
    if (st != LBM_OK) return st;
    if (report && report_len) {
        std::strncpy(report, rep.c_str(), report_len - 1);
        report[report_len - 1] = 0;
    }
    return LBM_OK;
}

void lbm_batch_tune_cache_clear(void) {
    std::lock_guard<std::mutex> lock(tune_mutex);
    tune_cache.clear();
}

lbm_status lbm_batch_check_finite(lbm_batch* b, int32_t* flags, hipStream_t stream) {
    if (!b || !flags) return fail(LBM_EINVAL, "NULL argument");
    int* df = reinterpret_cast<int*>(b->ws + b->off_flags);
    hipLaunchKernelGGL(k_fill_int, dim3(1), dim3(lbm::NT), 0, stream, df, b->n, 0);
    const int ty = b->tile_y;
    if (b->prec == LBM_F32) {
        const auto* descs = reinterpret_cast<const lbm::StepArgs<float>*>(b->ws + b->off_desc[b->cur]);
        hipLaunchKernelGGL((lbm::k_batch_finite<float>), dim3(b->ntiles), dim3(lbm::NT), 0, stream, descs,
                           reinterpret_cast<const lbm::BatchTile*>(b->ws + b->off_tiles), b->ntiles, ty, df);
    } else {
        const auto* descs = reinterpret_cast<const lbm::StepArgs<double>*>(b->ws + b->off_desc[b->cur]);
        hipLaunchKernelGGL((lbm::k_batch_finite<double>), dim3(b->ntiles), dim3(lbm::NT), 0, stream, descs,
                           reinterpret_cast<const lbm::BatchTile*>(b->ws + b->off_tiles), b->ntiles, ty, df);
    }
    HIP_TRY(hipGetLastError());
    std::vector<int> h(b->n);
    HIP_TRY(hipMemcpyAsync(h.data(), df, b->n * sizeof(int), hipMemcpyDeviceToHost, stream));
    HIP_TRY(hipStreamSynchronize(stream));
    int any = 0;
    for (int i = 0; i < b->n; ++i) { flags[i] = h[i] ? 1 : 0; any |= flags[i]; }
    return any ? fail(LBM_ENONFINITE, "non-finite density in at least one domain") : LBM_OK;
}

void lbm_batch_destroy(lbm_batch* b) {
    if (!b) return;
    if (b->graph_ok) (void)hipGraphExecDestroy(b->exec);
    if (b->cap) (void)hipStreamDestroy(b->cap);
    for (auto* d : b->doms) lbm_destroy(d);
    delete b;
}

}  // extern "C"
