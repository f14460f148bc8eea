// batch.hip -- many planning problems per launch sequence.
//
// Every kernel of one extend iteration is launched once for all member
// problems, blockIdx.y (blockIdx.z for the scans) selecting the member's launch
// record in device memory; the sampler and the edge item kernel, which are
// specialised by robot kind, obstacle tile and obstacle-time mode, are launched
// once per scene class over its members.  A small problem alone cannot fill
// the 256 compute units; hundreds of them together do, and the whole
// iteration sequence of all of them is one HIP graph replay.
#include <math.h>
#include <string.h>

#include <algorithm>
#include <chrono>
#include <map>
#include <set>
#include <tuple>
#include <vector>

#include "edge_flat.hpp"
#include "pipeline.hpp"

namespace st {

__global__ void k_batch_status(PlanDev *const *pls, int n, int32_t *first_iter, float *U, int32_t *done) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const PlanDev *pl = pls[i];
    first_iter[i] = pl->first_iter;
    U[i] = pl->U;
    done[i] = pl->done;
}

template <class T>
static hipError_t upload(std::vector<void *> &owned, const std::vector<T> &h, const T **out) {
    T *d = nullptr;
    hipError_t e = hipMalloc((void **)&d, std::max<size_t>(h.size(), 1) * sizeof(T));
    if (e != hipSuccess) return e;
    owned.push_back(d);
    if (!h.empty()) e = hipMemcpy(d, h.data(), h.size() * sizeof(T), hipMemcpyHostToDevice);
    *out = d;
    return e;
}

}  // namespace st

using namespace st;

struct st_batch {
    std::vector<st_problem *> given;   // as passed to st_batch_create
    std::vector<int> record_of;        // launch record per given problem, -1 when not launched
    std::vector<uint8_t> trivial;      // per given problem
    std::vector<st_problem *> mem;     // launched members, record order
    std::vector<void *> saved_bufs;    // per member: work and edge buffers the records point to
    BatchLaunch L;
    std::vector<void *> owned;         // device allocations of the batch
    PlanDev **d_pls = nullptr;
    int32_t *d_first = nullptr, *d_done = nullptr;
    float *d_U = nullptr;
    int32_t *h_first = nullptr, *h_done = nullptr;  // pinned
    float *h_U = nullptr;
    int K = 4;
    hipGraphExec_t graph = nullptr;
    hipStream_t cap = nullptr;
    std::vector<hipEvent_t> ev;
};

namespace st {

static void batch_free(st_batch *b) {
    if (!b) return;
    (void)hipDeviceSynchronize();
    if (b->graph) (void)hipGraphExecDestroy(b->graph);
    if (b->cap) (void)hipStreamDestroy(b->cap);
    for (hipEvent_t e : b->ev) (void)hipEventDestroy(e);
    for (void *x : b->owned) (void)hipFree(x);
    if (b->h_first) (void)hipHostFree(b->h_first);
    if (b->h_done) (void)hipHostFree(b->h_done);
    if (b->h_U) (void)hipHostFree(b->h_U);
    delete b;
}

static std::vector<void *> member_bufs(const st_problem *p) {
    return {p->work.dir, p->work.br_key, p->ebufs.n, p->ebufs.items, (void *)(intptr_t)p->work.Bcap,
            (void *)(intptr_t)p->ebufs.cap};
}

// The launch records point into the members' work and edge buffers; a member
// whose buffers were reallocated since would make them dangle.
static int check_members(const st_batch *b) {
    for (size_t m = 0; m < b->mem.size(); ++m) {
        const std::vector<void *> now = member_bufs(b->mem[m]);
        for (size_t k = 0; k < now.size(); ++k)
            if (now[k] != b->saved_bufs[m * now.size() + k]) {
                set_error("batch member %zu changed its work buffers after st_batch_create", m);
                return ST_EINVAL;
            }
    }
    return ST_OK;
}

static int batch_build(st_batch *b) {
    const int P = (int)b->mem.size();
    BatchLaunch &L = b->L;
    L.P = P;
    if (P == 0) return ST_OK;
    // node slices per scan tile: the tiles actually used are about one per
    // 256 workers plus a partial one per node set, far fewer than the bound;
    // aim at a few thousand scan blocks in total, at least 8 slices each so
    // that a member's large tree is never scanned by a single block
    int64_t tiles = 0;
    for (st_problem *p : b->mem) tiles += (p->prm.batch + 255) / 256 + 2;
    const int nch = (int)std::min<int64_t>(64, std::max<int64_t>(8, 8192 / std::max<int64_t>(tiles, 1)));
    // item blocks per member: about 16384 over the batch, at least four each,
    // so that a member whose bridges are long spreads them over many waves
    const int min_items = std::max(4, 16384 / P);
    int64_t all_edges = 0;
    for (st_problem *p : b->mem) all_edges += p->prm.batch;
    std::vector<SampleArgs> smp(P);
    std::vector<ScanArgs> scan_nn(P), scan_br(P);
    std::vector<SteerArgs> steer(P);
    std::vector<EdgeArgs> edge_ext(P), edge_br(P);
    std::vector<InsertArgs> ins(P);
    std::vector<BridgeArgs> merge(P);
    std::vector<PublishArgs> pub(P);
    std::vector<RootsArgs> roots(P);
    std::vector<int32_t> all, ir, rr;
    std::map<std::tuple<int, int, int, int, int>, std::vector<int32_t>> cls;
    std::vector<PlanDev *> pls(P);
    L.nch = nch;
    // one-wave scan blocks when every member draws at most 64 samples
    int64_t B_max = 0;
    for (st_problem *p : b->mem) B_max = std::max<int64_t>(B_max, p->prm.batch);
    L.scan_tq = B_max <= 64 ? 64 : 256;
    for (int m = 0; m < P; ++m) {
        st_problem *p = b->mem[m];
        const int64_t B = p->prm.batch;
        const st_samples s = work_samples_of(p);
        smp[m] = make_sample_args(p, -1, B, s, true);
        IterArgs a;
        make_iter_args(p, B, s, nullptr, nch, nch, min_items, all_edges, a);
        scan_nn[m] = a.scan_nn;
        scan_br[m] = a.scan_br;
        steer[m] = a.steer;
        // the batch's extension launch: the most edges per block (fewer, fuller
        // blocks for its many members)
        if (a.edge_ext.flat > 0) a.edge_ext.flat = kFlatEdges;
        edge_ext[m] = a.edge_ext;
        edge_br[m] = a.edge_br;
        ins[m] = a.insert;
        merge[m] = a.merge;
        pub[m] = a.publish;
        roots[m] = a.roots;
        pls[m] = p->d_plan;
        all.push_back(m);
        (p->prm.variant == ST_INTERVAL_ROOT ? ir : rr).push_back(m);
        cls[std::make_tuple(p->sc.stat ? (int)kDHStatic : p->sc.kind, p->sc.ot, p->sc.obs_mode, a.edge_ext.split_shift,
                            a.edge_br.split_shift)]
            .push_back(m);
        // query tiles of the scans (tiles of L.scan_tq queries: one per node
        // set and a full one per L.scan_tq samples at most); the two
        // nearest-node launches each over their own members
        const int tiles_b = (int)((B + L.scan_tq - 1) / L.scan_tq);
        int &mt = p->prm.variant == ST_INTERVAL_ROOT ? L.mt_nn_ir : L.mt_nn_rr;
        mt = std::max(mt, tiles_b + p->tree.n_pools);
        L.mt_br = std::max(L.mt_br, tiles_b + 2);
        L.nb_worker = std::max<int>(L.nb_worker, (int)((B + 255) / 256));
        L.nb_edge = std::max(L.nb_edge, std::max(a.edge_ext.nb_edge, a.edge_br.nb_edge));
        L.max_pools = std::max(L.max_pools, p->tree.n_pools);
        L.ins_threads = std::max(L.ins_threads, insert_threads(B));
        L.ext_flat = L.ext_flat && a.edge_ext.flat > 0;
        const std::vector<void *> sb = member_bufs(p);
        b->saved_bufs.insert(b->saved_bufs.end(), sb.begin(), sb.end());
    }
    ST_HIP(upload(b->owned, smp, &L.sample));
    ST_HIP(upload(b->owned, scan_nn, &L.scan_nn));
    ST_HIP(upload(b->owned, scan_br, &L.scan_br));
    ST_HIP(upload(b->owned, steer, &L.steer));
    ST_HIP(upload(b->owned, edge_ext, &L.edge_ext));
    ST_HIP(upload(b->owned, edge_br, &L.edge_br));
    ST_HIP(upload(b->owned, ins, &L.insert));
    ST_HIP(upload(b->owned, merge, &L.merge));
    ST_HIP(upload(b->owned, pub, &L.publish));
    ST_HIP(upload(b->owned, roots, &L.roots));
    ST_HIP(upload(b->owned, all, &L.all_members));
    ST_HIP(upload(b->owned, ir, &L.ir_members));
    ST_HIP(upload(b->owned, rr, &L.rr_members));
    L.n_ir = (int)ir.size();
    L.n_rr = (int)rr.size();
    for (auto &kv : cls) {
        BatchClass c;
        memset(&c, 0, sizeof c);
        const st_problem *p0 = b->mem[kv.second[0]];
        c.key = p0->sc;
        c.split_ext = std::get<3>(kv.first);
        c.split_br = std::get<4>(kv.first);
        c.n = (int)kv.second.size();
        for (int32_t m : kv.second) {
            c.nb_sample = std::max(c.nb_sample, smp[m].nb);
            c.nb_items_ext = std::max(c.nb_items_ext, edge_ext[m].nb_items);
            c.nb_items_br = std::max(c.nb_items_br, edge_br[m].nb_items);
            if (edge_ext[m].flat > 0) c.nb_flat = std::max(c.nb_flat, flat_blocks(edge_ext[m].E, edge_ext[m].flat));
            c.nb_bcheck = std::max<int>(c.nb_bcheck, (int)b->mem[m]->prm.batch);  // one wave each
            c.lds = std::max(c.lds, scene_lds_bytes(b->mem[m]->sc));
            c.lds_sample = std::max(c.lds_sample, sample_lds_bytes(b->mem[m], nullptr));
        }
        ST_HIP(upload(b->owned, kv.second, &c.members));
        L.classes.push_back(c);
    }
    const PlanDev *const *dp = nullptr;
    ST_HIP(upload(b->owned, std::vector<const PlanDev *>(pls.begin(), pls.end()), &dp));
    b->d_pls = const_cast<PlanDev **>(dp);
    ST_HIP(hipMalloc((void **)&b->d_first, P * sizeof(int32_t)));
    b->owned.push_back(b->d_first);
    ST_HIP(hipMalloc((void **)&b->d_done, P * sizeof(int32_t)));
    b->owned.push_back(b->d_done);
    ST_HIP(hipMalloc((void **)&b->d_U, P * sizeof(float)));
    b->owned.push_back(b->d_U);
    ST_HIP(hipHostMalloc((void **)&b->h_first, P * sizeof(int32_t), hipHostMallocDefault));
    ST_HIP(hipHostMalloc((void **)&b->h_done, P * sizeof(int32_t), hipHostMallocDefault));
    ST_HIP(hipHostMalloc((void **)&b->h_U, P * sizeof(float), hipHostMallocDefault));
    // capture K iterations of every member
    ST_HIP(hipStreamCreateWithFlags(&b->cap, hipStreamNonBlocking));
    ST_HIP(hipStreamBeginCapture(b->cap, hipStreamCaptureModeThreadLocal));
    int rc = ST_OK;
    for (int i = 0; i < b->K && rc == ST_OK; ++i) rc = launch_batch_iteration(L, b->cap);
    hipGraph_t g = nullptr;
    const hipError_t e = hipStreamEndCapture(b->cap, &g);
    if (rc != ST_OK) {
        if (g) (void)hipGraphDestroy(g);
        return rc;
    }
    if (e != hipSuccess) {
        set_error("batch graph capture failed: %s", hipGetErrorString(e));
        return ST_EHIP;
    }
    const hipError_t e2 = hipGraphInstantiate(&b->graph, g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    if (e2 != hipSuccess) {
        set_error("batch graph instantiation failed: %s", hipGetErrorString(e2));
        return ST_EHIP;
    }
    // the graph's device-side set-up now, not in the first launch of a plan
    ST_HIP(hipGraphUpload(b->graph, b->cap));
    ST_HIP(hipStreamSynchronize(b->cap));
    return ST_OK;
}

static int batch_launch(st_batch *b, int64_t launches, hipStream_t s) {
    for (int64_t i = 0; i < launches; ++i) ST_HIP(hipGraphLaunch(b->graph, s));
    for (st_problem *p : b->mem) p->iter += launches * b->K;
    return ST_OK;
}

}  // namespace st

extern "C" {

int st_batch_create(st_problem *const *problems, int32_t n, int32_t iters_per_launch, st_batch **out) {
    if (!problems || !out || n < 1 || n > 4096 || iters_per_launch < 0 || iters_per_launch > 64) {
        set_error("st_batch_create: bad arguments");
        return ST_EINVAL;
    }
    *out = nullptr;
    std::set<const st_problem *> seen;
    for (int i = 0; i < n; ++i) {
        if (!problems[i] || !seen.insert(problems[i]).second) {
            set_error("st_batch_create: problem %d is null or repeated", i);
            return ST_EINVAL;
        }
        // a member's samples index the second grid dimension of the batched
        // bridge check (one block each)
        if (problems[i]->prm.batch > kBatchMaxSamples) {
            set_error("st_batch_create: problem %d draws %d samples per iteration (at most %d in a batch)", i,
                      (int)problems[i]->prm.batch, kBatchMaxSamples);
            return ST_EINVAL;
        }
    }
    st_batch *b = new (std::nothrow) st_batch();
    if (!b) {
        set_error("st_batch_create: out of host memory");
        return ST_ENOMEM;
    }
    b->K = iters_per_launch > 0 ? iters_per_launch : 4;
    int rc = ST_OK;
    for (int i = 0; i < n && rc == ST_OK; ++i) {
        st_problem *p = problems[i];
        b->given.push_back(p);
        bool start_free = false, triv = false;
        if ((rc = start_check(p, &start_free, &triv)) != ST_OK) break;
        b->trivial.push_back(triv ? 1 : 0);
        if (!start_free || triv) {
            b->record_of.push_back(-1);
            continue;
        }
        const int64_t B = p->prm.batch;
        if ((rc = work_reserve(p, B)) != ST_OK) break;
        if (p->ebufs.cap < B) {
            graphs_free(p);
            if ((rc = edge_bufs_reserve(p->ebufs, B)) != ST_OK) break;
        }
        b->record_of.push_back((int)b->mem.size());
        b->mem.push_back(p);
    }
    if (rc == ST_OK) rc = batch_build(b);
    if (rc != ST_OK) {
        batch_free(b);
        return rc;
    }
    *out = b;
    return ST_OK;
}

void st_batch_destroy(st_batch *b) { batch_free(b); }

int st_batch_iterate(st_batch *b, int64_t iters, void *stream) {
    if (!b || iters < 0) {
        set_error("st_batch_iterate: bad arguments");
        return ST_EINVAL;
    }
    if (b->mem.empty() || iters == 0) return ST_OK;
    const int rc = check_members(b);
    if (rc != ST_OK) return rc;
    return batch_launch(b, (iters + b->K - 1) / b->K, (hipStream_t)stream);
}

int st_batch_plan(st_batch *b, const st_budget *budget, st_batch_result *res) {
    if (!b || !budget || !res) {
        set_error("st_batch_plan: bad arguments");
        return ST_EINVAL;
    }
    const auto t0 = std::chrono::steady_clock::now();
    auto ms_since = [&]() {
        return std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
    };
    const int n = (int)b->given.size(), P = (int)b->mem.size();
    res->iterations = 0;
    res->n_solved = 0;
    int rc = check_members(b);
    if (rc != ST_OK) return rc;
    std::vector<int64_t> base(P);
    for (int m = 0; m < P; ++m) base[m] = b->mem[m]->iter;
    int64_t launches = 0;
    hipStream_t s = nullptr;
    if (P > 0) {
        // work the caller queued on other streams (state import, proposal) comes first
        ST_HIP(hipDeviceSynchronize());
        ST_HIP(hipStreamCreateWithFlags(&s, hipStreamNonBlocking));
        if (b->ev.empty()) {
            hipEvent_t e;
            ST_HIP(hipEventCreate(&e));
            b->ev.push_back(e);
        }
        ST_HIP(hipEventRecord(b->ev[0], s));
        const int64_t per_sync = std::max<int64_t>(1, ((budget->iters_per_sync > 0 ? budget->iters_per_sync : 8) +
                                                       b->K - 1) / b->K);
        const int64_t max_launches = budget->max_iters > 0 ? (budget->max_iters + b->K - 1) / b->K : -1;
        while (rc == ST_OK) {
            int64_t k = per_sync;
            if (max_launches >= 0) k = std::min(k, max_launches - launches);
            if (k <= 0) break;
            for (int64_t i = 0; i < k && rc == ST_OK; ++i) {
                if ((rc = batch_launch(b, 1, s)) != ST_OK) break;
                ++launches;
                if ((size_t)launches >= b->ev.size()) {
                    hipEvent_t e;
                    if (hipEventCreate(&e) != hipSuccess) {
                        set_error("st_batch_plan: event creation failed");
                        rc = ST_EHIP;
                        break;
                    }
                    b->ev.push_back(e);
                }
                if (hipEventRecord(b->ev[launches], s) != hipSuccess) {
                    set_error("st_batch_plan: event record failed");
                    rc = ST_EHIP;
                }
            }
            if (rc != ST_OK) break;
            k_batch_status<<<(P + 255) / 256, 256, 0, s>>>(b->d_pls, P, b->d_first, b->d_U, b->d_done);
            if (hipGetLastError() != hipSuccess ||
                hipMemcpyAsync(b->h_first, b->d_first, P * sizeof(int32_t), hipMemcpyDeviceToHost, s) != hipSuccess ||
                hipMemcpyAsync(b->h_done, b->d_done, P * sizeof(int32_t), hipMemcpyDeviceToHost, s) != hipSuccess ||
                hipMemcpyAsync(b->h_U, b->d_U, P * sizeof(float), hipMemcpyDeviceToHost, s) != hipSuccess ||
                hipStreamSynchronize(s) != hipSuccess) {
                set_error("st_batch_plan: device synchronisation failed");
                rc = ST_EHIP;
                break;
            }
            bool all_done = true, all_solved = true;
            for (int m = 0; m < P; ++m) {
                all_done = all_done && b->h_done[m];
                all_solved = all_solved && b->h_first[m] >= 0;
            }
            if (all_done) break;
            if (budget->stop_at_first && all_solved) break;
            if (budget->max_ms > 0 && ms_since() >= budget->max_ms) break;
            if (budget->max_iters <= 0 && budget->max_ms <= 0 && !budget->stop_at_first) break;
        }
        // final status of every member
        if (rc == ST_OK) {
            k_batch_status<<<(P + 255) / 256, 256, 0, s>>>(b->d_pls, P, b->d_first, b->d_U, b->d_done);
            if (hipGetLastError() != hipSuccess ||
                hipMemcpyAsync(b->h_first, b->d_first, P * sizeof(int32_t), hipMemcpyDeviceToHost, s) != hipSuccess ||
                hipMemcpyAsync(b->h_U, b->d_U, P * sizeof(float), hipMemcpyDeviceToHost, s) != hipSuccess ||
                hipStreamSynchronize(s) != hipSuccess) {
                set_error("st_batch_plan: device synchronisation failed");
                rc = ST_EHIP;
            }
        }
    }
    res->iterations = launches * b->K;
    for (int i = 0; i < n && rc == ST_OK; ++i) {
        const int m = b->record_of[i];
        double fm = NAN, U = INFINITY;
        int64_t fi = -1;
        if (b->trivial[i]) {
            fm = 0.0;
            fi = 0;
            U = 0.0;
        } else if (m >= 0) {
            const int32_t f = b->h_first[m];
            U = b->h_U[m];
            if (f >= 0) {
                fi = f;
                if (f < base[m]) {
                    fm = 0.0;
                } else {
                    const int64_t li = (f - base[m]) / b->K + 1;  // launch that ran iteration f
                    float t = 0.f;
                    if (li <= launches && hipEventElapsedTime(&t, b->ev[0], b->ev[li]) == hipSuccess) fm = t;
                }
            }
        }
        if (fi >= 0) res->n_solved++;
        if (res->first_ms) res->first_ms[i] = fm;
        if (res->first_iter) res->first_iter[i] = fi;
        if (res->arrival) res->arrival[i] = U;
    }
    if (s) (void)hipStreamDestroy(s);
    res->total_ms = ms_since();
    return rc;
}

int st_path_get(st_problem *p, st_path *out) {
    if (!p || !out) {
        set_error("st_path_get: bad arguments");
        return ST_EINVAL;
    }
    memset(out, 0, sizeof *out);
    out->dof = p->d;
    out->first_solution_iter = -1;
    out->arrival = INFINITY;
    out->length = INFINITY;
    ST_HIP(hipDeviceSynchronize());
    hipStream_t s = nullptr;
    ST_HIP(hipStreamCreateWithFlags(&s, hipStreamNonBlocking));
    const int rc = fetch_path(p, s, out);
    (void)hipStreamDestroy(s);
    return rc;
}

}  // extern "C"
