// gram.hip -- batched sketched Gram matrices (the os_gram_* entry points):
// the Hessian sketch of the log-barrier interior-point method (Section 5.2,
// Eq. (int_point) and the Hessian after it), H = (A D^{1/2} S)(A D^{1/2} S)^T
// / K for a batch of problems of different sizes.
//
// The prepared sketches of all problems are built by one hash launch and one
// list launch; per problem the weighted sketch of A's rows (only the kept
// blocks stored) goes to the workspace; then one persistent launch computes
// the upper-triangle tiles of every H.  Its schedule is made on the
// host: tiles sorted by cost (the problem's K depth) and each given to the
// least-loaded workgroup (longest-processing-time-first), stored grouped by
// workgroup.
#include <algorithm>
#include <functional>
#include <new>
#include <queue>
#include <utility>
#include <vector>

#include "api_common.h"

using namespace osk::api;

struct os_gram_plan {
    struct Prob {
        os_sketch sk;
        const float* A;
        int64_t lda;
        const float* d;
        int64_t m;
        int64_t n;
        float* H;
        int64_t ldh;
        std::vector<uint8_t> keep;   // N+e flags
        int32_t K;                   // kept (= stored) blocks
        int32_t bp;
        int64_t ld;                  // sketch leading dimension: K * bp rounded up to 64
        size_t prep_off;
        size_t prep_bytes;
        size_t sketch_off;
    };
    std::vector<Prob> probs;
    int full = 1;
    size_t desc_off = 0;
    size_t prep_desc_off = 0;        // osk::PrepDesc per problem (batched prepare)
    int64_t hash_tasks = 0;
    int64_t list_tasks = 0;
    int32_t max_bp = 0;
    size_t tiles_off = 0;
    size_t starts_off = 0;
    size_t total = 0;
    int64_t max_tiles = 0;           // tile list capacity (the 128 tile side)
    int32_t tile = 0;
    int32_t grid = 0;
    const void* ws = nullptr;        // workspace of the last configuration
    // The sketch step runs the problems on kLanes streams (the caller's and
    // kLanes - 1 owned ones, default priority) joined by events, so small
    // sketches overlap; lane[k] is problem k's stream index (balanced by
    // bytes read).  Created by the first os_gram_configure.
    static constexpr int kLanes = 4;
    hipStream_t aux[kLanes - 1] = {};
    hipEvent_t fork = nullptr;
    hipEvent_t join[kLanes - 1] = {};
    std::vector<int32_t> lane;

    ~os_gram_plan() {
        for (auto& a : aux)
            if (a) (void)hipStreamDestroy(a);
        for (auto& j : join)
            if (j) (void)hipEventDestroy(j);
        if (fork) (void)hipEventDestroy(fork);
    }
};

namespace {

constexpr int32_t kMaxGrid = 65536;
// Longest tile list (tile side 128) a plan accepts.
constexpr int64_t kMaxTiles = int64_t(1) << 24;
// Cost of a tile's epilogue in K steps (one more for a mirrored tile).
constexpr int64_t kEpilogueCost = 2;

int64_t tiles_of(int64_t m, int tile) {
    const int64_t t = (m + tile - 1) / tile;
    return t * (t + 1) / 2;
}

os_status check_problem(const os_gram_problem& p) {
    os_status st = check_sketch(&p.sk);
    if (st != OS_OK) return st;
    if ((st = check_len(p.n)) != OS_OK) return st;
    if ((st = check_extent(p.m)) != OS_OK) return st;
    if ((st = check_matrix(p.A, p.m, p.n, p.lda, false)) != OS_OK) return st;
    if ((st = check_matrix(p.H, p.m, p.m, p.ldh, false)) != OS_OK) return st;
    if (p.d && !aligned(p.d, 4)) return OS_EALIGN;
    return OS_OK;
}

// Default number of persistent workgroups: as many as are resident at once.
int32_t default_grid(int tile) {
    int dev = 0, cus = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
        return 0;
    const int per_cu = osk::batch_sym_blocks_per_cu(tile);
    return (int32_t)std::min<int64_t>((int64_t)cus * std::max(per_cu, 1), kMaxGrid);
}

// Jobs of the mixed form for one problem of m rows and ksteps K steps
// (see launch_gemm_batch_sym): 256 tiles (i, j), i < j, with more than 128
// live columns are kind 0; each diagonal 256 tile becomes the 128 tiles on
// or above its diagonal, a last tile column of at most 128 live columns the
// 128 tiles that hold them, and those 128 tiles are paired in order into
// kind-1 jobs.  Costs are in sixteenths of a 256-tile K step on one CU:
// a 256 tile keeps each SIMD busy with 16 MFMA blocks per step, a pair of
// 128 tiles with 8 at about 10 % lower efficiency (more LDS reads per
// MFMA), a lone 128 tile with 4 on one wave per SIMD (less latency hidden).
template <typename ItemT>
void mixed_items(int64_t m, int32_t ksteps, bool full, int32_t prob, std::vector<ItemT>& items) {
    const int64_t T = (m + 255) / 256;
    std::vector<std::pair<int32_t, int32_t>> small;
    for (int64_t i = 0; i < T; ++i) {
        const bool rows2 = m - 256 * i > 128;          // tile row i holds two 128 rows
        for (int64_t j = i; j < T; ++j) {
            const bool cols2 = m - 256 * j > 128;
            if (i == j) {
                small.push_back({(int32_t)(2 * i), (int32_t)(2 * i)});
                if (rows2) {
                    small.push_back({(int32_t)(2 * i), (int32_t)(2 * i + 1)});
                    small.push_back({(int32_t)(2 * i + 1), (int32_t)(2 * i + 1)});
                }
            } else if (cols2) {
                const int64_t epi = 16 * kEpilogueCost * (1 + full);
                items.push_back({16 * (int64_t)ksteps + epi, prob, 0, (int32_t)i, (int32_t)j, 0, 0, 0});
            } else {
                small.push_back({(int32_t)(2 * i), (int32_t)(2 * j)});
                small.push_back({(int32_t)(2 * i + 1), (int32_t)(2 * j)});
            }
        }
    }
    auto epi128 = [&](const std::pair<int32_t, int32_t>& t) {
        return (int64_t)4 * kEpilogueCost * (1 + (full && t.first != t.second));
    };
    for (size_t t = 0; t < small.size(); t += 2) {
        const auto& x = small[t];
        if (t + 1 < small.size()) {
            const auto& y = small[t + 1];
            items.push_back({9 * (int64_t)ksteps + epi128(x) + epi128(y), prob, 1, x.first,
                             x.second, y.first, y.second, 1});
        } else {
            items.push_back({6 * (int64_t)ksteps + epi128(x), prob, 1, x.first, x.second, 0, 0, 0});
        }
    }
}

os_status check_ws(const os_gram_plan* plan, const void* ws, size_t ws_bytes) {
    if (!ws) return OS_ENULL;
    if (!aligned(ws, 256)) return OS_EALIGN;
    if (ws_bytes < plan->total) return OS_EWORKSPACE;
    return OS_OK;
}

char* at(void* ws, size_t off) { return static_cast<char*>(ws) + off; }

os_status enqueue(const os_gram_plan* plan, int stages, void* ws, hipStream_t s) {
    if (stages & OS_GRAM_PREPARE) {
        const auto* descs = reinterpret_cast<const osk::PrepDesc*>(at(ws, plan->prep_desc_off));
        const int32_t count = (int32_t)plan->probs.size();
        hipError_t e = osk::launch_table_batch(descs, count, plan->hash_tasks, s);
        if (e == hipSuccess)
            e = osk::launch_lists_batch(descs, count, plan->list_tasks, plan->max_bp, s);
        if (e != hipSuccess) return hip_status(e);
    }
    if (stages & OS_GRAM_SKETCH) {
        constexpr int L = os_gram_plan::kLanes;
        hipStream_t lanes[L] = {s, plan->aux[0], plan->aux[1], plan->aux[2]};
        hipError_t e = hipEventRecord(plan->fork, s);
        for (int j = 1; j < L && e == hipSuccess; ++j) e = hipStreamWaitEvent(lanes[j], plan->fork, 0);
        if (e != hipSuccess) return hip_status(e);
        os_status st = OS_OK;
        for (size_t k = 0; k < plan->probs.size() && st == OS_OK; ++k) {
            const auto& p = plan->probs[k];
            const void* prep = at(ws, p.prep_off);
            Blocks bs;
            if ((st = block_sets(&p.sk, p.keep.data(), 1, bs)) != OS_OK) break;
            st = hip_status(osk::launch_sketch_cols(
                p.A, p.m, p.n, p.lda, bs.stored, bs.nst, nblocks(&p.sk), p.bp,
                prep_lists(prep, &p.sk, p.n), reinterpret_cast<float*>(at(ws, p.sketch_off)),
                p.ld, lanes[plan->lane[k]], p.d));
        }
        // join every lane back into s, also after an error (a capture must end joined)
        for (int j = 1; j < L; ++j) {
            hipError_t ej = hipEventRecord(plan->join[j - 1], lanes[j]);
            if (ej == hipSuccess) ej = hipStreamWaitEvent(s, plan->join[j - 1], 0);
            if (ej != hipSuccess && st == OS_OK) st = hip_status(ej);
        }
        if (st != OS_OK) return st;
    }
    if (!(stages & OS_GRAM_PRODUCT)) return OS_OK;
    return hip_status(osk::launch_gemm_batch_sym(
        reinterpret_cast<const osk::BatchProblem*>(at(ws, plan->desc_off)),
        reinterpret_cast<const int4*>(at(ws, plan->tiles_off)),
        reinterpret_cast<const int32_t*>(at(ws, plan->starts_off)), plan->tile, plan->full,
        plan->grid, s));
}

os_status check_run(const os_gram_plan* plan, int stages, void* ws, size_t ws_bytes) {
    if (!plan) return OS_ENULL;
    if (stages < 1 || stages > OS_GRAM_ALL) return OS_EINVAL;
    const os_status st = check_ws(plan, ws, ws_bytes);
    if (st != OS_OK) return st;
    if (plan->tile == 0 || plan->ws != ws) return OS_EINVAL;   // not configured for ws
    return OS_OK;
}

}  // namespace

extern "C" {

os_status os_gram_plan_create(const os_gram_problem* probs, int32_t count, int full,
                              os_gram_plan** plan_out) {
    if (!plan_out) return OS_ENULL;
    *plan_out = nullptr;
    if (!probs) return OS_ENULL;
    if (count < 1 || count > OS_GRAM_MAX_PROBLEMS) return OS_EINVAL;
    os_gram_plan* plan = new (std::nothrow) os_gram_plan;
    if (!plan) return OS_EINVAL;
    os_status st = OS_OK;
    try {
        plan->full = full != 0;
        plan->probs.resize((size_t)count);
        size_t off = align256((size_t)count * sizeof(osk::BatchProblem));
        plan->desc_off = 0;
        plan->prep_desc_off = off;
        off += align256((size_t)count * sizeof(osk::PrepDesc));
        int64_t ntiles = 0;
        for (int32_t k = 0; k < count && st == OS_OK; ++k) {
            const os_gram_problem& p = probs[k];
            if ((st = check_problem(p)) != OS_OK) break;
            Blocks bs;
            if ((st = block_sets(&p.sk, p.keep, 1, bs)) != OS_OK) break;
            auto& q = plan->probs[(size_t)k];
            q.sk = p.sk;
            q.A = p.A;
            q.lda = p.lda;
            q.d = p.d;
            q.m = p.m;
            q.n = p.n;
            q.H = p.H;
            q.ldh = p.ldh;
            q.keep.resize((size_t)nblocks(&p.sk));
            bool kept[OS_MAX_BLOCKS];
            kept_flags(&p.sk, p.keep, kept);
            for (int32_t i = 0; i < nblocks(&p.sk); ++i) q.keep[(size_t)i] = kept[i] ? 1 : 0;
            q.K = bs.nst;
            q.bp = os_block_stride(p.sk.b);
            q.ld = osk::round_up((int64_t)q.K * q.bp, 64);   // whole pairs of 32-column steps
            if (!osk::plan_sketch_ok(p.m, q.K, q.bp, p.n) ||
                !osk::plan_gemm_ok(p.m, p.m, q.bp, q.ld, q.ld, 4)) {
                st = OS_EINVAL;
                break;
            }
            ntiles += tiles_of(p.m, 128);
            if (ntiles > kMaxTiles) {
                st = OS_EINVAL;
                break;
            }
        }
        if (st == OS_OK) {
            plan->max_tiles = ntiles;
            plan->tiles_off = off;
            off += align256((size_t)ntiles * 2 * sizeof(int4));   // mixed jobs: two int4
            plan->starts_off = off;
            off += align256((size_t)(kMaxGrid + 1) * sizeof(int32_t));
            for (auto& q : plan->probs) {
                const int64_t nt = table_stride(q.n);
                plan->hash_tasks += (int64_t)nblocks(&q.sk) * ((nt + 255) / 256);
                plan->list_tasks += (int64_t)nblocks(&q.sk) * ((q.n + osk::kSketchWindow - 1) /
                                                                osk::kSketchWindow);
                plan->max_bp = std::max(plan->max_bp, q.bp);
                q.prep_off = off;
                q.prep_bytes = prepare_bytes(&q.sk, q.n);
                off += align256(q.prep_bytes);
                q.sketch_off = off;
                off += align256((size_t)q.m * (size_t)q.ld * sizeof(float));
            }
            plan->total = off;
            // lanes of the sketch step: largest problems first, each to the
            // lane with the fewest bytes so far
            std::vector<int32_t> order((size_t)count);
            for (int32_t k = 0; k < count; ++k) order[(size_t)k] = k;
            auto bytes = [&](int32_t k) {
                const auto& q = plan->probs[(size_t)k];
                return (double)q.m * (double)q.n;
            };
            std::stable_sort(order.begin(), order.end(),
                             [&](int32_t a, int32_t b) { return bytes(a) > bytes(b); });
            double load[os_gram_plan::kLanes] = {};
            plan->lane.assign((size_t)count, 0);
            for (int32_t k : order) {
                int j = 0;
                for (int t = 1; t < os_gram_plan::kLanes; ++t)
                    if (load[t] < load[j]) j = t;
                plan->lane[(size_t)k] = j;
                load[j] += bytes(k);
            }
        }
    } catch (...) {
        st = OS_EINVAL;
    }
    if (st != OS_OK) {
        delete plan;
        return st;
    }
    *plan_out = plan;
    return OS_OK;
}

void os_gram_plan_destroy(os_gram_plan* plan) { delete plan; }

size_t os_gram_workspace_bytes(const os_gram_plan* plan) { return plan ? plan->total : 0; }

void os_gram_config(const os_gram_plan* plan, int32_t* tile, int32_t* grid) {
    if (tile) *tile = plan ? plan->tile : 0;
    if (grid) *grid = plan ? plan->grid : 0;
}

os_status os_gram_configure(os_gram_plan* plan, int32_t tile, int32_t grid, void* workspace,
                            size_t ws_bytes, void* stream) {
    if (!plan) return OS_ENULL;
    if (tile == 0) tile = OS_GRAM_MIXED;
    if ((tile != 128 && tile != 256 && tile != OS_GRAM_MIXED) || grid < 0 || grid > kMaxGrid)
        return OS_EINVAL;
    os_status st = check_ws(plan, workspace, ws_bytes);
    if (st != OS_OK) return st;
    if (grid == 0 && (grid = default_grid(tile)) < 1) return hip_status(hipErrorInvalidDevice);
    hipStream_t s = (hipStream_t)stream;
    if (!plan->fork) {
        hipError_t e = hipEventCreateWithFlags(&plan->fork, hipEventDisableTiming);
        for (int j = 0; j < os_gram_plan::kLanes - 1 && e == hipSuccess; ++j) {
            e = hipStreamCreateWithFlags(&plan->aux[j], hipStreamNonBlocking);
            if (e == hipSuccess) e = hipEventCreateWithFlags(&plan->join[j], hipEventDisableTiming);
        }
        if (e != hipSuccess) return hip_status(e);
    }
    try {
        const size_t count = plan->probs.size();
        std::vector<osk::BatchProblem> desc(count);
        std::vector<osk::PrepDesc> prep(count);
        int64_t hash_task0 = 0, list_task0 = 0;
        for (size_t k = 0; k < count; ++k) {
            const auto& q = plan->probs[k];
            osk::PrepDesc& d = prep[k];
            d = osk::PrepDesc{};
            d.seed = q.sk.seed;
            d.h = q.sk.h;
            d.sigma = q.sk.sigma;
            d.table = reinterpret_cast<uint32_t*>(at(workspace, q.prep_off));
            d.n = q.n;
            d.nt = table_stride(q.n);
            d.b = q.sk.b;
            d.bp = q.bp;
            d.nblk = nblocks(&q.sk);
            d.hash_chunks = (int32_t)((d.nt + 255) / 256);
            d.hash_task0 = hash_task0;
            d.ell_task0 = list_task0;
            osk::prep_desc_lists(d, const_cast<void*>(prep_lists(d.table, &q.sk, q.n)));
            hash_task0 += (int64_t)d.nblk * d.hash_chunks;
            list_task0 += (int64_t)d.nblk * d.nwin;
        }
        if (hash_task0 != plan->hash_tasks || list_task0 != plan->list_tasks) return OS_EINVAL;
        // (cost, problem, kind, tile row, tile col, second tile), in problem
        // and tile order; kind and the second tile are used by the mixed form
        struct Item {
            int64_t cost;
            int32_t prob, kind, ti, tj, ti2, tj2, has2;
        };
        std::vector<Item> items;
        items.reserve((size_t)plan->max_tiles);
        hipError_t e_pad = hipSuccess;
        for (size_t k = 0; k < count; ++k) {
            const auto& q = plan->probs[k];
            osk::BatchProblem& bp = desc[k];
            bp.S = reinterpret_cast<const float*>(at(workspace, q.sketch_off));
            bp.H = q.H;
            bp.ld = q.ld;
            bp.ldh = q.ldh;
            bp.m = q.m;
            bp.ksteps = (int32_t)(q.ld / osk::kBlockAlign);
            if (q.ld > (int64_t)q.K * q.bp && e_pad == hipSuccess)   // the padding step is zero
                e_pad = hipMemset2DAsync(at(workspace, q.sketch_off) + (size_t)q.K * q.bp * 4,
                                         (size_t)q.ld * 4, 0,
                                         (size_t)(q.ld - (int64_t)q.K * q.bp) * 4, (size_t)q.m, s);
            bp.scale = 1.0f / (float)q.K;
            if (tile == OS_GRAM_MIXED) {
                mixed_items(q.m, bp.ksteps, plan->full != 0, (int32_t)k, items);
                continue;
            }
            const int32_t T = (int32_t)((q.m + tile - 1) / tile);
            for (int32_t i = 0; i < T; ++i)
                for (int32_t j = i; j < T; ++j)
                    items.push_back({bp.ksteps + kEpilogueCost * (1 + (plan->full && i != j)),
                                     (int32_t)k, 0, i, j, 0, 0, 0});
        }
        std::stable_sort(items.begin(), items.end(),
                         [](const Item& a, const Item& b) { return a.cost > b.cost; });
        // longest-processing-time-first: each tile to the least-loaded workgroup
        using Load = std::pair<int64_t, int32_t>;
        std::priority_queue<Load, std::vector<Load>, std::greater<Load>> heap;
        for (int32_t g = 0; g < grid; ++g) heap.push({0, g});
        std::vector<int32_t> owner(items.size());
        std::vector<int32_t> starts((size_t)grid + 1, 0);
        for (size_t t = 0; t < items.size(); ++t) {
            Load l = heap.top();
            heap.pop();
            owner[t] = l.second;
            ++starts[(size_t)l.second + 1];
            heap.push({l.first + items[t].cost, l.second});
        }
        for (int32_t g = 0; g < grid; ++g) starts[(size_t)g + 1] += starts[(size_t)g];
        const int per = tile == OS_GRAM_MIXED ? 2 : 1;   // int4 per list entry
        std::vector<int4> tiles(items.size() * per);
        std::vector<int32_t> fill(starts.begin(), starts.end() - 1);
        for (size_t t = 0; t < items.size(); ++t) {
            const Item& it = items[t];
            const size_t at_ = (size_t)fill[(size_t)owner[t]]++ * per;
            if (per == 1) {
                tiles[at_] = make_int4(it.prob, it.ti, it.tj, 0);
            } else {
                tiles[at_] = make_int4(it.prob, it.kind, it.ti, it.tj);
                tiles[at_ + 1] = make_int4(it.ti2, it.tj2, it.has2, 0);
            }
        }
        hipError_t e = e_pad;
        if (e == hipSuccess)
            e = hipMemcpyAsync(at(workspace, plan->desc_off), desc.data(),
                                      desc.size() * sizeof(osk::BatchProblem),
                                      hipMemcpyHostToDevice, s);
        if (e == hipSuccess)
            e = hipMemcpyAsync(at(workspace, plan->prep_desc_off), prep.data(),
                               prep.size() * sizeof(osk::PrepDesc), hipMemcpyHostToDevice, s);
        if (e == hipSuccess)
            e = hipMemcpyAsync(at(workspace, plan->tiles_off), tiles.data(),
                               tiles.size() * sizeof(int4), hipMemcpyHostToDevice, s);
        if (e == hipSuccess)
            e = hipMemcpyAsync(at(workspace, plan->starts_off), starts.data(),
                               starts.size() * sizeof(int32_t), hipMemcpyHostToDevice, s);
        if (e == hipSuccess) e = hipStreamSynchronize(s);
        if (e != hipSuccess) return hip_status(e);
    } catch (...) {
        return OS_EINVAL;
    }
    plan->tile = tile;
    plan->grid = grid;
    plan->ws = workspace;
    return OS_OK;
}

os_status os_gram_run(const os_gram_plan* plan, int stages, void* workspace, size_t ws_bytes,
                      void* stream) {
    const os_status st = check_run(plan, stages, workspace, ws_bytes);
    if (st != OS_OK) return st;
    return enqueue(plan, stages, workspace, (hipStream_t)stream);
}

os_status os_gram_autotune_ex(os_gram_plan* plan, int32_t reps, void* workspace,
                              size_t ws_bytes, void* stream, os_gram_candidate* cands,
                              int32_t cap, int32_t* count, float* best_ms) {
    if (count) *count = 0;
    if (!plan) return OS_ENULL;
    if (reps < 1 || cap < 0 || (cap > 0 && !cands)) return OS_EINVAL;
    os_status st = check_ws(plan, workspace, ws_bytes);
    if (st != OS_OK) return st;
    hipStream_t s = (hipStream_t)stream;
    // the sketches the product reads: one run of the earlier stages in the
    // first candidate's configuration
    const int32_t tiles[3] = {OS_GRAM_MIXED, 256, 128};
    if ((st = os_gram_configure(plan, tiles[0], 0, workspace, ws_bytes, stream)) != OS_OK)
        return st;
    if ((st = enqueue(plan, OS_GRAM_PREPARE | OS_GRAM_SKETCH, workspace, s)) != OS_OK) return st;
    hipEvent_t t0 = nullptr, t1 = nullptr;
    hipError_t e = hipEventCreate(&t0);
    if (e == hipSuccess) e = hipEventCreate(&t1);
    if (e != hipSuccess) {
        if (t0) (void)hipEventDestroy(t0);
        return hip_status(e);
    }
    int32_t best_tile = 0, best_grid = 0, n = 0;
    float best = 0.f;
    for (int32_t c = 0; c < 3 && st == OS_OK && e == hipSuccess; ++c) {
        const int32_t resident = default_grid(tiles[c]);
        if (resident < 1) {
            st = hip_status(hipErrorInvalidDevice);
            break;
        }
        for (int32_t mult = 1; mult <= 2 && st == OS_OK; ++mult) {
            const int32_t grid = (int32_t)std::min<int64_t>((int64_t)resident * mult, kMaxGrid);
            if ((st = os_gram_configure(plan, tiles[c], grid, workspace, ws_bytes, stream)) != OS_OK)
                break;
            if ((st = enqueue(plan, OS_GRAM_PRODUCT, workspace, s)) != OS_OK) break;   // warm-up
            if ((e = hipEventRecord(t0, s)) != hipSuccess) break;
            for (int32_t r = 0; r < reps && st == OS_OK; ++r)
                st = enqueue(plan, OS_GRAM_PRODUCT, workspace, s);
            if (st != OS_OK) break;
            float ms = 0.f;
            if ((e = hipEventRecord(t1, s)) != hipSuccess || (e = hipEventSynchronize(t1)) != hipSuccess ||
                (e = hipEventElapsedTime(&ms, t0, t1)) != hipSuccess)
                break;
            ms /= (float)reps;
            if (n < cap) cands[n] = os_gram_candidate{tiles[c], grid, ms};
            ++n;
            if (best_tile == 0 || ms < best) {
                best = ms;
                best_tile = tiles[c];
                best_grid = grid;
            }
        }
    }
    (void)hipEventDestroy(t0);
    (void)hipEventDestroy(t1);
    if (e != hipSuccess) return hip_status(e);
    if (st != OS_OK) return st;
    if ((st = os_gram_configure(plan, best_tile, best_grid, workspace, ws_bytes, stream)) != OS_OK)
        return st;
    if (count) *count = n;
    if (best_ms) *best_ms = best;
    return OS_OK;
}

os_status os_gram_autotune(os_gram_plan* plan, int32_t reps, void* workspace, size_t ws_bytes,
                           void* stream, float* best_ms) {
    return os_gram_autotune_ex(plan, reps, workspace, ws_bytes, stream, nullptr, 0, nullptr,
                               best_ms);
}

os_status os_gram_graph_create(const os_gram_plan* plan, int stages, void* workspace,
                               size_t ws_bytes, void* stream, void** graph_out) {
    if (!graph_out) return OS_ENULL;
    *graph_out = nullptr;
    os_status st = check_run(plan, stages, workspace, ws_bytes);
    if (st != OS_OK) return st;
    if (!stream) return OS_EINVAL;      // the NULL stream cannot be captured
    hipStream_t s = (hipStream_t)stream;
    hipError_t e = hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal);
    if (e != hipSuccess) return hip_status(e);
    st = enqueue(plan, stages, workspace, s);
    hipGraph_t graph = nullptr;
    e = hipStreamEndCapture(s, &graph);
    if (st != OS_OK || e != hipSuccess) {
        if (graph) (void)hipGraphDestroy(graph);
        return st != OS_OK ? st : hip_status(e);
    }
    hipGraphExec_t exec = nullptr;
    e = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
    (void)hipGraphDestroy(graph);
    if (e != hipSuccess) return hip_status(e);
    *graph_out = exec;
    return OS_OK;
}

os_status os_graph_launch(void* graph, void* stream) {
    if (!graph) return OS_ENULL;
    return hip_status(hipGraphLaunch((hipGraphExec_t)graph, (hipStream_t)stream));
}

void os_graph_destroy(void* graph) {
    if (graph) (void)hipGraphExecDestroy((hipGraphExec_t)graph);
}

}  // extern "C"
