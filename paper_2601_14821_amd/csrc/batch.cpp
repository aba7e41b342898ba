// Batched scoring of many scenes and views of uneven sizes: a native runtime
// object that plans the buffers, enqueues project -> bin -> sort per job and one
// persistent render + removal launch over every (view, tile) of every job, and
// can record all of it into one HIP graph for replay.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <string>
#include <vector>

#include "common.h"
#include "fused.h"

namespace potr {
potr_status launch_count_pairs(int64_t N, int32_t V, const potr_camera* cams, const potr_config& cfg,
                               const float* means, const float* scales, const float* quats, const float* opac,
                               const float* sh, potr_proj* proj, int32_t* tt, int64_t* counts, hipStream_t s);
potr_status launch_check_overflow(const int64_t* n_pairs, const int64_t* caps, int32_t n, int32_t* flag,
                                  hipStream_t s);
potr_status launch_l1_grad(const float* image, const float* target, int64_t n, float w, float* dl, hipStream_t s);
}  // namespace potr

using namespace potr;

struct potr_batch_s {
    potr_config cfg;
    std::vector<potr_job> jobs;
    std::vector<std::vector<potr_camera>> cams;
    std::vector<int64_t> capacity;       // pairs per job (all its views)
    std::vector<int64_t> counted;        // pairs counted when planned
    // workspace layout (byte offsets)
    struct JobOff { size_t proj, ids, ranges; };
    std::vector<JobOff> off;
    // jobs run in lanes (job j in lane j % lanes): each lane has its own scratch
    // (tiles_touched, depth order, bin and sort workspaces) and, with more than
    // one lane, its own stream, forked from and joined back into the caller's
    struct LaneOff { size_t order, bin, stage, pix, g2d; };   // pix, g2d: fine-tuning scratch
    std::vector<LaneOff> lane_off;
    std::vector<size_t> lane_of;       // the lane of each job
    std::vector<hipStream_t> lane_s;
    std::vector<hipEvent_t> lane_ev;   // [0]: fork; [1 + l]: lane l done
    size_t off_table = 0, off_prefix = 0, off_counter = 0, off_npairs = 0, off_caps = 0, off_flag = 0;
    size_t bytes = 0;
    int32_t n_view_jobs = 0;
    int64_t n_items = 0;    // (view, tile) items of the render launch (none: no job asks for outputs)
    int32_t grid = 0;
    bool with_se = false;   // some job asks for dSE sums
    bool fixed = false;     // the jobs' outputs are fixed-point sums
    int n_out = 1;          // the most per-splat outputs of any job
    char* ws = nullptr;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
};

namespace {

constexpr size_t kLanes = 4;   // jobs in flight at once (streams of default priority)

int tiles_of(const potr_camera& c, const potr_config& g) { return tiles_x(c, g) * tiles_y(c, g); }

potr_status hip_ok(hipError_t e, const char* what) {
    if (e != hipSuccess) return fail(POTR_EHIP, "%s: %s", what, hipGetErrorString(e));
    return POTR_OK;
}

void plan_layout(potr_batch_s* b) {
    size_t o = 0;
    auto take = [&](size_t n) { size_t r = o; o += align_up(n > 0 ? n : 1); return r; };
    size_t max_vn = 0, max_bin = 0, max_stage = 0, max_pix = 0, max_g2d = 0;
    b->off.resize(b->jobs.size());
    b->n_view_jobs = 0;
    for (size_t j = 0; j < b->jobs.size(); ++j) {
        const potr_job& J = b->jobs[j];
        const int T = tiles_of(b->cams[j][0], b->cfg);
        b->off[j].proj = take((size_t)J.V * J.N * sizeof(potr_proj));
        b->off[j].ids = take((size_t)b->capacity[j] * 4);
        b->off[j].ranges = take((size_t)J.V * T * 2 * 4);
        max_vn = std::max(max_vn, (size_t)J.V * J.N * 4);
        max_bin = std::max(max_bin, bin_workspace_bytes(J.N, J.V, tiles_x(b->cams[j][0], b->cfg),
                                                         tiles_y(b->cams[j][0], b->cfg)));
        max_stage = std::max(max_stage, sort_workspace_bytes(b->capacity[j]));
        if (J.grad_target) {
            // image (then dL/dimage), P_K, T_final, stop position: 8 words per pixel;
            // the screen-space gradients: 9 per (view, splat)
            const size_t P = (size_t)b->cams[j][0].width * b->cams[j][0].height;
            max_pix = std::max(max_pix, (size_t)J.V * P * 8 * 4);
            max_g2d = std::max(max_g2d, (size_t)J.V * J.N * 9 * 4);
        }
        b->n_view_jobs += J.V;
    }
    b->lane_off.resize(std::min(kLanes, b->jobs.size()));
    // jobs go round the lanes, except that jobs adding into the same gradient
    // arrays (views of one scene with a fine-tuning step) share a lane: the
    // projection backward adds without atomics, so they must not overlap
    const size_t L = b->lane_off.size();
    std::vector<const float*> scenes;
    b->lane_of.resize(b->jobs.size());
    for (size_t j = 0; j < b->jobs.size(); ++j) {
        const potr_job& J = b->jobs[j];
        if (J.grad_target) {
            size_t k = std::find(scenes.begin(), scenes.end(), J.d_means) - scenes.begin();
            if (k == scenes.size()) scenes.push_back(J.d_means);
            b->lane_of[j] = k % L;
        } else {
            b->lane_of[j] = j % L;
        }
    }
    for (auto& L : b->lane_off) {
        L.order = take(max_vn);
        L.bin = take(max_bin);
        L.stage = take(max_stage);
        L.pix = take(max_pix);
        L.g2d = take(max_g2d);
    }
    b->off_table = take((size_t)b->n_view_jobs * sizeof(ViewJob));
    b->off_prefix = take((size_t)(b->n_view_jobs + 1) * 8);
    b->off_counter = take(8);
    b->off_npairs = take(b->jobs.size() * 8);
    b->off_caps = take(b->jobs.size() * 8);
    b->off_flag = take(4);
    b->bytes = o;
}

bool has_output(const potr_job& J) { return J.out.scores || J.out.scores_se || J.out.importance; }
bool has_step(const potr_job& J) { return J.grad_target != nullptr; }

potr_status validate_jobs(const potr_job* jobs, int32_t n_jobs, bool need_output = true) {
    if (!jobs || n_jobs < 1) return fail(POTR_EINVAL, "need at least one job");
    int fixed_mode = -1;   // the fixed_point of the first job with outputs
    for (int32_t j = 0; j < n_jobs; ++j) {
        const potr_job& J = jobs[j];
        if (J.N < 0 || J.V < 1 || J.N * (int64_t)J.V >= (int64_t(1) << 31) || !J.cams)
            return fail(POTR_EINVAL, "job %d: bad N/V/cams", j);
        if (J.N > 0 && (!J.means || !J.scales || !J.quats || !J.opac || !J.sh ||
                        (need_output && !has_output(J) && !has_step(J))))
            return fail(POTR_EINVAL, "job %d: NULL buffer", j);
        if (has_step(J) && J.N > 0 && (!J.d_means || !J.d_scales || !J.d_quats || !J.d_opac || !J.d_sh))
            return fail(POTR_EINVAL, "job %d: the fine-tuning step needs all five gradient arrays", j);
        if (has_step(J) && !(std::fabs(J.grad_weight) <= 3.0e38f))
            return fail(POTR_EINVAL, "job %d: grad_weight %g", j, (double)J.grad_weight);
        if (check_outputs(J.out, J.N, J.V, J.target) != POTR_OK) {
            const std::string why = potr_last_error();
            return fail(POTR_EINVAL, "job %d: %s", j, why.c_str());
        }
        if (J.N > 0 && (reinterpret_cast<uintptr_t>(J.sh) & 15u) != 0)
            return fail(POTR_EINVAL, "job %d: sh must be 16-byte aligned", j);
        if (has_output(J)) {
            if (fixed_mode < 0) fixed_mode = J.out.fixed_point;
            if (J.out.fixed_point != fixed_mode)
                return fail(POTR_EINVAL, "job %d: all jobs' outputs must be fixed point or none", j);
        }
    }
    return POTR_OK;
}

// Project every job once and count its pairs (synchronises; temporary memory).
potr_status count_jobs(const std::vector<potr_job>& jobs, const std::vector<std::vector<potr_camera>>& cams,
                       const potr_config& cfg, std::vector<int64_t>& out, hipStream_t s) {
    size_t need = 0;
    for (auto& J : jobs) need = std::max(need, (size_t)J.V * J.N * (sizeof(potr_proj) + 4) + 64 * 8 + 512);
    char* tmp = nullptr;
    potr_status st = hip_ok(hipMalloc(&tmp, need), "hipMalloc (pair count)");
    if (st != POTR_OK) return st;
    std::vector<int64_t> counts;
    out.assign(jobs.size(), 0);
    for (size_t j = 0; j < jobs.size() && st == POTR_OK; ++j) {
        const potr_job& J = jobs[j];
        if (J.N == 0) continue;
        potr_proj* proj = (potr_proj*)tmp;
        int32_t* tt = (int32_t*)(tmp + align_up((size_t)J.V * J.N * sizeof(potr_proj)));
        int64_t* cnt = (int64_t*)(tmp + align_up((size_t)J.V * J.N * sizeof(potr_proj)) +
                                  align_up((size_t)J.V * J.N * 4));
        for (int32_t v0 = 0; v0 < J.V && st == POTR_OK; v0 += 64) {
            const int32_t nv = std::min(64, J.V - v0);
            st = launch_count_pairs(J.N, nv, cams[j].data() + v0, cfg, J.means, J.scales, J.quats, J.opac, J.sh,
                                    proj, tt, cnt, s);
            if (st != POTR_OK) break;
            counts.assign(nv, 0);
            st = hip_ok(hipMemcpyAsync(counts.data(), cnt, nv * 8, hipMemcpyDeviceToHost, s), "copy counts");
            if (st == POTR_OK) st = hip_ok(hipStreamSynchronize(s), "sync");
            for (int32_t k = 0; k < nv; ++k) out[j] += counts[k];
        }
    }
    (void)hipFree(tmp);
    return st;
}

}  // namespace

extern "C" {

potr_status potr_batch_create(const potr_job* jobs, int32_t n_jobs, const potr_config* cfg, float margin,
                              potr_batch* out, void* stream) {
    if (!out || !cfg) return fail(POTR_EINVAL, "NULL argument");
    *out = nullptr;
    potr_status st = validate_jobs(jobs, n_jobs);
    if (st != POTR_OK) return st;
    if (!(margin >= 0.f) || margin > 10.f) return fail(POTR_EINVAL, "margin %g not in [0, 10]", margin);
    auto* b = new potr_batch_s();
    b->cfg = *cfg;
    for (int32_t j = 0; j < n_jobs; ++j) {
        b->jobs.push_back(jobs[j]);
        b->cams.emplace_back(jobs[j].cams, jobs[j].cams + jobs[j].V);
        b->jobs.back().cams = nullptr;
        for (int32_t v = 1; v < jobs[j].V; ++v)
            if (jobs[j].cams[v].width != jobs[j].cams[0].width || jobs[j].cams[v].height != jobs[j].cams[0].height) {
                delete b;
                return fail(POTR_EINVAL, "job %d: all views of a job need the same size", j);
            }
    }
    st = count_jobs(b->jobs, b->cams, b->cfg, b->counted, (hipStream_t)stream);
    if (st != POTR_OK) {
        delete b;
        return st;
    }
    b->capacity.resize(n_jobs);
    for (int32_t j = 0; j < n_jobs; ++j) {
        const double c = std::ceil((double)b->counted[j] * (1.0 + margin)) + 1024.0;
        if (c >= 2147483647.0) {
            delete b;
            return fail(POTR_EINVAL, "job %d: %lld pairs exceed one call's limit; split its views", j,
                        (long long)b->counted[j]);
        }
        b->capacity[j] = (int64_t)c;
    }
    plan_layout(b);
    b->with_se = false;
    b->n_out = 1;
    b->fixed = false;
    for (auto& J : b->jobs) {
        b->with_se = b->with_se || (J.N > 0 && J.out.scores_se != nullptr);
        const int n = (J.out.scores ? 1 : 0) + (J.out.importance ? 1 : 0) + (J.out.scores_se ? 1 : 0);
        b->n_out = std::max(b->n_out, n);
        b->fixed = b->fixed || (has_output(J) && J.out.fixed_point != 0);
    }
    b->grid = persistent_grid(b->cfg, b->n_out, b->fixed);
    if (b->lane_off.size() > 1) {
        st = POTR_OK;
        for (size_t l = 0; l < b->lane_off.size() && st == POTR_OK; ++l) {
            hipStream_t ls = nullptr;
            st = hip_ok(hipStreamCreateWithFlags(&ls, hipStreamNonBlocking), "lane stream");
            if (st == POTR_OK) b->lane_s.push_back(ls);
        }
        for (size_t e = 0; e < 1 + b->lane_off.size() && st == POTR_OK; ++e) {
            hipEvent_t ev = nullptr;
            st = hip_ok(hipEventCreateWithFlags(&ev, hipEventDisableTiming), "lane event");
            if (st == POTR_OK) b->lane_ev.push_back(ev);
        }
        if (st != POTR_OK) {
            potr_batch_destroy(b);
            return st;
        }
    }
    *out = b;
    return POTR_OK;
}

potr_status potr_batch_workspace_size(potr_batch b, size_t* bytes) {
    if (!b || !bytes) return fail(POTR_EINVAL, "NULL argument");
    *bytes = b->bytes;
    return POTR_OK;
}

potr_status potr_batch_pairs(potr_batch b, int64_t* counted, int64_t* capacity) {
    if (!b) return fail(POTR_EINVAL, "NULL batch");
    for (size_t j = 0; j < b->jobs.size(); ++j) {
        if (counted) counted[j] = b->counted[j];
        if (capacity) capacity[j] = b->capacity[j];
    }
    return POTR_OK;
}

potr_status potr_batch_bind(potr_batch b, void* ws, size_t ws_bytes, void* stream) {
    if (!b || !ws) return fail(POTR_EINVAL, "NULL argument");
    if (ws_bytes < b->bytes) return fail(POTR_ECAPACITY, "batch workspace %zu < %zu bytes", ws_bytes, b->bytes);
    b->ws = (char*)ws;
    std::vector<ViewJob> table;
    std::vector<int64_t> prefix(1, 0);
    // The render pulls items in table order, so the jobs go in by decreasing
    // mean pairs per tile (the counts of the plan): the costliest tiles are
    // taken first and the last items drawn, which set the launch's tail, are
    // the cheapest ones (longest processing time first, per job).
    std::vector<size_t> order(b->jobs.size());
    std::vector<double> cost(b->jobs.size());
    for (size_t j = 0; j < b->jobs.size(); ++j) {
        order[j] = j;
        const double items = (double)b->jobs[j].V * (double)tiles_of(b->cams[j][0], b->cfg);
        cost[j] = items > 0.0 ? (double)b->counted[j] / items : 0.0;
    }
    std::stable_sort(order.begin(), order.end(), [&](size_t x, size_t y) { return cost[x] > cost[y]; });
    for (size_t j : order) {
        const potr_job& J = b->jobs[j];
        const potr_camera& c0 = b->cams[j][0];
        const int T = tiles_of(c0, b->cfg);
        for (int32_t v = 0; v < J.V; ++v) {
            ViewJob vj{};
            vj.proj = (const potr_proj*)(b->ws + b->off[j].proj) + (int64_t)v * J.N;
            vj.ids = (const uint32_t*)(b->ws + b->off[j].ids);
            vj.ranges = (const int32_t*)(b->ws + b->off[j].ranges) + (int64_t)v * T * 2;
            vj.W = c0.width;
            vj.H = c0.height;
            vj.tiles_x = tiles_x(c0, b->cfg);
            vj.tiles = T;
            vj.target = J.target ? J.target + (int64_t)v * c0.width * c0.height * 3 : nullptr;
            set_outputs(vj, J.out, J.N, v);
            table.push_back(vj);
            prefix.push_back(prefix.back() + (J.N > 0 && has_output(J) ? T : 0));   // no items without outputs
        }
    }
    if (prefix.back() >= (int64_t(1) << 40))
        return fail(POTR_EINVAL, "%lld (view, tile) items in one batch", (long long)prefix.back());
    b->n_items = prefix.back();
    hipStream_t s = (hipStream_t)stream;
    potr_status st = hip_ok(hipMemcpyAsync(b->ws + b->off_table, table.data(), table.size() * sizeof(ViewJob),
                                           hipMemcpyHostToDevice, s), "upload job table");
    if (st == POTR_OK)
        st = hip_ok(hipMemcpyAsync(b->ws + b->off_prefix, prefix.data(), prefix.size() * 8, hipMemcpyHostToDevice, s),
                    "upload prefix");
    if (st == POTR_OK)
        st = hip_ok(hipMemcpyAsync(b->ws + b->off_caps, b->capacity.data(), b->capacity.size() * 8,
                                   hipMemcpyHostToDevice, s), "upload capacities");
    if (st == POTR_OK) st = hip_ok(hipStreamSynchronize(s), "sync");
    return st;
}

potr_status potr_batch_run(potr_batch b, void* stream) {
    if (!b || !b->ws) return fail(POTR_EINVAL, "batch not bound to a workspace");
    hipStream_t s = (hipStream_t)stream;
    char* ws = b->ws;
    int64_t* npairs = (int64_t*)(ws + b->off_npairs);
    // fork: every lane starts after what the caller enqueued before this run
    if (!b->lane_s.empty()) {
        potr_status st = hip_ok(hipEventRecord(b->lane_ev[0], s), "fork record");
        for (size_t l = 0; l < b->lane_s.size() && st == POTR_OK; ++l)
            st = hip_ok(hipStreamWaitEvent(b->lane_s[l], b->lane_ev[0], 0), "fork wait");
        if (st != POTR_OK) return st;
    }
    for (size_t j = 0; j < b->jobs.size(); ++j) {
        const potr_job& J = b->jobs[j];
        const potr_camera* cams = b->cams[j].data();
        potr_proj* proj = (potr_proj*)(ws + b->off[j].proj);
        const size_t lane = b->lane_of[j];
        const auto& L = b->lane_off[lane];
        const hipStream_t ls = b->lane_s.empty() ? s : b->lane_s[lane];
        uint32_t* order = (uint32_t*)(ws + L.order);
        uint32_t* ids = (uint32_t*)(ws + b->off[j].ids);
        int32_t* ranges = (int32_t*)(ws + b->off[j].ranges);
        // the projection also writes the bin's depth keys and rects
        const BinKeys bk = bin_keys(J.N, J.V, cams[0], b->cfg, ws + L.bin);
        potr_status st =
            launch_project(J.N, J.V, cams, b->cfg, J.means, J.scales, J.quats, J.opac, J.sh, proj, nullptr, ls, &bk);
        if (st == POTR_OK)
            st = launch_bin(J.N, J.V, cams[0], b->cfg, proj, ws + L.bin, order, npairs + j, ls, true);
        if (st == POTR_OK)
            st = launch_sort(J.N, J.V, cams[0], b->cfg, proj, order, ws + L.bin, npairs + j, b->capacity[j],
                             ws + L.stage, ids, ranges, ls);
        if (st == POTR_OK && has_step(J) && J.N > 0) {
            // the fine-tuning step: composite, L1 loss gradient (in place of the
            // image), screen-space then parameter gradients
            const int64_t P = (int64_t)cams[0].width * cams[0].height, VP = (int64_t)J.V * P;
            float* img = (float*)(ws + L.pix);
            float* pf = img + 3 * VP;
            float* tf = pf + 3 * VP;
            int32_t* nw = (int32_t*)(tf + VP);
            float* g2d = (float*)(ws + L.g2d);
            st = launch_blend(J.N, J.V, cams[0], b->cfg, proj, ids, ranges, img, pf, tf, nw, nullptr, ls);
            if (st == POTR_OK) st = launch_l1_grad(img, J.grad_target, 3 * VP, J.grad_weight, img, ls);
            if (st == POTR_OK) st = launch_zero(g2d, (int64_t)J.V * J.N * 9, ls);
            if (st == POTR_OK)
                st = launch_blend_backward(J.N, J.V, cams[0], b->cfg, proj, ids, ranges, pf, tf, nw, img, g2d, ls);
            if (st == POTR_OK)
                st = launch_project_backward(J.N, J.V, cams, b->cfg, J.means, J.scales, J.quats, J.opac, J.sh, g2d,
                                             J.d_means, J.d_scales, J.d_quats, J.d_opac, J.d_sh, ls);
        }
        if (st != POTR_OK) return st;
    }
    // join: the render waits for every lane
    for (size_t l = 0; l < b->lane_s.size(); ++l) {
        potr_status st = hip_ok(hipEventRecord(b->lane_ev[1 + l], b->lane_s[l]), "join record");
        if (st == POTR_OK) st = hip_ok(hipStreamWaitEvent(s, b->lane_ev[1 + l], 0), "join wait");
        if (st != POTR_OK) return st;
    }
    if (b->n_items > 0) {
        potr_status st = launch_render_score_persistent((const ViewJob*)(ws + b->off_table), b->n_view_jobs,
                                                        (const int64_t*)(ws + b->off_prefix),
                                                        (int64_t*)(ws + b->off_counter), b->grid, b->cfg,
                                                        b->with_se, b->n_out, b->fixed, s);
        if (st != POTR_OK) return st;
    }
    return launch_check_overflow(npairs, (const int64_t*)(ws + b->off_caps), (int32_t)b->jobs.size(),
                                 (int32_t*)(ws + b->off_flag), s);
}

potr_status potr_batch_render(potr_batch b, void* stream) {
    if (!b || !b->ws) return fail(POTR_EINVAL, "batch not bound to a workspace");
    char* ws = b->ws;
    if (b->n_items == 0) return POTR_OK;   // no job asks for outputs
    return launch_render_score_persistent((const ViewJob*)(ws + b->off_table), b->n_view_jobs,
                                          (const int64_t*)(ws + b->off_prefix), (int64_t*)(ws + b->off_counter),
                                          b->grid, b->cfg, b->with_se, b->n_out, b->fixed, (hipStream_t)stream);
}

potr_status potr_batch_capture(potr_batch b, void* stream) {
    if (!b || !b->ws) return fail(POTR_EINVAL, "batch not bound to a workspace");
    if (!stream) return fail(POTR_EINVAL, "capture needs a stream other than the null stream");
    hipStream_t s = (hipStream_t)stream;
    if (b->exec) { (void)hipGraphExecDestroy(b->exec); b->exec = nullptr; }
    if (b->graph) { (void)hipGraphDestroy(b->graph); b->graph = nullptr; }
    potr_status st = hip_ok(hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal), "begin capture");
    if (st != POTR_OK) return st;
    const potr_status run = potr_batch_run(b, stream);
    hipGraph_t g = nullptr;
    st = hip_ok(hipStreamEndCapture(s, &g), "end capture");
    if (run != POTR_OK) {
        if (g) (void)hipGraphDestroy(g);
        return run;
    }
    if (st != POTR_OK) return st;
    b->graph = g;
    return hip_ok(hipGraphInstantiate(&b->exec, g, nullptr, nullptr, 0), "graph instantiate");
}

potr_status potr_batch_replay(potr_batch b, void* stream) {
    if (!b || !b->exec) return fail(POTR_EINVAL, "no captured graph");
    return hip_ok(hipGraphLaunch(b->exec, (hipStream_t)stream), "graph launch");
}

potr_status potr_batch_overflow(potr_batch b, int32_t* n_overflowed, void* stream) {
    if (!b || !b->ws || !n_overflowed) return fail(POTR_EINVAL, "NULL argument");
    hipStream_t s = (hipStream_t)stream;
    potr_status st = hip_ok(hipMemcpyAsync(n_overflowed, b->ws + b->off_flag, 4, hipMemcpyDeviceToHost, s), "copy");
    if (st == POTR_OK) st = hip_ok(hipStreamSynchronize(s), "sync");
    return st;
}

potr_status potr_batch_destroy(potr_batch b) {
    if (!b) return POTR_OK;
    // teardown: nothing to report on failure
    if (b->exec) (void)hipGraphExecDestroy(b->exec);
    if (b->graph) (void)hipGraphDestroy(b->graph);
    for (hipStream_t ls : b->lane_s) {
        (void)hipStreamSynchronize(ls);
        (void)hipStreamDestroy(ls);
    }
    for (hipEvent_t ev : b->lane_ev) (void)hipEventDestroy(ev);
    delete b;
    return POTR_OK;
}

}  // extern "C"

// ---------------------------------------------------------------- autotuner
// Times every built tile shape with every LDS batch size on the given jobs and
// writes the fastest into *inout. Each candidate plans its own batch (pair
// counts depend on the tile shape) in temporary device memory; scores go to
// scratch buffers and fine-tuning steps are left out, so the caller's outputs
// are untouched.
extern "C" potr_status potr_autotune(const potr_job* jobs, int32_t n_jobs, potr_config* inout, int32_t reps,
                                     double* best_ms, potr_config* tried, double* tried_ms, int32_t* n_tried,
                                     void* stream) {
    if (!inout) return fail(POTR_EINVAL, "NULL config");
    potr_status st = validate_jobs(jobs, n_jobs, false);
    if (st != POTR_OK) return st;
    if (reps < 1) reps = 3;
    hipStream_t s = (hipStream_t)stream;
    // scratch outputs of the jobs' shapes (a job without outputs gets scores)
    std::vector<potr_job> scratch(jobs, jobs + n_jobs);
    std::vector<float*> bufs;
    for (auto& J : scratch) {
        J.grad_target = nullptr;   // the tuner times the scoring only; caller gradients stay untouched
        if (!has_output(J)) {
            J.out.scores = reinterpret_cast<float*>(1);
            J.out.scores_stride = 0;
            J.out.scores_weight = 1.f;
        }
        float** outs[3] = {&J.out.scores, &J.out.scores_se, &J.out.importance};
        const int64_t strides[3] = {J.out.scores_stride, J.out.se_stride, J.out.importance_stride};
        for (int o = 0; o < 3 && st == POTR_OK; ++o) {
            if (!*outs[o]) continue;
            const int64_t n = strides[o] > 0 ? (int64_t)(J.V - 1) * strides[o] + J.N : J.N;
            float* p = nullptr;
            // 8 bytes per element: room for fixed-point outputs too
            st = hip_ok(hipMalloc(&p, (size_t)(n > 0 ? n : 1) * 8), "hipMalloc (scratch outputs)");
            if (st != POTR_OK) break;
            bufs.push_back(p);
            *outs[o] = p;
        }
        if (st != POTR_OK) break;
    }
    const int shapes[3][2] = {{16, 16}, {8, 8}, {32, 8}};
    const int batches[4] = {64, 128, 320, 512};
    double best = 1e300;
    potr_config best_cfg = *inout;
    int32_t k = 0;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    if (st == POTR_OK) st = hip_ok(hipEventCreate(&e0), "event");
    if (st == POTR_OK) st = hip_ok(hipEventCreate(&e1), "event");
    for (int sh = 0; sh < 3 && st == POTR_OK; ++sh) {
        for (int bi = 0; bi < 4 && st == POTR_OK; ++bi) {
            potr_config c = *inout;
            c.tile_w = shapes[sh][0];
            c.tile_h = shapes[sh][1];
            c.lds_batch = batches[bi];
            potr_batch b = nullptr;
            st = potr_batch_create(scratch.data(), n_jobs, &c, 0.05f, &b, stream);
            if (st == POTR_EINVAL) {   // a job's pairs exceed one call's limit at this shape: not a candidate
                st = POTR_OK;
                continue;
            }
            if (st != POTR_OK) break;
            char* ws = nullptr;
            st = hip_ok(hipMalloc(&ws, b->bytes), "hipMalloc (autotune workspace)");
            if (st == POTR_OK) st = potr_batch_bind(b, ws, b->bytes, stream);
            if (st == POTR_OK) st = potr_batch_run(b, stream);       // warm-up
            float ms = 0.f;
            if (st == POTR_OK) st = hip_ok(hipEventRecord(e0, s), "event record");
            for (int r = 0; r < reps && st == POTR_OK; ++r) st = potr_batch_run(b, stream);
            if (st == POTR_OK) st = hip_ok(hipEventRecord(e1, s), "event record");
            if (st == POTR_OK) st = hip_ok(hipEventSynchronize(e1), "event sync");
            if (st == POTR_OK) st = hip_ok(hipEventElapsedTime(&ms, e0, e1), "elapsed");
            if (ws) (void)hipFree(ws);
            potr_batch_destroy(b);
            if (st != POTR_OK) break;
            const double per = ms / reps;
            if (tried) tried[k] = c;
            if (tried_ms) tried_ms[k] = per;
            ++k;
            if (per < best) {
                best = per;
                best_cfg = c;
            }
        }
    }
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    for (float* p : bufs) (void)hipFree(p);
    if (n_tried) *n_tried = k;
    if (st != POTR_OK) return st;
    if (k == 0) return fail(POTR_EINVAL, "no candidate fits: a job's pairs exceed one call's limit at every shape");
    inout->tile_w = best_cfg.tile_w;
    inout->tile_h = best_cfg.tile_h;
    inout->lds_batch = best_cfg.lds_batch;
    if (best_ms) *best_ms = best;
    return POTR_OK;
}
