// Host runtime around the kernels: HIP-graph capture of K-pass renders and
// the autotuner of the persistent kernels' launch parameters.
#include <algorithm>
#include <vector>

#include "rcp_internal.hpp"

namespace rcp {

// Record the render into a fresh graph and instantiate it, or update the
// existing executable graph in place when only kernel arguments changed.
//
// The graph renders into its own workspace, allocated before the first
// capture and never grown afterwards, so that no later call on the scene can
// move the buffers the graph's kernels hold.
rcp_status graph_capture(rcp_graph* g) {
    if (!g->capture_stream) RCP_HIP(hipStreamCreateWithFlags(&g->capture_stream, hipStreamNonBlocking));
    if (!g->ws.fixed) {
        // allocations happen here, not in the graph
        rcp_status st = prepare_render(g->scene, g->ws, g->W, g->H, g->K, g->disp.mode, g->capture_stream);
        if (st != RCP_OK) return st;
        RCP_HIP(hipStreamSynchronize(g->capture_stream));
        g->ws.fixed = true;
    }
    RCP_HIP(hipStreamBeginCapture(g->capture_stream, hipStreamCaptureModeThreadLocal));
    rcp_status st = render(g->scene, g->ws, g->cam, g->W, g->H, g->K, g->disp, g->out, g->ids, nullptr, nullptr,
                           nullptr, nullptr, g->capture_stream);
    hipGraph_t graph = nullptr;
    hipError_t ce = hipStreamEndCapture(g->capture_stream, &graph);
    if (st != RCP_OK) {
        if (graph) (void)hipGraphDestroy(graph);
        return st;
    }
    RCP_HIP(ce);
    if (g->exec) {
        hipGraphNode_t err_node = nullptr;
        hipGraphExecUpdateResult res;
        if (hipGraphExecUpdate(g->exec, graph, &err_node, &res) != hipSuccess || res != hipGraphExecUpdateSuccess) {
            (void)hipGetLastError();
            (void)hipGraphExecDestroy(g->exec);
            g->exec = nullptr;
        }
    }
    if (!g->exec) {
        hipError_t e = hipGraphInstantiate(&g->exec, graph, nullptr, nullptr, 0);
        if (e != hipSuccess) {
            (void)hipGraphDestroy(graph);
            return hip_status(e, "hipGraphInstantiate", __FILE__, __LINE__);
        }
    }
    if (g->graph) (void)hipGraphDestroy(g->graph);
    g->graph = graph;
    return RCP_OK;
}

void graph_free(rcp_graph* g) {
    if (g->exec) (void)hipGraphExecDestroy(g->exec);
    if (g->graph) (void)hipGraphDestroy(g->graph);
    g->ws.fixed = false;
    free_workspace(g->ws, g->capture_stream);
    if (g->capture_stream) {
        (void)hipStreamSynchronize(g->capture_stream);
        (void)hipStreamDestroy(g->capture_stream);
    }
    delete g;
}

namespace {

// Median of `repeats` timed runs of one workload (after one untimed run,
// which also sizes any buffer it needs).
template <class Run>
rcp_status time_runs(Run&& run, int repeats, hipStream_t stream, hipEvent_t e0, hipEvent_t e1, float& ms) {
    rcp_status st = run();
    if (st != RCP_OK) return st;
    std::vector<float> t;
    for (int r = 0; r < repeats; ++r) {
        RCP_HIP(hipEventRecord(e0, stream));
        st = run();
        if (st != RCP_OK) return st;
        RCP_HIP(hipEventRecord(e1, stream));
        RCP_HIP(hipEventSynchronize(e1));
        float x = 0.0f;
        RCP_HIP(hipEventElapsedTime(&x, e0, e1));
        t.push_back(x);
    }
    std::sort(t.begin(), t.end());
    ms = t[t.size() / 2];
    return RCP_OK;
}

// Coordinate descent over the launch parameters: each round tries every
// candidate of one parameter with the others fixed and keeps the fastest.
// The parameters: refill threshold, early-exit lanes, workgroups per CU,
// tile width, engine and tile order (single renders only; batches always run
// the chain engine in screen order), LDS-staged tree levels, LDS stack depth
// and workgroup size (the last two select among instantiations of the chain
// kernel).
template <class Run>
rcp_status descend(rcp_scene* s, Run&& run, bool tune_engine, int repeats, Tuning& best, float& best_ms,
                   hipStream_t stream) {
    hipEvent_t e0, e1;
    RCP_HIP(hipEventCreate(&e0));
    RCP_HIP(hipEventCreate(&e1));
    struct EvGuard { hipEvent_t a, b; ~EvGuard() { (void)hipEventDestroy(a); (void)hipEventDestroy(b); } } g{e0, e1};
    const std::vector<int> refill = {40, 48, 52, 56, 60, 64};
    const std::vector<int> exits = {4, 8, 12, 16, 24, 64};
    const std::vector<int> blocks = {0, 4, 3, 2};
    const std::vector<int> tiles = {3, 4, 2, 5};
    const std::vector<int> engines = {RCP_ENGINE_CHAIN, RCP_ENGINE_PASSES};
    const std::vector<int> top_levels = {4, 3, 2, 0};
    const std::vector<int> stacks = {16, 8};
    const std::vector<int> blocks_sz = {256, 512};
    const std::vector<int> orders = {1, 0};
    // start from the parameters the launches use now (defaults made explicit)
    Tuning cur = s->tuning;
    {
        const Launch l = launch_params(s, tune_engine && chain_ordered(s));
        cur.refill_min = l.refill_min;
        cur.exit_lanes = l.exit_lanes;
    }
    s->tuning = cur;
    float cur_ms = 0.0f;
    rcp_status st = time_runs(run, repeats, stream, e0, e1, cur_ms);
    if (st != RCP_OK) return st;
    for (int round = 0; round < 2; ++round) {
        for (int param = 0; param < 9; ++param) {
            if ((param == 4 || param == 8) && !tune_engine) continue;
            const std::vector<int>& cands = param == 0   ? refill
                                            : param == 1 ? exits
                                            : param == 2 ? blocks
                                            : param == 3 ? tiles
                                            : param == 4 ? engines
                                            : param == 5 ? top_levels
                                            : param == 6 ? stacks
                                            : param == 7 ? blocks_sz
                                                         : orders;
            for (int c : cands) {
                Tuning t = cur;
                int& field = param == 0   ? t.refill_min
                             : param == 1 ? t.exit_lanes
                             : param == 2 ? t.blocks_per_cu
                             : param == 3 ? t.tile_log2w
                             : param == 4 ? t.engine
                             : param == 5 ? t.top_levels
                             : param == 6 ? t.stack
                             : param == 7 ? t.block
                                          : t.tile_order;
                if (field == c) continue;
                field = c;
                s->tuning = t;
                float ms = 0.0f;
                st = time_runs(run, repeats, stream, e0, e1, ms);
                if (st != RCP_OK) { s->tuning = cur; return st; }
                if (ms < cur_ms) { cur = t; cur_ms = ms; }
            }
            s->tuning = cur;
        }
    }
    best = cur;
    best_ms = cur_ms;
    s->tuning = cur;
    // leave a result made with the chosen parameters in the outputs
    st = run();
    if (st != RCP_OK) return st;
    RCP_HIP(hipStreamSynchronize(stream));
    return take_device_error(s);
}

}  // namespace

rcp_status autotune(rcp_scene* s, const Camera& cam, int W, int H, int K, const Disp& d, float* out, int32_t* ids,
                    int repeats, Tuning& best, float& best_ms, hipStream_t stream) {
    auto run = [&]() -> rcp_status {
        return render(s, s->ws, cam, W, H, K, d, out, ids, nullptr, nullptr, nullptr, nullptr, stream);
    };
    return descend(s, run, true, repeats, best, best_ms, stream);
}

rcp_status autotune_batch(rcp_scene* s, const rcp_view* views, int n_views, int repeats, Tuning& best,
                          float& best_ms, hipStream_t stream) {
    auto run = [&]() -> rcp_status { return render_batch(s, views, n_views, s->bws, stream); };
    return descend(s, run, false, repeats, best, best_ms, stream);
}

}  // namespace rcp
