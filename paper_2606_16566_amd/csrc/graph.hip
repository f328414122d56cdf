// Capture and replay of a sequence of library calls as one HIP graph: the
// calls of a training or rendering step are recorded once on a stream and
// then launched with a single API call per step.
#include <new>

#include "common.hpp"

struct lgs_graph {
    hipGraph_t graph;
    hipGraphExec_t exec;
};

using namespace lgs;

extern "C" lgs_status lgs_graph_begin(void *stream)
{
    LGS_REQUIRE(stream != nullptr, "lgs_graph_begin: capture needs a created stream, not the null stream");
    LGS_HIP(hipStreamBeginCapture(as_stream(stream), hipStreamCaptureModeThreadLocal));
    return LGS_OK;
}

extern "C" lgs_status lgs_graph_end(void *stream, lgs_graph **out)
{
    LGS_REQUIRE(stream != nullptr && out != nullptr, "lgs_graph_end: null stream or output");
    *out = nullptr;
    hipGraph_t g = nullptr;
    LGS_HIP(hipStreamEndCapture(as_stream(stream), &g));
    hipGraphExec_t e = nullptr;
    const hipError_t err = hipGraphInstantiate(&e, g, nullptr, nullptr, 0);
    if (err != hipSuccess) {
        (void)hipGraphDestroy(g);
        set_error("lgs_graph_end: hipGraphInstantiate: %s", hipGetErrorString(err));
        return LGS_ERR_HIP;
    }
    lgs_graph *h = new (std::nothrow) lgs_graph{g, e};
    if (!h) {
        (void)hipGraphExecDestroy(e);
        (void)hipGraphDestroy(g);
        set_error("lgs_graph_end: out of host memory");
        return LGS_ERR_HIP;
    }
    *out = h;
    return LGS_OK;
}

extern "C" lgs_status lgs_graph_launch(lgs_graph *graph, void *stream)
{
    LGS_REQUIRE(graph != nullptr, "lgs_graph_launch: null graph");
    LGS_HIP(hipGraphLaunch(graph->exec, as_stream(stream)));
    return LGS_OK;
}

extern "C" lgs_status lgs_graph_destroy(lgs_graph *graph)
{
    if (!graph) return LGS_OK;
    const hipError_t a = hipGraphExecDestroy(graph->exec);
    const hipError_t b = hipGraphDestroy(graph->graph);
    delete graph;
    if (a != hipSuccess || b != hipSuccess) {
        set_error("lgs_graph_destroy: %s", hipGetErrorString(a != hipSuccess ? a : b));
        return LGS_ERR_HIP;
    }
    return LGS_OK;
}
