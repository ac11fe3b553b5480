// HIP graph capture of launch sequences: any run of enqueue-only entry points (rank, rank4,
// quadfm_count, quadfm_count_ws, quadfm_count_batched) issued between qr_graph_begin and
// qr_graph_end on one stream is recorded once and replayed with a single launch.  None of those
// entry points records a memset, a host synchronisation or an allocation, so they are capturable.
#include <new>

#include "common.hpp"

using qr::set_error;

struct qr_graph_s {
    hipGraph_t graph;
    hipGraphExec_t exec;
};

extern "C" {

int qr_graph_begin(hipStream_t stream) {
    if (!stream) {
        set_error("qr_graph_begin: capture needs a non-null stream");
        return QR_EINVAL;
    }
    QR_HIP(hipStreamBeginCapture(stream, hipStreamCaptureModeThreadLocal));
    return QR_OK;
}

int qr_graph_end(hipStream_t stream, qr_graph *out) {
    if (!out) return QR_EINVAL;
    *out = nullptr;
    hipGraph_t g = nullptr;
    QR_HIP(hipStreamEndCapture(stream, &g));
    qr_graph_s *h = new (std::nothrow) qr_graph_s{g, nullptr};
    if (!h) {
        (void)hipGraphDestroy(g);
        return QR_ENOMEM;
    }
    hipError_t e = hipGraphInstantiate(&h->exec, g, nullptr, nullptr, 0);
    if (e != hipSuccess) {
        set_error("hipGraphInstantiate: %s", hipGetErrorString(e));
        (void)hipGraphDestroy(g);
        delete h;
        return QR_EHIP;
    }
    *out = h;
    return QR_OK;
}

int qr_graph_launch(qr_graph g, hipStream_t stream) {
    if (!g) return QR_EINVAL;
    QR_HIP(hipGraphLaunch(g->exec, stream));
    return QR_OK;
}

int qr_graph_free(qr_graph g) {
    if (!g) return QR_OK;
    if (g->exec) (void)hipGraphExecDestroy(g->exec);
    if (g->graph) (void)hipGraphDestroy(g->graph);
    delete g;
    return QR_OK;
}

}  // extern "C"
