// Stream capture of FC calls into HIP graphs (host code).
//
// Every call of the library is a fixed sequence of kernel launches, fills
// and event fork/joins on the caller's stream with no allocation and no host
// synchronisation, so any sequence of calls (several plans, TX and RX) can
// be recorded once and replayed with one launch. Buffers and plans are
// captured by address: they must outlive the graph; weights set later with
// fc_set_weights* are seen by later replays (the kernels read the plan's
// weight table when they run).
#include <hip/hip_runtime.h>

#include "fc.h"

struct fc_graph {
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
};

extern "C" {

fc_status fc_graph_begin(void* stream) {
  if (!stream) return FC_E_ARG;      // the legacy null stream cannot be captured
  return hipStreamBeginCapture((hipStream_t)stream, hipStreamCaptureModeThreadLocal) == hipSuccess
             ? FC_OK : FC_E_DEVICE;
}

fc_status fc_graph_end(void* stream, fc_graph** out) {
  if (!stream || !out) return FC_E_ARG;
  *out = nullptr;
  fc_graph* g = new fc_graph();
  if (hipStreamEndCapture((hipStream_t)stream, &g->graph) != hipSuccess || !g->graph) {
    delete g;
    return FC_E_DEVICE;
  }
  if (hipGraphInstantiate(&g->exec, g->graph, nullptr, nullptr, 0) != hipSuccess) {
    (void)hipGraphDestroy(g->graph);
    delete g;
    return FC_E_DEVICE;
  }
  *out = g;
  return FC_OK;
}

fc_status fc_graph_launch(fc_graph* g, void* stream) {
  if (!g || !g->exec) return FC_E_ARG;
  return hipGraphLaunch(g->exec, (hipStream_t)stream) == hipSuccess ? FC_OK : FC_E_DEVICE;
}

void fc_graph_destroy(fc_graph* g) {
  if (!g) return;
  if (g->exec) (void)hipGraphExecDestroy(g->exec);
  if (g->graph) (void)hipGraphDestroy(g->graph);
  delete g;
}

}  // extern "C"
