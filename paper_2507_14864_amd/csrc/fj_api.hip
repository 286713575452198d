// C ABI: error reporting and graph entry points.
#include <string>

#include "fj_internal.h"

namespace fj {
namespace {
thread_local std::string g_last_error;
}
void set_error(const std::string& msg) { g_last_error = msg; }
const char* last_error() { return g_last_error.c_str(); }
fj_status hip_fail(hipError_t e, const char* what) {
    set_error(std::string("HIP error ") + hipGetErrorName(e) + " (" + hipGetErrorString(e) + ") in " + what);
    return FJ_ERR_HIP;
}
}  // namespace fj

using namespace fj;

extern "C" const char* fj_last_error(void) { return last_error(); }

extern "C" int32_t fj_version(void) { return 1; }

static bool desc_ok(const fj_graph_desc* d) {
    if (!d) return false;
    if (d->n < 0 || d->nnz < 0 || d->n >= (int64_t(1) << 31) - 1 || d->nnz >= (int64_t(1) << 31) - 1) return false;
    if (!d->row_ptr) return false;
    if (d->nnz > 0 && !d->col) return false;
    return true;
}

extern "C" size_t fj_graph_workspace_bytes(const fj_graph_desc* desc, int32_t flags) {
    if (!desc_ok(desc)) return 0;
    return graph_ws_bytes(desc, flags);
}

extern "C" fj_status fj_graph_create(const fj_graph_desc* desc, int32_t flags, void* ws, size_t ws_bytes,
                                     void* stream, fj_graph** out) {
    if (!out) {
        set_error("fj_graph_create: out is NULL");
        return FJ_ERR_INVALID_ARGUMENT;
    }
    if (!desc_ok(desc)) {
        set_error("fj_graph_create: invalid descriptor (need 0 <= n, nnz < 2^31 - 1 and non-NULL arrays)");
        return FJ_ERR_INVALID_ARGUMENT;
    }
    if (flags & ~FJ_GRAPH_COLOUR) {
        set_error("fj_graph_create: unknown flags");
        return FJ_ERR_INVALID_ARGUMENT;
    }
    if (!ws && graph_ws_bytes(desc, flags) > 0) {
        set_error("fj_graph_create: workspace is NULL");
        return FJ_ERR_INVALID_ARGUMENT;
    }
    if (reinterpret_cast<uintptr_t>(ws) % 256 != 0) {
        set_error("fj_graph_create: workspace must be 256-byte aligned");
        return FJ_ERR_INVALID_ARGUMENT;
    }
    fj_graph* g = new (std::nothrow) fj_graph();
    if (!g) {
        set_error("fj_graph_create: host allocation failed");
        return FJ_ERR_INVALID_ARGUMENT;
    }
    fj_status rc = graph_build(g, desc, flags, ws, ws_bytes, static_cast<hipStream_t>(stream));
    if (rc != FJ_OK) {
        delete g;
        return rc;
    }
    *out = g;
    return FJ_OK;
}

extern "C" fj_status fj_graph_destroy(fj_graph* g) {
    delete g;
    return FJ_OK;
}

extern "C" fj_status fj_graph_get_info(const fj_graph* g, fj_graph_info* out) {
    if (!g || !out) {
        set_error("fj_graph_get_info: null argument");
        return FJ_ERR_INVALID_ARGUMENT;
    }
    out->n = g->n;
    out->nnz = g->nnz;
    out->directed = g->directed;
    out->weighted = g->weighted;
    out->max_degree = g->max_degree;
    out->max_in_degree = g->max_in_degree;
    out->num_colours = g->num_colours;
    out->colour_rounds = g->colour_rounds;
    return FJ_OK;
}

extern "C" fj_status fj_graph_colour_sizes(const fj_graph* g, int64_t* sizes) {
    if (!g || !sizes || g->num_colours == 0) {
        set_error("fj_graph_colour_sizes: null argument or graph without colouring");
        return FJ_ERR_INVALID_ARGUMENT;
    }
    for (int k = 0; k < g->num_colours; ++k) sizes[k] = g->class_off[k + 1] - g->class_off[k];
    return FJ_OK;
}

extern "C" fj_status fj_graph_colours(const fj_graph* g, int32_t* colours, void* stream) {
    if (!g || !colours || g->num_colours == 0) {
        set_error("fj_graph_colours: null argument or graph without colouring");
        return FJ_ERR_INVALID_ARGUMENT;
    }
    hipStream_t st = static_cast<hipStream_t>(stream);
    FJ_HIP(hipMemcpyAsync(colours, g->colour, sizeof(int32_t) * g->n, hipMemcpyDeviceToDevice, st));
    FJ_HIP(hipStreamSynchronize(st));
    return FJ_OK;
}
