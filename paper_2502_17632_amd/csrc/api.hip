// C ABI plumbing: errors, stream-ordered allocation, graph info/export/destroy.
#include <cmath>
#include <cstdarg>
#include <cstring>

#include "common.h"

namespace gift {

namespace {
thread_local std::string t_last_error;
}

gift_status set_error(gift_status s, const char *fmt, ...) {
  char buf[1024];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  t_last_error = buf;
  return s;
}

void clear_error() { t_last_error.clear(); }

gift_status check_launch(const char *what) {
  hipError_t e = hipGetLastError();
  if (e != hipSuccess)
    return set_error(GIFT_EDEVICE, "launch of %s failed: %s", what, hipGetErrorString(e));
  return GIFT_OK;
}

gift_status dev_alloc(void **p, size_t bytes, hipStream_t s, const char *what) {
  *p = nullptr;
  if (bytes == 0) bytes = 16;
  hipError_t e = hipMallocAsync(p, bytes, s);
  if (e != hipSuccess) {
    *p = nullptr;
    (void)hipGetLastError();
    return set_error(e == hipErrorOutOfMemory ? GIFT_ENOMEM : GIFT_EDEVICE,
                     "device allocation of %zu bytes for %s failed: %s", bytes, what,
                     hipGetErrorString(e));
  }
  return GIFT_OK;
}

void dev_free(void *p, hipStream_t s) {
  if (p) (void)hipFreeAsync(p, s);
}

const SigmaBlock *find_sigma(const gift_graph *g, double sigma) {
  for (const SigmaBlock &b : g->sig)
    if (b.sigma == sigma) return &b;
  return nullptr;
}

}  // namespace gift

using namespace gift;

extern "C" {

const char *gift_status_string(gift_status s) {
  switch (s) {
    case GIFT_OK: return "GIFT_OK";
    case GIFT_EINVAL: return "GIFT_EINVAL: invalid argument";
    case GIFT_ENOMEM: return "GIFT_ENOMEM: out of memory";
    case GIFT_EDEVICE: return "GIFT_EDEVICE: HIP runtime error";
    case GIFT_EUNSUPPORTED: return "GIFT_EUNSUPPORTED: unsupported combination or size";
    case GIFT_EBUSY: return "GIFT_EBUSY: object in use";
  }
  return "unknown gift_status";
}

const char *gift_last_error(void) { return t_last_error.c_str(); }

int32_t gift_abi_version(void) { return GIFT_ABI_VERSION; }

gift_status gift_graph_get_info(const gift_graph *g, gift_graph_info *info) {
  clear_error();
  if (!g || !info) return set_error(GIFT_EINVAL, "gift_graph_get_info: NULL argument");
  info->num_cells = g->num_cells;
  info->num_virtual = g->num_virtual;
  info->num_rows = g->num_rows;
  info->nnz = g->nnz;
  info->bytes_resident = g->bytes;
  info->storage = g->storage;
  info->num_sigmas = static_cast<int32_t>(g->sig.size());
  return GIFT_OK;
}

gift_status gift_graph_export(const gift_graph *g, int64_t *row_ptr, int32_t *col, double *w,
                              double *deg, void *stream) {
  clear_error();
  if (!g) return set_error(GIFT_EINVAL, "gift_graph_export: NULL graph");
  hipStream_t s = static_cast<hipStream_t>(stream);
  if (row_ptr) {
    std::vector<int32_t> tmp(static_cast<size_t>(g->num_rows + 1));
    GIFT_HIP(hipMemcpyAsync(tmp.data(), g->row_ptr, tmp.size() * 4, hipMemcpyDeviceToHost, s));
    GIFT_HIP(hipStreamSynchronize(s));
    for (size_t i = 0; i < tmp.size(); ++i) row_ptr[i] = tmp[i];
  }
  if (col && g->nnz)
    GIFT_HIP(hipMemcpyAsync(col, g->col, g->nnz * 4, hipMemcpyDeviceToHost, s));
  if (w && g->nnz) GIFT_HIP(hipMemcpyAsync(w, g->w, g->nnz * 8, hipMemcpyDeviceToHost, s));
  if (deg && g->num_rows)
    GIFT_HIP(hipMemcpyAsync(deg, g->deg, g->num_rows * 8, hipMemcpyDeviceToHost, s));
  GIFT_HIP(hipStreamSynchronize(s));
  return GIFT_OK;
}

gift_status gift_destroy_graph(gift_graph *g, void *stream) {
  clear_error();
  if (!g) return GIFT_OK;
  hipStream_t s = static_cast<hipStream_t>(stream);
  dev_free(g->row_ptr, s);
  dev_free(g->col, s);
  dev_free(g->w, s);
  dev_free(g->deg, s);
  dev_free(g->tile_row, s);
  for (SigmaBlock &b : g->sig) {
    dev_free(b.val, s);
    dev_free(b.diag, s);
  }
  delete g;
  return GIFT_OK;
}

}  // extern "C"
