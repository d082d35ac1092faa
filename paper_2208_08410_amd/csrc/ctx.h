// Context object and host helpers shared by the C-ABI translation units.
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include <string>

#include "../../include/tsvd.h"

struct tsvd_ctx {
  int device = 0;
  int num_cu = 0;
  size_t max_lds = 0;
  std::string last_error;
  void* ws = nullptr;
  size_t ws_bytes = 0;
  hipEvent_t ev[4] = {nullptr, nullptr, nullptr, nullptr};
  hipStream_t copy_stream = nullptr;  // host->device batch copies (pinned-host input)
  tsvd_tuning tuning = {};
};

namespace tsvd {

// record a failure message on the context and return `st`
tsvd_status fail(tsvd_ctx* ctx, tsvd_status st, const char* fmt, ...);
// map an internal return code (0, TSVD_ERR_HIP or other) to a status
tsvd_status from_internal(tsvd_ctx* ctx, int rc, const char* where);
// grow-only device workspace of the context; fails with OUT_OF_MEMORY past `budget` (0 = none)
tsvd_status ensure_ws(tsvd_ctx* ctx, size_t bytes, int64_t budget);
int gram_mode(int32_t gram, int32_t dtype);
tsvd_status check_mode(tsvd_ctx* ctx, int mode, int32_t dtype);
bool right_side(int64_t m, int64_t n, int32_t branch);

// carves 256-byte aligned pieces out of a workspace
struct Bump {
  char* base;
  size_t off = 0;
  size_t cap;
  explicit Bump(void* b, size_t c) : base((char*)b), cap(c) {}
  void* take(size_t bytes) {
    off = (off + 255) & ~(size_t)255;
    void* p = base + off;
    off += bytes;
    return p;
  }
};

inline size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

}  // namespace tsvd
