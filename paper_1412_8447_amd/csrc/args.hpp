// Argument checks of the C ABI (include/idcur.h), free of any GPU call: the
// library runs them before it sizes the workspace or enqueues anything, and the
// CPU tests build this file alone (with the address and undefined-behaviour
// sanitizers) to drive every error code.
#pragma once

#include <stdint.h>

#include "../../include/idcur.h"

namespace idcur {

constexpr int kMaxRank = 4096;       // largest k (and k + p): bounds the k x k FP64 work buffers
constexpr int kSrhtMaxRowsArg = 512;  // sampled rows of the structured sketch

enum Op { OP_COL = 0, OP_ROW = 1, OP_TWO = 2, OP_CUR = 3, OP_SKETCH = 4, OP_SKETCH_ROW = 5 };

// Output arrays of one call (device pointers, leading dimensions in elements).
struct Outs {
  int* k_out = nullptr;
  int* J = nullptr; void* T = nullptr; int64_t ldt = 0;
  int* I = nullptr; void* Tr = nullptr; int64_t ldtr = 0;
  void* U = nullptr; int64_t ldu = 0;
  void* C = nullptr; int64_t ldc = 0;
  void* R = nullptr; int64_t ldr = 0;
  void* Yt = nullptr; int64_t ldy = 0;
};

// code IDCUR_OK with msg null, or the error code and its message (a literal)
struct ArgCheck {
  idcur_status code;
  const char* msg;
};

// sizes, types and options of a dense ID / CUR / sketch call
ArgCheck check_id_args(int op, int dtype, int64_t m, int64_t n, int64_t lda, const idcur_opts* opts);
// the input pointer and the output arrays that op writes (after check_id_args)
ArgCheck check_id_outs(int op, int64_t m, int64_t n, const void* A, const idcur_opts& opts, const Outs& out);
// sizes and options of a batched ID call; max_width and max_sketch are the
// batched kernel's limits on a block's columns and on k (kmax) + p
ArgCheck check_batched_args(int dtype, int nblk, int mmax, int nmax, const idcur_opts* o, int max_width,
                            int max_sketch);

}  // namespace idcur
