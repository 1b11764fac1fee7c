// The Zolo-PD solve on a caller-placed workspace, shared by zolo_pd (the
// handle's arena) and zolo_pd_noalloc (the library's fixed device scratch).
#pragma once

#include <cstddef>

#include "../../include/zolo.h"

namespace zolo {

// Argument checks of zolo_pd (LAPACK-style negative codes); fills *opts
// with the defaults overridden by *opts_in.
int check_pd_args(zolo_handle h, int m, int n, const double* A, int lda, double alpha, double l, int r,
                  const double* Qp, int ldq, const double* H, int ldh, const zolo_opts* opts_in, zolo_opts* opts);
// Bytes of device workspace one solve of m x n with degree r (<= 0: any)
// and these options uses.
size_t workspace_bytes(zolo_handle h, int m, int n, int r, const zolo_opts& opts);
// Writes status into *info (when given) for a return before a solve starts.
int report(zolo_info* info, int status);
// The solve (Algorithm 1 and H) with its workspace at `base`
// (workspace_bytes long, 256-byte aligned); writes *info on every return.
int pd_core(zolo_handle h, char* base, int m, int n, const double* A, int lda, double alpha, double l, int r,
            double* Qp, int ldq, double* H, int ldh, const zolo_opts& opts, zolo_info* info);

}  // namespace zolo
