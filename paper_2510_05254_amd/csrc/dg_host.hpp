// dg_host.hpp -- host-only declarations of the runtime (not part of the ABI).
#pragma once

#include "dg_internal.hpp"

namespace dg {

// LGL nodes xi[N+1], weights w[N+1] and D[(N+1)^2] (row-major, D[i*(N+1)+j]).
void lgl_operator(int N, double *xi, double *w, double *D);

}  // namespace dg
