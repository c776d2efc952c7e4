// dg_host.hpp -- host-only declarations of the runtime (not part of the ABI).
#pragma once

#include "dg_internal.hpp"

namespace dg {

// LGL nodes xi[N+1], weights w[N+1] and D[(N+1)^2] (row-major, D[i*(N+1)+j]).
void lgl_operator(int N, double *xi, double *w, double *D);

// Face-point descriptor table of a workgroup tile (4 uint32 per face point).
int face_table_size(int dim, int N, int epb);
void build_face_table(int dim, int N, int epb, uint32_t *tab);

}  // namespace dg
