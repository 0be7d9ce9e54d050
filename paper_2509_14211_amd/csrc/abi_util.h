// Internal helpers shared by the C entry points (abi.hip: objects and
// operations; drivers.hip: the iterative drivers): argument checks, the
// recording of operations as runtime nodes, and the error text.
#pragma once

#include <string>

#include "runtime.h"

namespace nbgrb {

// Text returned by GrM_error() for the calling thread.
std::string& api_error();

void need(const void* p, const char* what);
GB_Vector_opaque* vec(GrB_Vector v, const char* what);
GB_Scalar_opaque* sca(GrB_Scalar s, const char* what);
// A pattern (CSR) matrix; a dense one is GrB_INVALID_VALUE.
GB_Matrix_opaque* mat(GrB_Matrix A, const char* what);
// Any matrix handle, pattern or dense.
GB_Matrix_opaque* mat_any(GrB_Matrix A, const char* what);
void no_mask_accum(const void* mask, const void* accum);
void float_type(int t, const char* what);
bool desc_comp(GrB_Descriptor d);
bool desc_struct(GrB_Descriptor d);
bool desc_replace(GrB_Descriptor d);

// Record (nonblocking) or run (blocking) one operation into its output.
NodeP iso_node(int type, int64_t n, double v);
void rec_ewise(GB_Vector_opaque* w, int op, GB_Vector_opaque* u, GB_Vector_opaque* v, bool set_union);
void rec_unop(GB_Vector_opaque* w, int op, GB_Vector_opaque* u);
void rec_bind(GB_Vector_opaque* w, int op, GB_Vector_opaque* u, double k, bool first);
void rec_bind_scalar(GB_Vector_opaque* w, int op, GB_Vector_opaque* u, GB_Scalar_opaque* s);
void rec_mxv(GB_Vector_opaque* w, GB_Matrix_opaque* A, GB_Vector_opaque* u, GB_Vector_opaque* mask,
             GrB_Descriptor desc);
void rec_assign(GB_Vector_opaque* w, GB_Vector_opaque* mask, double x, GrB_Descriptor desc);
void rec_reduce(GB_Scalar_opaque* s, GB_Vector_opaque* u, GB_Vector_opaque* mask, bool comp, bool watch);
void rec_affine(GB_Scalar_opaque* out, double alpha, GB_Scalar_opaque* in, double beta);
// Give an iso vector storage.
void store_if_iso(const NodeP& v);
MatP new_matdata(int64_t nrows, int64_t ncols);
// out[k] = v[idx[k]] as a new materialised node (iso vectors stay iso).
NodeP permuted(const NodeP& v, const BufP& idx);
// One int from device memory (synchronises).
int read_flag(const BufP& f);

}  // namespace nbgrb

// Entry-point bodies: GrbError and allocation failures become GrB_Info
// codes with their text kept for GrM_error().
#define API_BEGIN \
  try {           \
    nbgrb::api_error().clear();
#define API_END                                      \
  }                                                  \
  catch (const nbgrb::GrbError& e) {                 \
    nbgrb::api_error() = e.msg;                      \
    return e.info;                                   \
  }                                                  \
  catch (const std::bad_alloc&) {                    \
    nbgrb::api_error() = "host allocation failed";   \
    return GrB_OUT_OF_MEMORY;                        \
  }                                                  \
  catch (const std::exception& e) {                  \
    nbgrb::api_error() = e.what();                   \
    return GrB_PANIC;                                \
  }                                                  \
  return GrB_SUCCESS;
