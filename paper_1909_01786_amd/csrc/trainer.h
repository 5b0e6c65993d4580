// trainer.h -- launch interface of the scorer's training kernels (internal).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace asp {

hipError_t tr_mm(const float* X, const float* W, int trans, float* Y, int64_t rows, float alpha,
                 int acc, hipStream_t s);
hipError_t tr_mm_tn(const float* X, const float* D, float* dW, int64_t rows, hipStream_t s);
hipError_t tr_segsum(const int64_t* off, const int32_t* idx, const float* SP, const float* SN,
                     const float* sscale, const float* oscale, float* out, int64_t rows, int acc,
                     hipStream_t s);
hipError_t tr_act_fwd(const float* U, const float* b, float* A, int64_t rows, hipStream_t s);
hipError_t tr_act_bwd(const float* dA, const float* A, float* G, float* db, int64_t rows,
                      hipStream_t s);
hipError_t tr_embed_fwd(const float* X8, const float* E, const float* e, float* A, int64_t rows,
                        hipStream_t s);
hipError_t tr_embed_bwd(const float* X8, const float* G, float* dE, int64_t rows, hipStream_t s);
hipError_t tr_readout(const float* A, const float* y, const float* wo, const float* bo, float* dA,
                      float* dwo, float* dbo, float* loss, int64_t rows, float inv_n,
                      hipStream_t s);
hipError_t tr_adam(float* p, const float* g, float* m, float* v, int64_t n, float lr, int t,
                   const uint8_t* range, const float* lim, hipStream_t s);

}  // namespace asp
