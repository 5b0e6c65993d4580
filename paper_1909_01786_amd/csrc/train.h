// train.h -- host side of the scorer's training (internal).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <string>
#include <vector>

#include "../../include/asp.h"
#include "encode.h"

namespace asp {

int64_t train_nparam();
int32_t train_workspace(const std::vector<const HostProgram*>& progs, uint64_t* bytes);
int32_t train_run(const std::vector<const HostProgram*>& progs, const float* labels, float* params,
                  int32_t steps, float lr, uint8_t* ws, uint64_t ws_bytes, float* loss_out,
                  float* grad_out, hipStream_t s, std::string* err);
void train_quantize(const float* params, asp_scorer_weights* w);
void train_dequantize(const asp_scorer_weights* w, float* params);

}  // namespace asp
