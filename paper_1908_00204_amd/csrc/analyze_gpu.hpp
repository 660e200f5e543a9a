// Relaxed dependency detection (Alg. 4) and levelization on the GPU, with the
// host analysis's results bit for bit (analyze_gpu.hip).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <vector>

namespace glu {

// From the filled pattern (host arrays; uploaded, processed on the current
// device, results copied back): the dependency CSR (dag_ptr[n+1], dag_idx)
// and each column's level.  spin_err is set non-zero if a bounded wait of
// the level sweep gave up (the results are then not valid).
hipError_t gpu_dag_levels(int32_t n, const std::vector<int64_t>& lu_colptr, const std::vector<int32_t>& lu_rowind,
                          const std::vector<int64_t>& diag, std::vector<int64_t>& dag_ptr,
                          std::vector<int32_t>& dag_idx, std::vector<int32_t>& level_of, int32_t* spin_err);

}  // namespace glu
