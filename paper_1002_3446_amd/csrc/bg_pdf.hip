// Per-class setup of the inverse-CDF table of the synthetic parton density (one thread per
// segment; the table layout and the interpolant are described at pdf_sample).
#include "bg_kernels.hpp"
#include "bg_launch.hpp"

namespace bgk {

__global__ __launch_bounds__(64) void k_pdf_table(PdfParams P, double* tab) {
  const int seg = blockIdx.x * blockDim.x + threadIdx.x;
  if (seg < kPdfSegs) pdf_table_segment(P, seg, tab + 4 * seg);
}

hipError_t launch_pdf_table(const PdfParams& P, double* tab, hipStream_t s) {
  hipLaunchKernelGGL(k_pdf_table, dim3((kPdfSegs + 63) / 64), dim3(64), 0, s, P, tab);
  return hipGetLastError();
}

}  // namespace bgk
