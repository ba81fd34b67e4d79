// Kernels and launchers of the bcc_linear spline (one translation unit per spline
// type, so the library builds in parallel).
#include "lsp_launch.hip"

LSP_INSTANTIATE(lsp::SplineBccLinear)
