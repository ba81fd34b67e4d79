// Kernels and launchers of the d4s_8dir spline (one translation unit per spline
// type, so the library builds in parallel).
#include "lsp_launch.hip"

LSP_INSTANTIATE(lsp::SplineD4s8)
