// Kernels and launchers of the bcc_voronoi1 spline (one translation unit per spline
// type, so the library builds in parallel).
#include "lsp_launch.hip"

LSP_INSTANTIATE(lsp::SplineBccVoronoi1)
