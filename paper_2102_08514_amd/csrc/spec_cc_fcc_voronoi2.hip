// Kernels and launchers of the cc_fcc_voronoi2 spline (one translation unit per spline
// type, so the library builds in parallel).
#include "lsp_launch.hip"

LSP_INSTANTIATE(lsp::SplineCcFccVoronoi2)
