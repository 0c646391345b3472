"""MI355X-native integral-histogram library (gfx950 HIP kernels behind a C ABI).

Integral histograms, O(1) plain and spatially weighted region histograms,
spatial-pyramid descriptors and exhaustive pyramid-distance candidate search,
after Poostchi 2017 (arXiv:1711.01656).  See ``include/ih.h`` for the C ABI
and ``paper_1711_01656_amd.ih`` for the Python binding.
"""
from .ih import (  # noqa: F401
    Batch,
    IHError,
    TileCfg,
    cells,
    ih_build,
    ih_camshift,
    ih_color_likelihood,
    ih_build_moments2,
    ih_build_weighted,
    ih_jih_update,
    ih_local_median,
    ih_match_candidates,
    ih_moment_images,
    ih_profile_events,
    ih_pyramid_desc,
    ih_query_quadratic,
    ih_query_rect,
    ih_query_wedding,
    ih_query_weighted,
    lib,
    lib_path,
    version,
    shape_of,
    workspace_size,
)
