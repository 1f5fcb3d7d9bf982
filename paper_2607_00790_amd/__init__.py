"""MI355X (gfx950) library for the weakly singular Burton-Miller Nystrom system
of 2D TE-mode transmission scattering, with a proxy-surface HSS direct solver.

This module is a thin ctypes binding of the C-ABI in include/bmhss.h: the
functions carry the same names and only marshal arguments (torch tensors supply
device memory and the current HIP stream).  Every computation runs in the HIP
kernels of libbmhss.so; if the library is not built, calls raise RuntimeError.
"""
from ._binding import (  # noqa: F401
    BmError,
    Geometry,
    HSS,
    Problem,
    bm_assemble_block,
    bm_assemble_dense,
    bm_assemble_proxy,
    bm_far_field,
    bm_geom_create,
    bm_geom_nodes,
    bm_geom_size,
    bm_matvec,
    bm_matvec_noalloc,
    bm_dense_inverse,
    bm_sketch,
    bm_interp_decomp,
    bm_problem_create,
    bm_problem_create_bodies,
    bm_rhs_plane_wave,
    bm_rhs_incident,
    bm_hss_build,
    bm_hss_solve,
    bm_hss_stats,
    bm_hss_level,
    bm_hss_solve_transpose,
    bm_hss_solve_graph,
    bm_far_field_weights,
    bm_shape_derivative,
    bm_fourier_curve,
    bm_fourier_chain,
    lib_path,
    load,
)
from .shape import backscatter_intensity  # noqa: F401


def __getattr__(name):
    # the torch.autograd.Function subclass, created on first use
    if name == "BackscatterIntensity":
        from .shape import _function_class
        return _function_class()
    raise AttributeError(name)
