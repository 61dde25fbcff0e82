"""MI355X (gfx950) NPGA mean-variance solver: Python binding of libnpga.

The HIP library ``libnpga.so`` (built in-tree by ``paper_2604_02917_amd/build.py``)
does all the work; this package only marshals torch tensors and the current
HIP stream into the C ABI declared in ``include/npga.h``.  Importing the
package loads the library and raises if it is missing: there is no fallback.
"""
from .api import (  # noqa: F401
    NPGAFunction,
    NpgaError,
    auto_path,
    Options,
    backward,
    batched_tune,
    gradient_batched,
    solve_batched,
    build_factor,
    gradient,
    gradient_noalloc,
    lib_path,
    project,
    project_dykstra,
    sketch_str,
    sketch_str_ex,
    philox_sketch,
    solve,
    spectral_norm_sq,
    syrk,
    to_bf16,
    status_string,
)
