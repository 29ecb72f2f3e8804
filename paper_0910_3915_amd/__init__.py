"""MI355X-native two-component Shan-Chen D3Q19 lattice Boltzmann engine with
interacting walls and the contact-angle observable (libscdrop, HIP/gfx950).

The compute path is the C-ABI library ``libscdrop.so`` (include/scdrop.h);
this package only binds it.  PyTorch supplies device memory and streams.
"""
from .binding import (SCD_EDRIFT, SCD_ENONFINITE, SCD_OK, Batch, Lattice, ScdError, check,  # noqa: F401
                      header_symbols, lib, make_ca_cfg, make_params, stream_copy, tile_list,
                      variant_index)
from .grad import ContactAngleFn, GradSetup  # noqa: F401
