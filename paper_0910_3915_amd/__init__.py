"""MI355X-native two-component Shan-Chen D3Q19 lattice Boltzmann engine with
interacting walls and the contact-angle observable (libscdrop, HIP/gfx950).

The compute path is the C-ABI library ``libscdrop.so`` (include/scdrop.h);
this package only binds it.  PyTorch supplies device memory and streams.
"""
from .binding import (Batch, Lattice, ScdError, check, header_symbols, lib,  # noqa: F401
                      make_ca_cfg, make_params, stream_copy, tile_list, variant_index)
from .grad import ContactAngleFn, GradSetup  # noqa: F401
