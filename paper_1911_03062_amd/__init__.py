"""MI355X-native npFEM deformable-cell solver: C-ABI library (libnpfem.so) with hand-written
HIP kernels for gfx950, and its Python binding."""
from .npfem import (CellType, Batch, NpfemError, lib, header_symbols, make_cell_types, STATUS,
                    FORMS)
