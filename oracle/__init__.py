"""Plain FP64 CPU oracle for the RGF transmission path.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path (the HIP library
and its Python binding) may import, call or link anything in this package;
only the test-suite, the smoke check and the benchmark's CPU-baseline leg
use it.  It shares no code with the GPU path: its only common dependency is
the seeded input generator module ``synth``, which holds no transport
arithmetic.
"""
from .rgf_oracle import (  # noqa: F401
    lead_operators,
    sancho_rubio,
    surface_gf_bloch,
    self_energies,
    broadening,
    transmission_dense,
    transmission_block_thomas,
    transmission,
    channel_count,
    band_extrema,
    dyson_residual,
)
from .bias import (  # noqa: F401
    G0,
    shifted_lead,
    transmission_bias,
    fermi,
    landauer_current,
    current,
)
from .kmesh import (  # noqa: F401
    bloch_sum,
    device_at_k,
    transmission_kmesh,
    monkhorst_pack,
)
from .ldos import (  # noqa: F401
    local_dos,
    ldos_dense,
    ldos_layers,
    device_matrix,
)
from .kpm import (  # noqa: F401
    central_matrices,
    jackson,
    states_below,
    fermi_level,
)
from . import kpm  # noqa: F401
