"""FP64 CPU oracle for the on-the-fly training-data generator.

TEST INFRASTRUCTURE ONLY.  This package is the plain, slow, obviously
correct definition that the HIP path is checked against.  Only the test
suite, the smoke check and the CPU-baseline leg of the benchmark may import
it.  The product path (the HIP library and its Python binding) never imports,
links or executes anything in here, and nothing in here imports the product.
Inputs shared by both sides (the synthetic background, configurations) come
from the seeded input generators, which hold none of the method's arithmetic.

What is computed follows the paper, "Rapid Likelihood Free Inference of
Compact Binary Coalescences using Accelerated Hardware" (AMPLFI), section 3
("Simulations on Accelerated Hardware"): draw binary-black-hole parameters
from the priors of Table 1, generate frequency-domain plus/cross waveforms
(section 3.1), project them onto the detectors, inject them into coloured
Gaussian noise, estimate the noise power spectrum from a background stretch,
whiten, and emit the windows (section 3.2).  Where the paper is silent, the
readings listed in the module docstrings are used.

Every floating-point step runs in IEEE binary64 with NumPy.  Library
primitives used as steps: numpy.fft (rfft/irfft), numpy.linalg.svd.

Parity status per function is stated in each module docstring; functions
whose physics fidelity cannot be checked against an external source here
are marked "parity unpinned" (see waveform.py).
"""

from .rng import philox4x32_10, philox_uniform, philox_uniforms
from .priors import sample_params, PARAM_NAMES
from .detectors import (detector_geometry, antenna_patterns, time_delays,
                        DETECTOR_SITES)
from .waveform import (taylorf2_phase, newtonian_amplitude, imr_form_model,
                       fd_waveform, remnant, ringdown_frequencies)
from .spectral import (welch_psd, interp_psd, whiten, hann_periodic)
from .pipeline import (derived_sizes, project_detectors, inject,
                       generate_sample, generate_batch, fd_grid)

__all__ = [
    "philox4x32_10", "philox_uniform", "philox_uniforms",
    "sample_params", "PARAM_NAMES",
    "detector_geometry", "antenna_patterns", "time_delays", "DETECTOR_SITES",
    "taylorf2_phase", "newtonian_amplitude", "imr_form_model", "fd_waveform",
    "remnant", "ringdown_frequencies",
    "welch_psd", "interp_psd", "whiten", "hann_periodic",
    "derived_sizes", "project_detectors", "inject", "generate_sample",
    "generate_batch", "fd_grid",
]
