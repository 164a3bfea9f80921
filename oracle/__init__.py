"""FP64 CPU oracle for the tile-based 3D Gaussian Splatting forward render.

TEST INFRASTRUCTURE ONLY.  Nothing on the product path may import or call this
package: only the test-suite, the smoke check of the graft entry point and the
CPU-baseline leg of the benchmark do.  It shares no code with the HIP library;
the seeded input generators in ``workloads`` are the only common module.

The oracle is the algorithm written out step by step in numpy float64, in the
order the paper gives it:

* ``plan``     tile grid and the resolution-adaptive key bit split (Sec. IV-A,
               "Resolution-Adaptive Sorting-Key Encoding", Eq. depth_quant);
* ``quant``    compact attribute storage: INT8 SH with symmetric per-degree,
               per-channel scales (Eq. quant), FP16 rotation/scale/opacity,
               FP32 mean (Sec. IV-A, "Compact Attribute Storage");
* ``project``  EWA projection, frustum/opacity culling, tile extents and SH
               colour (Sec. II-A and III-A, following 3DGS);
* ``tiles``    duplication, 64-bit and 32-bit keys, sort and tile ranges
               (Sec. III-B/C, IV-A);
* ``fastexp``  the range-aware bit-level exponential and its error
               (Sec. IV-B, Eq. fma_exp, Eq. fast_exp_range);
* ``blend``    front-to-back alpha blending per pixel (Eq. alpha_computation,
               Eq. power, Eq. opacity_clamped, Eq. folded_exponent);
* ``render``   the whole frame for the plain and the fast path.

Every function cites the passage it follows.  Readings of passages where the
paper is silent or ambiguous are stated where they are used.
"""
from .plan import TILE, FramePlan, frame_plan, key_bits
from .quant import FastScene, quantize_scene, dequantize_scene, quantize_sh
from .project import Projection, project, sh_basis, LN255
from .tiles import (duplicate, sort_entries, tile_ranges, plain_keys, fast_keys, ellipse_meets_tile,
                    exact_tile_filter, EXACT_TILE_MAX_AREA)
from .fastexp import fast_exp, fast_exp_rel_error, SIGMA
from .blend import blend_tile, BlendResult
from .render import OracleFrame, render, prepare_plain, prepare_fast, prepare_fast_ablated

__all__ = [
    "TILE", "FramePlan", "frame_plan", "key_bits",
    "FastScene", "quantize_scene", "dequantize_scene", "quantize_sh",
    "Projection", "project", "sh_basis", "LN255",
    "duplicate", "sort_entries", "tile_ranges", "plain_keys", "fast_keys",
    "fast_exp", "fast_exp_rel_error", "SIGMA",
    "blend_tile", "BlendResult",
    "OracleFrame", "render", "prepare_plain", "prepare_fast", "prepare_fast_ablated",
]
