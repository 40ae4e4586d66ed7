"""Seeded synthetic inputs shared by the oracle and the HIP path (no solver arithmetic)."""
from .silicon import (SiliconSystem, BlockList, make_system, diamond_positions, image_pairs,
                      counter_uniform, random_blocks, batch_cells, displaced_frame, si64_b4, si4096_b9,
                      SMALL_CUTOFFS, BIG_CUTOFFS, A_SI, T_BOND)
