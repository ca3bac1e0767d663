"""Seeded synthetic inputs shared by the oracle and the GPU path."""
from .scene import (SceneConfig, Scene, make_frame, make_sequence, tiny_plane_config,
                    vga_config, hd_config, sized_config, rectified_F,
                    calib_of, batch_resolutions, halfway_flows_from_positions,
                    IMAGE_NAMES)
