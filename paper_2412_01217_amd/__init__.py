"""MI355X (gfx950) pyramid Gaussian-splatting rasterizer: HIP kernels behind a C ABI
(include/gs.h), with a thin torch binding. See raster.py for the binding and
scenes.py for the seeded synthetic inputs."""
__version__ = "0.1.0"
