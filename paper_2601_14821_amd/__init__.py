"""MI355X-native removal-effect rasterizer for 3D Gaussian splatting (POTR, Sec. 4.2).

    from paper_2601_14821_amd import synth, raster
    ds = raster.to_device(scene)
    scores, _, _ = raster.Rasterizer(synth.RenderSettings()).score_views(ds, cams)

`synth` draws seeded inputs; `raster` drives libpotr.so (built by
`paper_2601_14821_amd.build`); `_lib` is the ctypes binding of include/potr.h.
Importing this package loads nothing; the HIP library is loaded on first use.
"""
__all__ = ["synth", "raster", "build"]
