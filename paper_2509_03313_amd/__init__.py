"""MI355X-native step-by-step (SBS) diffusion-reaction engine for water
radiolysis in periodic cubes (arXiv 2509.03313, multi-pulse gMicroMC).

  paper_2509_03313_amd.gsbs      ctypes binding of libgsbs.so (include/gsbs.h)
  paper_2509_03313_amd.workload  seeded synthetic inputs (spurs, tables, times)
  paper_2509_03313_amd.build     builds libgsbs.so for gfx950

The binding is imported on demand so that the input generator can be used
without a built library; importing `gsbs` without the library raises.
"""
__all__ = ["gsbs", "workload", "build"]
