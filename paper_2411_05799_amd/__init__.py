"""MI355X-native batched legged-robot step of NeoPhysIx (arXiv 2411.05799).

Importing the package loads nothing native; `paper_2411_05799_amd.native`
loads the HIP library on first use and fails loudly when it is missing.
"""
__all__ = ["workloads", "native"]
