"""MI355X-native hot path of the iterative HPS Helmholtz solver (arXiv 2112.02211).

Importing the package loads nothing; ``paper_2112_02211_amd.hps`` holds the
binding to the HIP library, ``paper_2112_02211_amd.problems`` the seeded
synthetic workloads.
"""
__all__ = ["hps", "problems"]
