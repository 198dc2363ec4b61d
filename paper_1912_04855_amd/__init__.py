"""CSPH-TVD on MI355X: the HIP library binding and problem generators."""
