"""Seeded synthetic problem instances for the Lagrangian-decomposition bounding step.

This module only builds *inputs*: network weights, input boxes, objective vectors
and intermediate pre-activation bounds.  It contains none of the bounding
method's arithmetic; the intermediate bounds are produced by interval bound
propagation from the root input box (the cheap "@root" recipe of the paper's
branch-and-bound framework, Sec. 5.1.1), then each subdomain fixes a random 5 %
of the root-ambiguous ReLUs to one phase by editing one side of its bound
(ReLU branching, Sec. 2.3.2).  Everything is float32-representable so that any
two implementations solve the identical instance.
"""
from .instances import (Instance, LayerSpec, make_instance, CONFIGS, config_names, random_duals,
                        instance_to_torch)

__all__ = ["Instance", "LayerSpec", "make_instance", "CONFIGS", "config_names", "random_duals",
           "instance_to_torch"]
