"""MI355X-native hot path of DiffPower (arXiv 2608.03778): differentiable
switching-power propagation on levelized gate netlists."""
