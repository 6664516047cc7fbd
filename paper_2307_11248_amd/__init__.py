"""MI355X-native hot path of the pairwise-exchange QAP heuristics (arXiv 2307.11248)."""
