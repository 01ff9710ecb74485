"""MI355X-native APIC augury contact step (arXiv 2108.02259)."""
